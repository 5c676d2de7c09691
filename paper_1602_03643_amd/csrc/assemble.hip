// Colour-by-colour P1 assembly into an existing CSR pattern, and the
// stand-alone sparse product.
//
// Alg. 2 of the paper re-assembles the convection matrix into the storage
// of A every step.  Here the cells of one colour share no dof, so one
// launch per colour scatters into rows that no other thread touches: no
// atomics, deterministic results.  Each block stages the element matrices
// of its 256 cells in LDS (one thread per cell computes geometry and the
// (D+1)^2 entries), then all threads cooperate on the scatter so that the
// lanes writing one row sit next to each other.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "assemble.hpp"
#include "p1.hpp"
#include "spmv.hpp"

namespace oasis {

template <int D>
__global__ __launch_bounds__(kBlock) void k_assemble(int ncell, const int *__restrict__ clist,
                                                     const double *__restrict__ X,
                                                     const int *__restrict__ cells,
                                                     const int *__restrict__ v2d,
                                                     const int *__restrict__ rp,
                                                     const int *__restrict__ ci,
                                                     double *__restrict__ out, int form,
                                                     double alpha, P3 U1, P3 U2, double c1,
                                                     double c2, int *missing) {
    constexpr int NV = D + 1;
    constexpr int NE = NV * NV;
    __shared__ double lm[kBlock * NE];
    __shared__ int ld[kBlock * NV];
    const int c0 = blockIdx.x * kBlock;
    const int nloc = min(kBlock, ncell - c0);
    const int t = threadIdx.x;
    if (t < nloc) {
        const int cell = clist[c0 + t];
        double x[NV][D];
        int dof[NV];
#pragma unroll
        for (int a = 0; a < NV; ++a) {
            const int v = cells[(long long)cell * NV + a];
            dof[a] = v2d[v];
#pragma unroll
            for (int k = 0; k < D; ++k) x[a][k] = X[(long long)v * D + k];
        }
        Elem<D> e;
        p1_element<D>(x, e);
        double ub[NV][D];
        if (form == OASIS_FORM_CONV) {
#pragma unroll
            for (int a = 0; a < NV; ++a)
#pragma unroll
                for (int k = 0; k < D; ++k)
                    ub[a][k] = c1 * U1.p[k][dof[a]] + (c2 != 0.0 ? c2 * U2.p[k][dof[a]] : 0.0);
        } else {
#pragma unroll
            for (int a = 0; a < NV; ++a)
#pragma unroll
                for (int k = 0; k < D; ++k) ub[a][k] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            ld[t * NV + i] = dof[i];
#pragma unroll
            for (int j = 0; j < NV; ++j) lm[t * NE + i * NV + j] = alpha * p1_entry<D>(form, e, i, j, ub);
        }
    }
    __syncthreads();
    for (int q = t; q < nloc * NE; q += kBlock) {
        const int cl = q / NE, ij = q - cl * NE;
        const int i = ij / NV, j = ij - i * NV;
        const int row = ld[cl * NV + i], col = ld[cl * NV + j];
        const int s = rp[row], e = rp[row + 1];
        int pos = -1;
        for (int k = s; k < e; ++k)
            if (ci[k] == col) {
                pos = k;
                break;
            }
        if (pos >= 0)
            out[pos] += lm[q];
        else if (missing)
            atomicOr(missing, 1);
    }
}

int assemble_colored(hipStream_t s, const oasis_mesh *m, const int *rp, const int *ci, double *out,
                     int form, double alpha, P3 U1, P3 U2, double c1, double c2, int *missing) {
    for (int k = 0; k < m->n_colors; ++k) {
        const int a = m->color_ptr[k], b = m->color_ptr[k + 1];
        if (b <= a) continue;
        const int g = (b - a + kBlock - 1) / kBlock;
        if (m->dim == 3)
            hipLaunchKernelGGL(k_assemble<3>, dim3(g), dim3(kBlock), 0, s, b - a, m->color_cells + a,
                               m->coords, m->cells, m->vert2dof, rp, ci, out, form, alpha, U1, U2,
                               c1, c2, missing);
        else
            hipLaunchKernelGGL(k_assemble<2>, dim3(g), dim3(kBlock), 0, s, b - a, m->color_cells + a,
                               m->coords, m->cells, m->vert2dof, rp, ci, out, form, alpha, U1, U2,
                               c1, c2, missing);
        OASIS_TRY_LAUNCH();
    }
    return OASIS_OK;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpby_copy(long long n, T *__restrict__ y,
                                                       const T *__restrict__ x, T a) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = x ? a * x[i] : T(0);
}

int scale_copy(hipStream_t s, long long n, double *y, const double *x, double a) {
    const int g = (int)std::min<long long>((n + kBlock - 1) / kBlock, 16384);
    hipLaunchKernelGGL((k_axpby_copy<double>), dim3(g), dim3(kBlock), 0, s, n, y, x, a);
    OASIS_TRY_LAUNCH();
    return OASIS_OK;
}

template <typename T, class C>
__global__ __launch_bounds__(kBlock) void k_spmv(int n, const int *__restrict__ rp,
                                                 const int *__restrict__ ci,
                                                 const T *__restrict__ val,
                                                 const T *__restrict__ x, T *__restrict__ y, T alpha,
                                                 T beta) {
    csr_rows<T, 1, C>(
        n, rp, ci, val,
        [&](int, int c, T v, bool ok, T(&a)[1]) {
            const T t = v * x[c];
            a[0] += ok ? t : T(0);
        },
        [&](int row, int lane, T(&a)[1]) {
            if (lane == 0) y[row] = beta == T(0) ? alpha * a[0] : alpha * a[0] + beta * y[row];
        });
}

template <typename T>
static int spmv_launch(hipStream_t s, const oasis_csr *A, const T *x, T *y, T alpha, T beta) {
    const T *val = static_cast<const T *>(A->val);
    return with_cfg([&](auto c) -> int {
        using C = decltype(c);
        // one lane group per row group: the grid is not capped (no partials)
        const int g = grid_for(A->n, rows_per_block<C>(), 1 << 20);
        hipLaunchKernelGGL((k_spmv<T, C>), dim3(g), dim3(kBlock), 0, s, A->n, A->row_ptr, A->col_idx, val, x,
                           y, alpha, beta);
        OASIS_TRY_LAUNCH();
        return OASIS_OK;
    });
}

int check_csr(const oasis_csr *A) {
    if (!A || A->n <= 0 || A->nnz < 0 || !A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
        return OASIS_EINVAL;
    if (A->dtype != OASIS_F64 && A->dtype != OASIS_F32) return OASIS_EINVAL;
    if (!aligned(A->val, A->dtype == OASIS_F64 ? 8 : 4)) return OASIS_EINVAL;
    return OASIS_OK;
}

int check_mesh_colored(const oasis_mesh *m) {
    if (!m || (m->dim != 2 && m->dim != 3) || m->n_vert <= 0 || m->n_cell <= 0 || m->n_dof <= 0)
        return OASIS_EINVAL;
    if (!m->coords || !m->cells || !m->vert2dof || m->n_colors <= 0 || !m->color_ptr ||
        !m->color_cells)
        return OASIS_EINVAL;
    if (m->color_ptr[0] != 0 || m->color_ptr[m->n_colors] != m->n_cell) return OASIS_EINVAL;
    return OASIS_OK;
}

}  // namespace oasis

using namespace oasis;

extern "C" int oasis_spmv(void *stream, const oasis_csr *A, const void *x, void *y, double alpha,
                          double beta) {
    OASIS_TRY(check_csr(A));
    if (!x || !y) return OASIS_EINVAL;
    hipStream_t s = as_stream(stream);
    if (A->dtype == OASIS_F64)
        return spmv_launch<double>(s, A, static_cast<const double *>(x), static_cast<double *>(y),
                                   alpha, beta);
    return spmv_launch<float>(s, A, static_cast<const float *>(x), static_cast<float *>(y),
                              static_cast<float>(alpha), static_cast<float>(beta));
}

extern "C" int oasis_assemble_p1(void *stream, const oasis_mesh *mesh, int32_t form,
                                 const double *const *uab, double alpha, const oasis_csr *base,
                                 oasis_csr *out) {
    OASIS_TRY(check_mesh_colored(mesh));
    OASIS_TRY(check_csr(out));
    if (out->dtype != OASIS_F64 || out->n != mesh->n_dof) return OASIS_EINVAL;
    if (form < OASIS_FORM_MASS || form > OASIS_FORM_CONV) return OASIS_EINVAL;
    if (form == OASIS_FORM_GRAD_Z && mesh->dim != 3) return OASIS_EINVAL;
    P3 U1{}, U2{};
    if (form == OASIS_FORM_CONV) {
        if (!uab) return OASIS_EINVAL;
        for (int k = 0; k < mesh->dim; ++k) {
            if (!uab[k]) return OASIS_EINVAL;
            U1.p[k] = uab[k];
        }
    }
    if (base) {
        OASIS_TRY(check_csr(base));
        if (base->dtype != OASIS_F64 || base->nnz != out->nnz || base->n != out->n) return OASIS_EINVAL;
    }
    hipStream_t s = as_stream(stream);
    OASIS_TRY(scale_copy(s, out->nnz, static_cast<double *>(out->val),
                         base ? static_cast<const double *>(base->val) : nullptr, 1.0));
    // entries absent from the pattern are skipped (no flag without a workspace)
    OASIS_TRY(assemble_colored(s, mesh, out->row_ptr, out->col_idx, static_cast<double *>(out->val),
                               form, alpha, U1, U2, 1.0, 0.0, nullptr));
    return OASIS_OK;
}
