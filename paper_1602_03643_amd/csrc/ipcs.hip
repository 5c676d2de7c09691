// The IPCS_ABCN time step on the device, and the stand-alone Krylov entry
// points.
//
// Per step (Alg. 1 with one inner iteration, Alg. 2, Sec. 5):
//   1  A = B + C(u_bar)/2 with B = M/dt + nu K/2 preassembled and
//      u_bar = 1.5 U^{n-1} - 0.5 U^{n-2} formed inside the assembly.
//      This is the coefficient matrix Alg. 2 leaves in A; its intermediate
//      M/dt - C/2 - nu K/2 = 2M/dt - A is never stored: the explicit part of
//      the right-hand side is evaluated row by row as (2M/dt - A) U^{n-1}.
//   2  one pass per row: b^k = f_k M_L + (2M/dt - A) U^{k,n-1} - dP^k p*,
//      Dirichlet rows (identity row, b = g) and the diagonal D of A; then
//      the columns are divided by D (right Jacobi: A D^{-1} y = b, x = y/D).
//   3  BiCGStab for all velocity components at once (x0 = U^{k,n-1}, so
//      y0 = D U^{k,n-1}); x = y / D afterwards.
//   4  b_phi = -(1/dt) sum_k dP^k U^{k,I}, projected on 1-perp, symmetric
//      Jacobi scaling, CG from phi_prev (or the better of phi_prev and a
//      supplied guess).
//   5  phi and p^{n-1/2} = p* + phi shifted to zero mean.
//   6  U^{k,n} = U^{k,I} - dt (dP^k phi) / M_L, Dirichlet values restored.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "amg.hpp"
#include "assemble.hpp"
#include "krylov.hpp"
#include "mpnn.hpp"
#include "p1.hpp"
#include "spmv.hpp"

namespace oasis {

int incidence_codes(hipStream_t s, const oasis_mesh *m, int *iptr, int *inc, int *cnt, int *tmp, int *flag);
size_t incidence_tmp_ints(int n);

// ---------------------------------------------------------------------------
// matrix preparation kernels

// diag[i] = A_ii (0 when absent)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                 const T *__restrict__ val, double *__restrict__ d) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int j = rp[i]; j < rp[i + 1]; ++j)
            if (ci[j] == i) v = val[j];
        d[i] = v;
    }
}

// kScaleSym: out_ij = a_ij / (s_i s_j) (symmetric Jacobi scaling);
// kScaleCol: out_ij = a_ij / s_j (right Jacobi).  Optional FP32 copy.
constexpr int kScaleSym = 1, kScaleCol = 2;
__global__ __launch_bounds__(kBlock) void k_scale_matrix(int n, const int *__restrict__ rp,
                                                         const int *__restrict__ ci,
                                                         const double *__restrict__ a,
                                                         const double *__restrict__ s, int mode,
                                                         double *__restrict__ out,
                                                         float *__restrict__ out32) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double si = mode == kScaleSym ? s[i] : 1.0;
        for (int j = rp[i]; j < rp[i + 1]; ++j) {
            const double v = a[j] / (si * s[ci[j]]);
            out[j] = v;
            if (out32) out32[j] = static_cast<float>(v);
        }
    }
}

// In place: a_ij /= d_j (right Jacobi), one row per kEll lanes, with the
// optional FP32 CSR copy and the optional ELL values (e64 or e32; the
// rows then have at most kEll entries, padding written as 0).
__global__ __launch_bounds__(kBlock) void k_colscale(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                     const double *__restrict__ d, double *__restrict__ a,
                                                     float *__restrict__ a32, double *__restrict__ e64,
                                                     float *__restrict__ e32) {
    const int k = threadIdx.x & (kEll - 1);
    for (long long row = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / kEll; row < n;
         row += (static_cast<long long>(gridDim.x) * blockDim.x) / kEll) {
        const int s = rp[row], len = rp[row + 1] - s;
        double v = 0.0;
        for (int j = s + k; j < s + len; j += kEll) {
            const double t = a[j] / d[ci[j]];
            a[j] = t;
            if (a32) a32[j] = static_cast<float>(t);
            if (j == s + k) v = t;
        }
        if (e64) e64[row * kEll + k] = k < len ? v : 0.0;
        if (e32) e32[row * kEll + k] = k < len ? static_cast<float>(v) : 0.f;
    }
}

// x_k *= d (op 1) or x_k /= d (op 2) for up to 3 vectors, in place
__global__ __launch_bounds__(kBlock) void k_scale3(int n, const double *__restrict__ d, int op, double *x0,
                                                   double *x1, double *x2) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double di = d[i];
        double *xs[3] = {x0, x1, x2};
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (xs[k]) xs[k][i] = op == 1 ? xs[k][i] * di : xs[k][i] / di;
    }
}

// per-row vector set-up from a diagonal: mode 0 (CG): s = sqrt(d), w = d;
// mode 1 (BiCGStab, right Jacobi: its residual is the true one): s = d,
// w = 1.  flag set if a diagonal is unusable.
__global__ __launch_bounds__(kBlock) void k_diag_vectors(int n, const double *d, int mode, double *s,
                                                         double *w, float *w32, int *flag) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double v = d[i];
        if (mode == 0 ? !(v > 0.0) : !(v != 0.0) || !__builtin_isfinite(v)) atomicOr(flag, 1);
        s[i] = mode == 0 ? sqrt(v) : v;
        w[i] = mode == 0 ? v : 1.0;
        if (w32) w32[i] = static_cast<float>(w[i]);
    }
}

// y = x * a / s (op 0) or y = x * s (op 1) or y = x / s (op 2)
__global__ __launch_bounds__(kBlock) void k_vscale(int n, const double *__restrict__ x,
                                                   const double *__restrict__ s, int op,
                                                   double *__restrict__ y) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = op == 1 ? x[i] * s[i] : x[i] / s[i];
}

__global__ __launch_bounds__(kBlock) void k_row_sums(int n, const int *__restrict__ rp,
                                                     const double *__restrict__ a, double *__restrict__ out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int j = rp[i]; j < rp[i + 1]; ++j) v += a[j];
        out[i] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_lincomb(long long n, double *__restrict__ y, const double *__restrict__ a,
                                                    double ca, const double *__restrict__ b, double cb) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = ca * a[i] + cb * b[i];
}

__global__ __launch_bounds__(kBlock) void k_bc_index(int nbc, int n, const int *bc, int *idx, int *flag) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nbc;
         q += (long long)gridDim.x * blockDim.x) {
        const int d = bc[q];
        if (d >= 0 && d < n)
            idx[d] = (int)q;
        else
            atomicOr(flag, 1);
    }
}

__global__ __launch_bounds__(kBlock) void k_to_f32(long long n, const double *__restrict__ x, float *__restrict__ y) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = static_cast<float>(x[i]);
}

__global__ __launch_bounds__(kBlock) void k_add_f32(long long n, double *__restrict__ x, const float *__restrict__ e) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] += static_cast<double>(e[i]);
}

// x_q += e_q for the first nq of up to three (x, e) pairs, one launch
struct AddSet {
    double *x[3];
    const float *e[3];
};
__global__ __launch_bounds__(kBlock) void k_add3_f32(long long n, AddSet a, int nq) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        for (int q = 0; q < nq; ++q) a.x[q][i] += static_cast<double>(a.e[q][i]);
}

// partial sums of x^2
__global__ __launch_bounds__(kBlock) void k_sumsq(int n, const double *__restrict__ x, double *part) {
    __shared__ double lds[kBlock / kWave];
    double acc[1] = {0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        acc[0] += x[i] * x[i];
    write_partials<1>(acc, part, lds);
}

// partial sums of x . (r + b): the CG energy J(x) = 1/2 x^T K x - b^T x
// = -1/2 x^T (r + b) with r = b - K x
__global__ __launch_bounds__(kBlock) void k_energy_part(int n, const double *__restrict__ x,
                                                        const double *__restrict__ r, const double *__restrict__ b,
                                                        double *part) {
    __shared__ double lds[kBlock / kWave];
    double acc[1] = {0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        acc[0] += x[i] * (r[i] + b[i]);
    write_partials<1>(acc, part, lds);
}

// out32 = x / ||x||
__global__ __launch_bounds__(kBlock) void k_unit_f32(int n, const double *__restrict__ x, const double *part,
                                                     int np, float *__restrict__ out32) {
    __shared__ double lds[kBlock / kWave];
    double v[1];
    read_partials<1>(part, np, v, lds);
    const double inv = 1.0 / sqrt(v[0]);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out32[i] = static_cast<float>(x[i] * inv);
}

// out = x / ||x|| in FP32; *norm2 (host) = ||x||^2 (synchronises).
static int unit_vector_f32(hipStream_t s, int n, const double *x, double *part, float *out, double *norm2) {
    const int g = grid_for(n, kBlock);
    hipLaunchKernelGGL(k_sumsq, dim3(g), dim3(kBlock), 0, s, n, x, part);
    OASIS_TRY_LAUNCH();
    hipLaunchKernelGGL(k_unit_f32, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, x, part, g, out);
    OASIS_TRY_LAUNCH();
    std::vector<double> h(g);
    OASIS_TRY_HIP(hipMemcpyAsync(h.data(), part, g * sizeof(double), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (double v : h) t += v;
    *norm2 = t;
    return OASIS_OK;
}

// ---------------------------------------------------------------------------
// step kernels

// Right-hand side, Dirichlet rows and the diagonal of A, one row per
// lane group.  x0 of the velocity solve (U^{n-1}) is copied on the way.
// cv (nullable per component): an explicit convection vector subtracted
// from the right-hand side (eq:convection_ABE).  The pressure term is
// dP^k p, from the stored gradient matrices, or with GP the value that the
// row-gather assembly left in b_k for the row (the same sums over the
// row's cells, formed there from the cells it already walks).  With CS the
// diagonal is already in dA (written by the assembly), and the kernel also
// applies the right Jacobi scaling a_ij / d_j that k_colscale does
// otherwise, writing the scaled row and its FP32 CSR or ELL copies.  With
// r0o set (CS only) it also writes the refinement loop's first residual:
// r0 = b - A U^{n-1} (= b - Â y0) in FP32, from the same row and gathers,
// with the partials (sum r0^2, sum b^2) per component that k_ir_resid would
// produce (unit weights: right Jacobi).
struct P3F {
    float *p[3];
};

template <int D, int L, bool GP = false, bool CS = false>
__global__ __launch_bounds__(kBlock) void k_tent_rows(
    int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ M,
    double *__restrict__ A, P3 dP, P3 U1, P3 cv, const double *__restrict__ p,
    const double *__restrict__ ML, const int *__restrict__ bc_index, const double *__restrict__ g,
    int nbc, double f0, double f1, double f2, double two_over_dt, double *__restrict__ b0,
    double *__restrict__ b1, double *__restrict__ b2, double *__restrict__ x0, double *__restrict__ x1,
    double *__restrict__ x2, double *__restrict__ dA, double *__restrict__ wA,
    float *__restrict__ wA32, float *__restrict__ a32, double *__restrict__ e64, float *__restrict__ e32,
    P3F r0o, double *__restrict__ rpart) {
    static_assert(L >= D + 3, "one lane per output array");
    __shared__ double lds[2 * D * kBlock / kWave];
    double rr = 0.0, rb = 0.0;   // this lane's component's r0^2 and b^2 (lane < D)
    const int lane = threadIdx.x & (L - 1);
    const long long gid = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) / L;
    const long long ngroups = (static_cast<long long>(gridDim.x) * blockDim.x) / L;
    double *bo[3] = {b0, b1, b2};
    double *xo[3] = {x0, x1, x2};
    const double f[3] = {f0, f1, f2};
    for (long long row = gid; row < n; row += ngroups) {
        const int i = static_cast<int>(row);
        const int s = rp[i], e = rp[i + 1];
        const int q = bc_index[i];
        double acc[D], accp[D], acca[D], diag = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = accp[k] = acca[k] = 0.0;
        for (int j = s + lane; j < e; j += L) {
            const int c = ci[j];
            const double a = A[j];
            const double rhs_coef = two_over_dt * M[j] - a;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double u = U1.p[k][c];
                acc[k] += rhs_coef * u;
                if (CS) acca[k] += a * u;
            }
            if (!GP && p) {                           // no pressure gradient for a scalar
                const double pc = p[c];
#pragma unroll
                for (int k = 0; k < D; ++k) accp[k] += dP.p[k][j] * pc;
            }
            if (!CS && c == i) diag = a;
            if constexpr (CS) {
                // the Dirichlet row is the identity row; then a_ij / d_j
                const double t = (q >= 0 ? (c == i ? 1.0 : 0.0) : a) / dA[c];
                A[j] = t;
                if (a32) a32[j] = static_cast<float>(t);
                if (e64) e64[row * kEll + (j - s)] = t;
                if (e32) e32[row * kEll + (j - s)] = static_cast<float>(t);
            }
        }
        if constexpr (CS) {
            // the ELL copies' padding slots (rows of at most kEll entries)
            for (int k = e - s + lane; k < kEll; k += L) {
                if (e64) e64[row * kEll + k] = 0.0;
                if (e32) e32[row * kEll + k] = 0.f;
            }
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            acc[k] = group_sum<L>(acc[k]);
            if (!GP) accp[k] = group_sum<L>(accp[k]);
            if (CS) acca[k] = group_sum<L>(acca[k]);
        }
        double dd;
        if constexpr (CS) {
            dd = dA[i];
        } else {
            diag = group_sum<L>(diag);
            dd = q >= 0 ? 1.0 : diag;
            if (q >= 0)
                for (int j = s + lane; j < e; j += L) A[j] = (ci[j] == i) ? 1.0 : 0.0;
        }
        // the row's outputs spread over the group's lanes (every lane holds
        // the sums): lane k < D writes component k, the next three lanes the
        // diagonal and the two weights
        if (lane < D) {
            double ak = acc[0], apk = accp[0], aak = acca[0], fk = f[0];
            double *bk = bo[0], *xk = xo[0];
            const double *uk = U1.p[0], *ck = cv.p[0];
            float *rk = r0o.p[0];
#pragma unroll
            for (int k = 1; k < D; ++k)
                if (lane == k) {
                    ak = acc[k];
                    apk = accp[k];
                    aak = acca[k];
                    fk = f[k];
                    bk = bo[k];
                    xk = xo[k];
                    uk = U1.p[k];
                    ck = cv.p[k];
                    rk = r0o.p[k];
                }
            const double gp = GP ? bk[i] : apk;
            const double bv = q >= 0 ? g[lane * nbc + q] : fk * ML[i] + ak - gp - (ck ? ck[i] : 0.0);
            const double u = uk[i];
            bk[i] = bv;
            xk[i] = dd * u;      // y0 = D x0 for the column-scaled system
            if (CS && rk) {
                // a Dirichlet row of Â is the unit row and y0_i = U^{n-1}_i there
                const double r = bv - (q >= 0 ? u : aak);
                rk[i] = static_cast<float>(r);
                rr += r * r;
                rb += bv * bv;
            }
        } else if (lane == D) {
            if (!CS) dA[i] = dd;
        } else if (lane == D + 1) {
            wA[i] = 1.0;
        } else if (lane == D + 2 && wA32) {
            wA32[i] = 1.f;
        }
    }
    if (CS && rpart) {
        double v[2 * D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            v[2 * k] = lane == k ? rr : 0.0;
            v[2 * k + 1] = lane == k ? rb : 0.0;
        }
        write_partials<2 * D>(v, rpart, lds);
    }
}

// u_bar = 1.5 U^{n-1} - 0.5 U^{n-2} (Alg. 2), interleaved per dof
// ([n][4] in 3D, [n][2] in 2D) for the assembly's per-vertex gathers.  In
// 3D the fourth slot of a record carries p (zero without one), so that the
// row-gather assembly reads the pressure in the same load.
template <int D>
__global__ __launch_bounds__(kBlock) void k_ubar(int n, P3 U1, P3 U2, const double *__restrict__ p,
                                                 double *__restrict__ ubar) {
    constexpr int UW = D == 3 ? 4 : 2;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < D; ++c) ubar[i * UW + c] = 1.5 * U1.p[c][i] - 0.5 * U2.p[c][i];
        if (D == 3) ubar[i * UW + 3] = p ? p[i] : 0.0;
    }
}

// U^{n-1} and U^{n-2} interleaved per dof for k_conv_rows' gathers
template <int D>
__global__ __launch_bounds__(kBlock) void k_uu(int n, P3 U1, P3 U2, double *__restrict__ uu) {
    constexpr int UW = D == 3 ? 4 : 2;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            uu[i * 2 * UW + c] = U1.p[c][i];
            uu[i * 2 * UW + UW + c] = U2.p[c][i];
        }
        if (D == 3) uu[i * 2 * UW + 3] = uu[i * 2 * UW + 7] = 0.0;
    }
}

// Row-gather form of step 1: every row assembles its own entries of
// A = B + C(u_bar)/2 from the cells around its dof (the convection part of
// Alg. 2's coefficient matrix); k_tent_rows then forms the right-hand side,
// the Dirichlet row and the diagonal.  One thread owns one row; the row's
// columns and values live in MAXC registers and an element contribution
// (column dof c, value v) is added to the slot whose column equals c (a
// compile-time unrolled match).  The incident cells are visited in
// ascending order, so the sums are deterministic; no other thread writes
// the row, so no atomics and no colouring are needed.  The kernel is bound
// by how many dependent gathers are in flight (incidence -> vertices ->
// dofs -> coordinates and u_bar): NC cells are loaded before any is added
// (an odd tail's clamped copy is added with weight 0, so the compiler
// cannot sink its loads behind the first cell's arithmetic), and the rows
// are split XCD-aware so that neighbouring rows' cells share one L2.
// With GP (3D) the walk also forms the tentative step's pressure term
// (dP^k p)_i = sum over the row's cells of vol/(D+1) * sum_j p_j d_k phi_j
// (eq:dp_matrix applied to p, the 4th slot of the u_bar records) into gp_k,
// instead of k_tent_rows streaming the three gradient matrices.
template <int D, int MAXC, bool GP = false, int NC = (MAXC <= 16 ? 3 : 2)>
__global__ __launch_bounds__(kBlock) void k_asm_rows(
    int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ B,
    const int *__restrict__ iptr, const int *__restrict__ inc, const int *__restrict__ cells,
    const int *__restrict__ v2d, const double *__restrict__ X, const double *__restrict__ ubar,
    double *__restrict__ A, double *__restrict__ gp0, double *__restrict__ gp1, double *__restrict__ gp2,
    const int *__restrict__ bc_index, double *__restrict__ dA) {
    static_assert(!GP || D == 3, "the pressure rides in the 3D records' spare slot");
    constexpr int NV = D + 1;
    constexpr int UW = D == 3 ? 4 : 2;                  // u_bar row width
    constexpr double mfac = 0.5 / ((D + 1) * (D + 2));   // C/2 and the mass-moment factor
    const RowRange<1> rr(n);
    for (long long row = rr.first + rr.gid; row < rr.last; row += rr.ngroups) {
        const int i = static_cast<int>(row);
        const int s = rp[i], len = rp[i + 1] - s;
        int col[MAXC];
        double a[MAXC];
#pragma unroll
        for (int q = 0; q < MAXC; ++q) {
            col[q] = q < len ? ci[s + q] : -1;
            a[q] = q < len ? B[s + q] : 0.0;
        }
        struct Cell {
            double x[NV][D], ub[NV][D], pp[GP ? NV : 1];
            int dd[NV], la;
        };
        double gp[D];
#pragma unroll
        for (int c = 0; c < D; ++c) gp[c] = 0.0;
        auto load = [&](int t, Cell &C) {
            const int code = inc[t];
            const int cell = code / NV;
            C.la = code - cell * NV;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int v = cells[(long long)cell * NV + k];
                C.dd[k] = v2d[v];
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    C.x[k][c] = X[(long long)v * D + c];
                    C.ub[k][c] = ubar[(long long)C.dd[k] * UW + c];
                }
                if constexpr (GP) C.pp[k] = ubar[(long long)C.dd[k] * UW + 3];
            }
        };
        auto add = [&](const Cell &C, double keep) {
            Elem<D> e;
            p1_element<D>(C.x, e);
            double w[D];   // S + u_bar at the row's local vertex
#pragma unroll
            for (int c = 0; c < D; ++c) {
                double S = 0.0;
#pragma unroll
                for (int k = 0; k < NV; ++k) S += C.ub[k][c];
                double ua = C.ub[0][c];
#pragma unroll
                for (int k = 1; k < NV; ++k) ua = (C.la == k) ? C.ub[k][c] : ua;
                w[c] = S + ua;
            }
            const double fac = keep * e.vol * mfac;
            if constexpr (GP) {
                const double fg = keep * e.vol * (1.0 / NV);
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    double t = 0.0;
#pragma unroll
                    for (int jl = 0; jl < NV; ++jl) t += e.g[jl][c] * C.pp[jl];
                    gp[c] += fg * t;
                }
            }
#pragma unroll
            for (int jl = 0; jl < NV; ++jl) {
                double gw = 0.0;
#pragma unroll
                for (int c = 0; c < D; ++c) gw += e.g[jl][c] * w[c];
                const double v = fac * gw;
                const int target = C.dd[jl];
                // a[q] + v where the column matches, as an FMA with a 0/1
                // factor (one select per slot instead of a 64-bit select of
                // v and an add; the same sums)
#pragma unroll
                for (int q = 0; q < MAXC; ++q) a[q] = __fma_rn((col[q] == target) ? 1.0 : 0.0, v, a[q]);
            }
        };
        // NC cells' loads in flight, then their contributions in ascending
        // order (as one at a time)
        const int t0 = iptr[i], t1 = iptr[i + 1];
        for (int t = t0; t < t1; t += NC) {
            Cell cc[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) load(t + k < t1 ? t + k : t, cc[k]);
#pragma unroll
            for (int k = 0; k < NC; ++k) add(cc[k], t + k < t1 ? 1.0 : 0.0);
        }
#pragma unroll
        for (int q = 0; q < MAXC; ++q)
            if (q < len) A[s + q] = a[q];
        if (dA) {
            // the diagonal the column scaling divides by (1 on a Dirichlet row)
            double dg = 0.0;
#pragma unroll
            for (int q = 0; q < MAXC; ++q) dg = col[q] == i ? a[q] : dg;
            dA[i] = bc_index[i] >= 0 ? 1.0 : dg;
        }
        if constexpr (GP) {
            gp0[i] = gp[0];
            gp1[i] = gp[1];
            gp2[i] = gp[2];
        }
    }
}

// Explicit Adams-Bashforth convection (eq:convection_ABE) as vectors:
// cv_k = 1.5 C(u^{n-1}) U_k^{n-1} - 0.5 C(u^{n-2}) U_k^{n-2}, with C(w)
// the convection matrix of the P1 field w.  On a cell the gradient of a
// P1 field is constant and int_T phi_i w = vol/((D+1)(D+2)) (S + w_i),
// S = sum of w over the cell's vertices, so the cell adds
// vol/((D+1)(D+2)) (S + w_i) . grad U_k.  Row i gathers its incident cells
// in ascending order (deterministic, no atomics), with two cells' loads in
// flight and XCD-aware rows, as k_asm_rows.  uu: U^{n-1} and U^{n-2}
// interleaved per dof (k_uu), one 64-byte record in 3D.
template <int D>
__global__ __launch_bounds__(kBlock) void k_conv_rows(int n, const int *__restrict__ iptr,
                                                      const int *__restrict__ inc, const int *__restrict__ cells,
                                                      const int *__restrict__ v2d, const double *__restrict__ X,
                                                      const double *__restrict__ uu, double *__restrict__ cv0,
                                                      double *__restrict__ cv1, double *__restrict__ cv2) {
    constexpr int UW = D == 3 ? 4 : 2;
    constexpr int NV = D + 1;
    constexpr double mfac = 1.0 / ((D + 1) * (D + 2));
    double *co[3] = {cv0, cv1, cv2};
    struct Cell {
        double x[NV][D], u1[NV][D], u2[NV][D];
        int la;
    };
    const RowRange<1, kBlock> rr(n);
    for (long long row = rr.first + rr.gid; row < rr.last; row += rr.ngroups) {
        const int i = static_cast<int>(row);
        double acc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = 0.0;
        auto load = [&](int t, Cell &C) {
            const int code = inc[t];
            const int cell = code / NV;
            C.la = code - cell * NV;
#pragma unroll
            for (int m = 0; m < NV; ++m) {
                const int v = cells[(long long)cell * NV + m];
                const long long dd = v2d[v];
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    C.x[m][c] = X[(long long)v * D + c];
                    C.u1[m][c] = uu[dd * 2 * UW + c];
                    C.u2[m][c] = uu[dd * 2 * UW + UW + c];
                }
            }
        };
        // coef * vol/((D+1)(D+2)) (S + w_la) . grad(w_k) for every component k
        auto field = [&](const Elem<D> &e, const double (&w)[NV][D], int la, double coef) {
            double a[D];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                double S = 0.0;
#pragma unroll
                for (int m = 0; m < NV; ++m) S += w[m][c];
                double wl = w[0][c];
#pragma unroll
                for (int m = 1; m < NV; ++m) wl = (la == m) ? w[m][c] : wl;
                a[c] = S + wl;
            }
            const double fac = coef * e.vol * mfac;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    double gr = 0.0;
#pragma unroll
                    for (int m = 0; m < NV; ++m) gr += e.g[m][c] * w[m][k];
                    s += a[c] * gr;
                }
                acc[k] += fac * s;
            }
        };
        auto add = [&](const Cell &C, double keep) {
            Elem<D> e;
            p1_element<D>(C.x, e);
            field(e, C.u1, C.la, 1.5 * keep);
            field(e, C.u2, C.la, -0.5 * keep);
        };
        const int t0 = iptr[i], t1 = iptr[i + 1];
        for (int t = t0; t < t1; t += 2) {
            const bool two = t + 1 < t1;
            Cell c0, c1;
            load(t, c0);
            load(two ? t + 1 : t, c1);
            add(c0, 1.0);
            add(c1, two ? 1.0 : 0.0);   // weight 0 on an odd tail's clamped copy
        }
#pragma unroll
        for (int k = 0; k < D; ++k) co[k][i] = acc[k];
    }
}

// G^k = M_L^{-1} dP^k: the rows of dP^k over the lumped mass (the weighted
// gradient matrix of the direct velocity update)
__global__ __launch_bounds__(kBlock) void k_row_div(int n, const int *__restrict__ rp, const double *__restrict__ a,
                                                    const double *__restrict__ d, double *__restrict__ out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double r = d[i];
        for (int j = rp[i]; j < rp[i + 1]; ++j) out[j] = a[j] / r;
    }
}

// b_phi = -(1/dt) sum_k dP^k U^{k,I}; partial sum of b_phi
template <int D, int L>
__global__ __launch_bounds__(kBlock) void k_div_rows(int n, const int *__restrict__ rp,
                                                     const int *__restrict__ ci, P3 dP, P3 UI,
                                                     double minv_dt, double *__restrict__ bphi,
                                                     double *part) {
    __shared__ double lds[kBlock / kWave];
    double tot[1] = {0.0};
    const int lane = threadIdx.x & (L - 1);
    const long long gid = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) / L;
    const long long ngroups = (static_cast<long long>(gridDim.x) * blockDim.x) / L;
    for (long long row = gid; row < n; row += ngroups) {
        const int s = rp[row], e = rp[row + 1];
        double acc = 0.0;
        // two entries per lane and pass, the second from a clamped index,
        // so that both entries' loads are in flight together
        for (int j0 = s + lane; j0 < e; j0 += 2 * L) {
            const bool ok1 = j0 + L < e;
            const int j1 = ok1 ? j0 + L : j0;
            const int c0 = ci[j0], c1 = ci[j1];
            double t0 = 0.0, t1 = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                t0 += dP.p[k][j0] * UI.p[k][c0];
                t1 += dP.p[k][j1] * UI.p[k][c1];
            }
            acc += t0 + (ok1 ? t1 : 0.0);
        }
        acc = group_sum<L>(acc);
        if (lane == 0) {
            const double v = minv_dt * acc;
            bphi[row] = v;
            tot[0] += v;
        }
    }
    write_partials<1>(tot, part, lds);
}

// projection on 1-perp and scaling: b_s = (b_phi - mean)/s, x_s = s * phi_prev
__global__ __launch_bounds__(kBlock) void k_bphi_finish(int n, const double *part, int np,
                                                        double *__restrict__ bphi,
                                                        const double *__restrict__ s,
                                                        const double *__restrict__ phi_prev, int zero_start,
                                                        double *__restrict__ bs, double *__restrict__ xs) {
    __shared__ double lds[kBlock / kWave];
    double v[1];
    read_partials<1>(part, np, v, lds);
    const double mean = v[0] / n;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double b = bphi[i] - mean;
        bphi[i] = b;
        bs[i] = b / s[i];
        xs[i] = zero_start ? 0.0 : phi_prev[i] * s[i];
    }
}

// phi = x_s / s; partial sum
__global__ __launch_bounds__(kBlock) void k_phi_a(int n, const double *__restrict__ xs,
                                                  const double *__restrict__ s, double *__restrict__ phi,
                                                  double *part) {
    __shared__ double lds[kBlock / kWave];
    double tot[1] = {0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double v = xs[i] / s[i];
        phi[i] = v;
        tot[0] += v;
    }
    write_partials<1>(tot, part, lds);
}

// phi -= mean(phi); p += phi; partial sum of p
__global__ __launch_bounds__(kBlock) void k_phi_b(int n, const double *partIn, int np,
                                                  double *__restrict__ phi, double *__restrict__ p,
                                                  double *partOut) {
    __shared__ double lds[kBlock / kWave];
    double v[1];
    read_partials<1>(partIn, np, v, lds);
    const double mean = v[0] / n;
    double tot[1] = {0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double f = phi[i] - mean;
        phi[i] = f;
        const double q = p[i] + f;
        p[i] = q;
        tot[0] += q;
    }
    write_partials<1>(tot, partOut, lds);
}

// p -= mean(p)
__global__ __launch_bounds__(kBlock) void k_phi_c(int n, const double *partIn, int np, double *__restrict__ p) {
    __shared__ double lds[kBlock / kWave];
    double v[1];
    read_partials<1>(partIn, np, v, lds);
    const double mean = v[0] / n;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] -= mean;
}

// U^{k,n} = U^{k,I} - dt (dP^k phi) / M_L; Dirichlet values
template <int D, int L>
__global__ __launch_bounds__(kBlock) void k_update_rows(int n, const int *__restrict__ rp,
                                                        const int *__restrict__ ci, P3 dP, P3 UI,
                                                        const double *__restrict__ phi,
                                                        const double *__restrict__ ML,
                                                        const int *__restrict__ bc_index,
                                                        const double *__restrict__ g, int nbc,
                                                        double dt, double *__restrict__ u0,
                                                        double *__restrict__ u1, double *__restrict__ u2) {
    double *uo[3] = {u0, u1, u2};
    const int lane = threadIdx.x & (L - 1);
    const long long gid = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) / L;
    const long long ngroups = (static_cast<long long>(gridDim.x) * blockDim.x) / L;
    for (long long row = gid; row < n; row += ngroups) {
        const int s = rp[row], e = rp[row + 1];
        double acc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = 0.0;
        // two entries per lane and pass (see k_div_rows)
        for (int j0 = s + lane; j0 < e; j0 += 2 * L) {
            const bool ok1 = j0 + L < e;
            const int j1 = ok1 ? j0 + L : j0;
            const double f0 = phi[ci[j0]], f1 = phi[ci[j1]];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double a0 = dP.p[k][j0] * f0, a1 = dP.p[k][j1] * f1;
                acc[k] += a0 + (ok1 ? a1 : 0.0);
            }
        }
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = group_sum<L>(acc[k]);
        // lane k < D writes component k (every lane holds the sums)
        if (lane < D) {
            double ak = acc[0];
            double *uk = uo[0];
            const double *vk = UI.p[0];
#pragma unroll
            for (int k = 1; k < D; ++k)
                if (lane == k) {
                    ak = acc[k];
                    uk = uo[k];
                    vk = UI.p[k];
                }
            const int q = bc_index[row];
            const double inv = ML ? dt / ML[row] : dt;   // no M_L: the gradient matrix
            uk[row] = q >= 0 ? g[lane * nbc + q] : vk[row] - inv * ak;
        }
    }
}

// Inner iterations (Alg. 1): the tentative right-hand sides b^k -= dP^k phi
// on the non-Dirichlet rows (p* grew by phi; the explicit part stays).
template <int D, int L>
__global__ __launch_bounds__(kBlock) void k_rhs_dp(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                   P3 dP, const double *__restrict__ phi,
                                                   const int *__restrict__ bc_index, double *__restrict__ b0,
                                                   double *__restrict__ b1, double *__restrict__ b2) {
    double *bo[3] = {b0, b1, b2};
    const int lane = threadIdx.x & (L - 1);
    const long long gid = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) / L;
    const long long ngroups = (static_cast<long long>(gridDim.x) * blockDim.x) / L;
    for (long long row = gid; row < n; row += ngroups) {
        double acc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = 0.0;
        for (int j = rp[row] + lane; j < rp[row + 1]; j += L) {
            const double f = phi[ci[j]];
#pragma unroll
            for (int k = 0; k < D; ++k) acc[k] += dP.p[k][j] * f;
        }
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = group_sum<L>(acc[k]);
        if (lane == 0 && bc_index[row] < 0) {
#pragma unroll
            for (int k = 0; k < D; ++k) bo[k][row] -= acc[k];
        }
    }
}

// Consistent update (eq:velocity_update): M with the rows and columns of
// the Dirichlet dofs removed and a unit diagonal there (symmetric
// elimination keeps the matrix SPD for CG).
__global__ __launch_bounds__(kBlock) void k_mass_bc(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                    const double *__restrict__ M, const int *__restrict__ bc_index,
                                                    double *__restrict__ out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const bool bi = bc_index[i] >= 0;
        for (int j = rp[i]; j < rp[i + 1]; ++j) {
            const int c = ci[j];
            out[j] = (bi || bc_index[c] >= 0) ? (bi && c == i ? 1.0 : 0.0) : M[j];
        }
    }
}

// Its right-hand sides M U^I - dt dP^k phi - M_{I,B} g (g on the Dirichlet
// rows), scaled for the symmetrically scaled system: b_s = rhs / s, and the
// scaled start x_s = s U^I (s g on the Dirichlet rows).
template <int D, int L>
__global__ __launch_bounds__(kBlock) void k_mass_rhs(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                     const double *__restrict__ M, P3 dP, P3 UI,
                                                     const double *__restrict__ phi,
                                                     const int *__restrict__ bc_index, const double *__restrict__ g,
                                                     int nbc, double dt, const double *__restrict__ sM,
                                                     double *__restrict__ b0, double *__restrict__ b1,
                                                     double *__restrict__ b2, double *__restrict__ x0,
                                                     double *__restrict__ x1, double *__restrict__ x2) {
    double *bo[3] = {b0, b1, b2};
    double *xo[3] = {x0, x1, x2};
    const int lane = threadIdx.x & (L - 1);
    const long long gid = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) / L;
    const long long ngroups = (static_cast<long long>(gridDim.x) * blockDim.x) / L;
    for (long long row = gid; row < n; row += ngroups) {
        double acc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = 0.0;
        for (int j = rp[row] + lane; j < rp[row + 1]; j += L) {
            const int c = ci[j];
            const double m = M[j], f = phi[c];
            const int qc = bc_index[c];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                acc[k] += m * UI.p[k][c] - dt * dP.p[k][j] * f;
                if (qc >= 0) acc[k] -= m * g[k * nbc + qc];
            }
        }
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = group_sum<L>(acc[k]);
        if (lane == 0) {
            const int q = bc_index[row];
            const double si = sM[row];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double gk = q >= 0 ? g[k * nbc + q] : 0.0;
                bo[k][row] = (q >= 0 ? gk : acc[k]) / si;
                xo[k][row] = si * (q >= 0 ? gk : UI.p[k][row]);
            }
        }
    }
}

// outer residual of the refinement loop: r = b - A x (FP64), r32 = (float) r,
// partials (sum w r^2, sum w b^2) per component
template <int NR, class C>
__global__ __launch_bounds__(kBlock) void k_ir_resid(int n, const int *__restrict__ rp,
                                                     const int *__restrict__ ci,
                                                     const double *__restrict__ val, EllCols cols,
                                                     const double *__restrict__ w, P3 b, P3 x,
                                                     float *r0, float *r1, float *r2, double *part) {
    __shared__ double lds[6 * kBlock / kWave];
    float *ro[3] = {r0, r1, r2};
    double acc2[2 * NR];
#pragma unroll
    for (int k = 0; k < 2 * NR; ++k) acc2[k] = 0.0;
    auto gather = [&](int, int c, double v, bool ok, double(&a)[NR]) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const double t = v * x.p[k][c];
            a[k] += ok ? t : 0.0;
        }
    };
    auto finish = [&](int row, int lane, double(&a)[NR]) {
        if (lane != 0) return;
        const double wd = w[row];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const double bk = b.p[k][row];
            const double r = bk - a[k];
            ro[k][row] = static_cast<float>(r);
            acc2[2 * k] += wd * r * r;
            acc2[2 * k + 1] += wd * bk * bk;
        }
    };
    // the CSR values with an ELL copy's columns when there is one
    if (cols.any())
        csr_cols_rows<double, NR, 2>(n, rp, val, cols, gather, finish);
    else
        csr_rows<double, NR, C>(n, rp, ci, val, gather, finish);
    write_partials<2 * NR>(acc2, part, lds);
}

template <int NV>
__global__ __launch_bounds__(kBlock) void k_sum_to(const double *part, int np, double *out) {
    __shared__ double lds[NV * kBlock / kWave];
    double v[NV];
    read_partials<NV>(part, np, v, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) out[k] = v[k];
}


__global__ __launch_bounds__(kBlock) void k_fill_i32(int n, int *x, int v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_copy_d(long long n, double *__restrict__ y, const double *__restrict__ x) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = x[i];
}

__global__ __launch_bounds__(kBlock) void k_zero_f(long long n, float *x) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = 0.f;
}

// ---------------------------------------------------------------------------
// refinement drivers (FP32 inner Krylov, FP64 outer residual)

struct IRBufs {
    float *r32[3] = {nullptr, nullptr, nullptr};
    float *e32[3] = {nullptr, nullptr, nullptr};
    double *part = nullptr;
    double *sums = nullptr;   // device [8]
    HostStage stage;          // the owner's read-back block (may be null)
};

static void carve_ir(Carver &c, int n, int nr, IRBufs &ir) {
    for (int k = 0; k < nr; ++k) {
        ir.r32[k] = c.take<float>(n);
        ir.e32[k] = c.take<float>(n);
    }
    ir.part = c.take<double>(6 * kMaxPartials);
    ir.sums = c.take<double>(8);
}

// FP64 residuals of nr systems; the ELL copy's columns (when the tuning
// allows the ELL storage) replace the int32 CSR columns.
static int ir_outer_resid(hipStream_t s, int n, int nr, const int *rp, const int *ci,
                          const double *val, const EllCols &ecols, const Tuning &tun, const double *w, P3 b, P3 x,
                          IRBufs &ir, double *host_sums) {
    using L = Cfg8x2x1;
    const EllCols cols = tun.ell() ? ecols : EllCols{};
    const int g = grid_for(n, rows_per_block<L>(), tun.grid_cap);
    if (nr == 1) {
        hipLaunchKernelGGL((k_ir_resid<1, L>), dim3(g), dim3(kBlock), 0, s, n, rp, ci, val, cols, w, b, x,
                           ir.r32[0], ir.r32[1], ir.r32[2], ir.part);
        OASIS_TRY_LAUNCH();
        hipLaunchKernelGGL((k_sum_to<2>), dim3(1), dim3(kBlock), 0, s, ir.part, g, ir.sums);
    } else if (nr == 2) {
        hipLaunchKernelGGL((k_ir_resid<2, L>), dim3(g), dim3(kBlock), 0, s, n, rp, ci, val, cols, w, b, x,
                           ir.r32[0], ir.r32[1], ir.r32[2], ir.part);
        OASIS_TRY_LAUNCH();
        hipLaunchKernelGGL((k_sum_to<4>), dim3(1), dim3(kBlock), 0, s, ir.part, g, ir.sums);
    } else {
        hipLaunchKernelGGL((k_ir_resid<3, L>), dim3(g), dim3(kBlock), 0, s, n, rp, ci, val, cols, w, b, x,
                           ir.r32[0], ir.r32[1], ir.r32[2], ir.part);
        OASIS_TRY_LAUNCH();
        hipLaunchKernelGGL((k_sum_to<6>), dim3(1), dim3(kBlock), 0, s, ir.part, g, ir.sums);
    }
    OASIS_TRY_LAUNCH();
    return read_state(s, ir.stage, ir.sums, host_sums, 2 * nr * sizeof(double));
}

// the sums of partials a producer left in ir.part (2 nr values per block)
static int ir_sum_resid(hipStream_t s, int nr, int nparts, IRBufs &ir, double *host_sums) {
    if (nr == 1)
        hipLaunchKernelGGL((k_sum_to<2>), dim3(1), dim3(kBlock), 0, s, ir.part, nparts, ir.sums);
    else if (nr == 2)
        hipLaunchKernelGGL((k_sum_to<4>), dim3(1), dim3(kBlock), 0, s, ir.part, nparts, ir.sums);
    else
        hipLaunchKernelGGL((k_sum_to<6>), dim3(1), dim3(kBlock), 0, s, ir.part, nparts, ir.sums);
    OASIS_TRY_LAUNCH();
    return read_state(s, ir.stage, ir.sums, host_sums, 2 * nr * sizeof(double));
}

struct KOpts {
    double rtol;
    int maxit;
    double inner_rtol;
    int max_outer;
    int check_every;
    bool time;
};

// CG with FP32 inner solves on the scaled system; x (FP64) refined until the
// FP64 weighted residual meets rtol.
static int ir_cg(hipStream_t s, int n, const int *rp, const int *ci, const double *val,
                 const float *val32, const double *w, const float *w32, const double *b, double *x,
                 const KOpts &o, CGWork<float> &cw, IRBufs &ir, SolveOut &out) {
    out = SolveOut();
    const int gv = grid_for(n, kBlock, 8192);
    P3 pb{}, px{};
    pb.p[0] = b;
    px.p[0] = x;
    double hs[2];
    int total = 0;
    for (int outer = 0;; ++outer) {
        OASIS_TRY(ir_outer_resid(s, n, 1, rp, ci, val, cw.cols, cw.tun, w, pb, px, ir, hs));
        out.rel_res = hs[1] > 0 ? std::sqrt(hs[0] / hs[1]) : std::sqrt(hs[0]);
        if (!std::isfinite(hs[0])) {
            out.status = OASIS_ENAN;
            break;
        }
        if (hs[0] <= o.rtol * o.rtol * hs[1]) {
            out.status = OASIS_OK;
            break;
        }
        if (outer >= o.max_outer || total >= o.maxit) {
            out.status = OASIS_ENOTCONV;
            break;
        }
        hipLaunchKernelGGL(k_zero_f, dim3(gv), dim3(kBlock), 0, s, (long long)n, ir.e32[0]);
        OASIS_TRY_LAUNCH();
        SolveOut in;
        const int rc = cg_solve<float>(s, n, rp, ci, val32, w32, ir.r32[0], ir.e32[0], o.inner_rtol,
                                       o.maxit - total, o.check_every, o.time, cw, in);
        if (rc == OASIS_EHIP) return rc;
        total += in.iters;
        out.kernel_ms += in.kernel_ms;
        out.kernel_count += in.kernel_count;
        out.outer += 1;
        hipLaunchKernelGGL(k_add_f32, dim3(gv), dim3(kBlock), 0, s, (long long)n, x, ir.e32[0]);
        OASIS_TRY_LAUNCH();
        if (rc == OASIS_ENAN) {
            out.status = OASIS_ENAN;
            break;
        }
    }
    out.iters = total;
    return out.status;
}

// BiCGStab for nr right-hand sides with FP32 inner solves (column-scaled system).
// r0_parts > 0: ir.r32 and ir.part already hold the first outer residual
// (FP32 copy and r0_parts blocks of partials, as k_ir_resid leaves them)
static int ir_bicgstab(hipStream_t s, int n, int nr, const int *rp, const int *ci,
                       const double *val, const float *val32, const double *w, const float *w32,
                       double *const *b, double *const *x, const KOpts &o, BiWork<float> &bw,
                       IRBufs &ir, SolveOut *out, int r0_parts = 0) {
    const int gv = grid_for(n, kBlock, 8192);
    P3 pb{}, px{};
    for (int k = 0; k < nr; ++k) {
        pb.p[k] = b[k];
        px.p[k] = x[k];
        out[k] = SolveOut();
        out[k].status = OASIS_ENOTCONV;
    }
    bool done[3] = {false, false, false};
    double hs[6];
    for (int outer = 0;; ++outer) {
        if (outer == 0 && r0_parts > 0)
            OASIS_TRY(ir_sum_resid(s, nr, r0_parts, ir, hs));
        else
            OASIS_TRY(ir_outer_resid(s, n, nr, rp, ci, val, bw.cols, bw.tun, w, pb, px, ir, hs));
        int active[3], na = 0;
        for (int k = 0; k < nr; ++k) {
            if (done[k]) continue;
            out[k].rel_res = hs[2 * k + 1] > 0 ? std::sqrt(hs[2 * k] / hs[2 * k + 1]) : std::sqrt(hs[2 * k]);
            if (!std::isfinite(hs[2 * k])) {
                out[k].status = OASIS_ENAN;
                done[k] = true;
            } else if (hs[2 * k] <= o.rtol * o.rtol * hs[2 * k + 1]) {
                out[k].status = OASIS_OK;
                done[k] = true;
            } else if (outer >= o.max_outer || out[k].iters >= o.maxit) {
                out[k].status = OASIS_ENOTCONV;
                done[k] = true;
            } else {
                active[na++] = k;
            }
        }
        if (na == 0) break;
        // inner tolerance: the configured one, loosened when less suffices to reach rtol
        double inner = o.inner_rtol;
        double need = 1.0;
        for (int q = 0; q < na; ++q) {
            const int k = active[q];
            if (hs[2 * k] > 0) need = std::min(need, 0.5 * o.rtol * std::sqrt(hs[2 * k + 1] / hs[2 * k]));
        }
        inner = std::max(inner, need);
        const float *bb[3];
        float *xx[3];
        for (int q = 0; q < na; ++q) {
            const int k = active[q];
            bb[q] = ir.r32[k];
            xx[q] = ir.e32[k];
        }
        // the correction starts from zero, which the solve writes itself,
        // and the FP64 residual above decides whether it is enough
        SolveOut in[3];
        const int rc = bicgstab_solve<float>(s, n, na, rp, ci, val32, w32, bb, xx, inner,
                                             o.maxit, o.check_every, o.time, bw, in, true);
        if (rc == OASIS_EHIP) return rc;
        AddSet as{};
        for (int q = 0; q < na; ++q) {
            const int k = active[q];
            out[k].iters += in[q].iters;
            out[k].outer += 1;
            out[k].kernel_ms += in[q].kernel_ms;
            out[k].kernel_count += in[q].kernel_count;
            as.x[q] = x[k];
            as.e[q] = ir.e32[k];
        }
        hipLaunchKernelGGL(k_add3_f32, dim3(gv), dim3(kBlock), 0, s, (long long)n, as, na);
        OASIS_TRY_LAUNCH();
    }
    int worst = OASIS_OK;
    for (int k = 0; k < nr; ++k)
        if (out[k].status != OASIS_OK && (worst == OASIS_OK || out[k].status < worst)) worst = out[k].status;
    return worst;
}

static double reliable_delta(double inner) { return (inner > 0.0 && inner < 1.0) ? inner : 0.1; }

// Default replacement factor of the step's mixed pressure solve
// (oasis_ipcs_params.pressure_delta = 0).  On the 129x129x97 channel (zero
// start, 1e-8) 0.1 takes 8 replacements per solve, 0.03 takes 6 at the same
// iteration count (0.6 ms less per step), 0.01 about 4 but 90 more
// iterations, 0.3 16.
constexpr double kPressureDelta = 0.03;

static KOpts kopts(const oasis_krylov_opts *o) {
    KOpts k;
    k.rtol = o->rtol;
    k.maxit = o->maxit > 0 ? o->maxit : 10000;
    k.inner_rtol = o->inner_rtol > 0 ? o->inner_rtol : 1e-4;
    k.max_outer = o->max_outer > 0 ? o->max_outer : 50;
    k.check_every = o->check_every;
    k.time = (o->flags & OASIS_KRYLOV_TIME) != 0;
    return k;
}

}  // namespace oasis

using namespace oasis;

// ---------------------------------------------------------------------------
// the IPCS handle

struct oasis_ipcs {
    oasis_ipcs() = default;
    oasis_ipcs(const oasis_ipcs &) = delete;
    oasis_ipcs &operator=(const oasis_ipcs &) = delete;
    ~oasis_ipcs() { stage_free(stage); }
    HostStage stage;   // pinned read-back block of the solver loops
    oasis_mesh mesh;
    std::vector<int> color_ptr;
    int dim = 0, n = 0, nnz = 0;
    const int *rp = nullptr, *ci = nullptr;
    oasis_ipcs_params par;
    Tuning tun;
    bool mixed = false;
    double *M = nullptr, *Ks = nullptr, *dP[3] = {nullptr, nullptr, nullptr}, *B = nullptr, *A = nullptr;
    float *A32 = nullptr, *Ks32 = nullptr;
    double *ML = nullptr, *sK = nullptr, *wK = nullptr, *dA = nullptr, *wA = nullptr, *dtmp = nullptr;
    double *rtmp = nullptr;   // residual scratch of the warm-start guard
    short *ecol = nullptr;    // ELL column offsets of the shared pattern (when they fit)
    unsigned short *pid = nullptr;   // their pattern dictionary: id per row,
    short *ptab = nullptr;           // offset lists
    EllCols cols;             // what the ELL products use (none when the offsets do not fit)
    double *eval = nullptr;   // ELL values of the pressure matrix: FP64 (FP64 mode) or
    float *eval32 = nullptr;  // their FP32 rounding (mixed mode)
    double *eA = nullptr;     // ELL values of the column-scaled tentative matrix, per step:
    float *eA32 = nullptr;    // FP64 (FP64 mode) or FP32 (mixed mode)
    bool ell = false;         // the offsets fit
    float *wK32 = nullptr, *wA32 = nullptr, *vnull32 = nullptr, *xlo = nullptr;
    double vscale = 0.0;      // ||s||^2: the pressure norm weights are vscale * vnull32^2
    double *rhi = nullptr;
    int *bc_index = nullptr, *flag = nullptr;
    int *iptr = nullptr, *inc = nullptr, *icnt = nullptr, *itmp = nullptr;
    // the row kernels' copy of the mesh: vertices in dof order, cells in
    // order of their lowest dof (locality of the per-row cell walks whatever
    // order the caller's arrays have); same geometry and dofs
    oasis_mesh rmesh{};
    int *rcells = nullptr, *rv2d = nullptr;
    double *rcoords = nullptr;
    int assembly = OASIS_ASSEMBLE_ROWS, maxc = 16;
    int r0_grid = 0;          // one-round grid of the tentative kernel that writes r0 (0: not yet known)
    double *ubar = nullptr;   // per step u_bar, interleaved ([n][D == 3 ? 4 : 2])
    double *bt[3] = {nullptr, nullptr, nullptr}, *ui[3] = {nullptr, nullptr, nullptr};
    double *bphi = nullptr, *bs = nullptr, *xs = nullptr, *xg = nullptr, *red = nullptr;
    CGWork<double> cg;
    CGWork<float> cg32;
    BiWork<double> bi;
    BiWork<float> bi32;
    IRBufs ir;
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // multigrid preconditioner of the pressure solve (optional)
    oasis_amg *amg = nullptr;
    // options of Alg. 1 / Sec. 5 / eq:scalar_disc
    int inner = 1;            // inner velocity-pressure iterations
    bool consistent = false;  // consistent-mass velocity update
    double *Ms = nullptr, *eM = nullptr, *sM = nullptr, *wM = nullptr;   // its scaled matrix
    CGWork<double> cgM;
    bool abe = false;         // explicit Adams-Bashforth convection
    double *cv[3] = {nullptr, nullptr, nullptr};   // its right-hand-side vectors
    double *uu = nullptr;     // U^{n-1}, U^{n-2} interleaved per dof
    bool gradient = false;    // weighted-gradient-matrix velocity update
    double *G[3] = {nullptr, nullptr, nullptr};    // G^k = M_L^{-1} dP^k
    int nsc = 0;              // passive scalars
    double *Bs[OASIS_MAX_SCALARS] = {nullptr, nullptr, nullptr, nullptr};   // M/dt + D K/2 each
    // learned warm start (optional)
    const float *ws_params = nullptr;
    const double *ws_coords = nullptr;
    void *ws_mem = nullptr;
    size_t ws_bytes = 0;
};

// ELL copy of a matrix on a CSR pattern and the pattern dictionary of its
// offsets; *cols receives the columns the products use (none when the
// offsets do not fit, and the products then run on CSR).  Synchronises.
static int ell_setup(hipStream_t s, int n, const int *rp, const int *ci, const double *val, short *ecol,
                     unsigned short *pid, short *ptab, double *eval, float *eval32, int *tmp, const Tuning &tun,
                     EllCols *cols, int *storage = nullptr) {
    bool fits = false;
    *cols = EllCols{};
    if (storage) *storage = 0;
    if (!tun.ell()) return OASIS_OK;
    OASIS_TRY(csr_to_ell(s, n, rp, ci, val, ecol, eval, eval32, tmp, &fits));
    if (!fits) return OASIS_OK;
    int npat = 0;
    OASIS_TRY(ell_dictionary(s, n, ecol, pid, ptab, &npat, tun.dict()));
    *cols = ell_cols(ecol, pid, ptab, npat);
    if (storage) *storage = npat > 0 ? npat : -1;
    return OASIS_OK;
}

static void carve_ipcs(Carver &c, int dim, int n, int ncell, int nvert, int nnz, bool mixed, bool consistent,
                       int nsc, bool abe, bool gradient, bool rows, oasis_ipcs &h) {
    h.ecol = c.take<short>((size_t)n * kEll);
    h.pid = c.take<unsigned short>(n);
    h.ptab = c.take<short>((size_t)kMaxEllPatterns * kEll);
    if (mixed) {
        h.eval32 = c.take<float>((size_t)n * kEll);
        h.eA32 = c.take<float>((size_t)n * kEll);
    } else {
        h.eval = c.take<double>((size_t)n * kEll);
        h.eA = c.take<double>((size_t)n * kEll);
    }
    h.M = c.take<double>(nnz);
    h.Ks = c.take<double>(nnz);
    for (int k = 0; k < dim; ++k) h.dP[k] = c.take<double>(nnz);
    h.B = c.take<double>(nnz);
    h.A = c.take<double>(nnz);
    if (mixed) {
        h.A32 = c.take<float>(nnz);
        h.Ks32 = c.take<float>(nnz);
        h.wK32 = c.take<float>(n);
        h.wA32 = c.take<float>(n);
        h.vnull32 = c.take<float>(n);
        h.xlo = c.take<float>(n);
        h.rhi = c.take<double>(n);
    }
    h.ML = c.take<double>(n);
    h.sK = c.take<double>(n);
    h.wK = c.take<double>(n);
    h.dA = c.take<double>(n);
    h.wA = c.take<double>(n);
    h.dtmp = c.take<double>(n);
    h.rtmp = c.take<double>(n);
    h.bc_index = c.take<int>(n);
    h.flag = c.take<int>(32);
    for (int k = 0; k < dim; ++k) {
        h.bt[k] = c.take<double>(n);
        h.ui[k] = c.take<double>(n);
    }
    h.bphi = c.take<double>(n);
    h.bs = c.take<double>(n);
    h.xs = c.take<double>(n);
    h.xg = c.take<double>(n);
    h.red = c.take<double>(2 * kMaxPartials);
    const int nmax = std::max(n, ncell);
    h.ubar = c.take<double>((size_t)n * (dim == 3 ? 4 : 2));
    h.iptr = c.take<int>((size_t)n + 1);
    if (rows || abe) {
        h.rcells = c.take<int>((size_t)ncell * (dim + 1));
        h.rv2d = c.take<int>((size_t)nvert);
        h.rcoords = c.take<double>((size_t)nvert * dim);
    }
    h.inc = c.take<int>((size_t)ncell * (dim + 1));
    h.icnt = c.take<int>((size_t)nmax + 1);
    h.itmp = c.take<int>(incidence_tmp_ints(nmax));
    carve_cg<double>(c, n, h.cg);
    carve_bi<double>(c, n, dim, h.bi);
    if (mixed) {
        carve_cg<float>(c, n, h.cg32);
        carve_bi<float>(c, n, dim, h.bi32);
        carve_ir(c, n, dim, h.ir);
    }
    if (consistent) {
        h.Ms = c.take<double>(nnz);
        h.eM = c.take<double>((size_t)n * kEll);
        h.sM = c.take<double>(n);
        h.wM = c.take<double>(n);
        carve_cg<double>(c, n, h.cgM);
    }
    for (int a = 0; a < nsc; ++a) h.Bs[a] = c.take<double>(nnz);
    if (abe) {
        for (int k = 0; k < dim; ++k) h.cv[k] = c.take<double>(n);
        h.uu = c.take<double>((size_t)n * (dim == 3 ? 8 : 4));
    }
    if (gradient)
        for (int k = 0; k < dim; ++k) h.G[k] = c.take<double>(nnz);
}

static int check_params(const oasis_ipcs_params *p) {
    if (!p || !(p->dt > 0) || !(p->nu >= 0) || p->n_bc < 0 || (p->n_bc > 0 && !p->bc_dofs)) return OASIS_EINVAL;
    if (!(p->rtol_u > 0) || !(p->rtol_p > 0)) return OASIS_EINVAL;
    if (p->precision != OASIS_F64 && p->precision != OASIS_F32) return OASIS_EINVAL;
    if (p->pressure_start != OASIS_PSTART_PREV && p->pressure_start != OASIS_PSTART_ZERO) return OASIS_EINVAL;
    if (!(p->pressure_delta >= 0.0 && p->pressure_delta < 1.0)) return OASIS_EINVAL;
    if (p->inner_iters < 0 || p->inner_iters > 16) return OASIS_EINVAL;
    if (p->velocity_update != OASIS_UPDATE_LUMPED && p->velocity_update != OASIS_UPDATE_CONSISTENT &&
        p->velocity_update != OASIS_UPDATE_GRADIENT)
        return OASIS_EINVAL;
    if (p->convection != OASIS_CONV_ABCN && p->convection != OASIS_CONV_ABE) return OASIS_EINVAL;
    if (p->n_scalars < 0 || p->n_scalars > OASIS_MAX_SCALARS) return OASIS_EINVAL;
    for (int a = 0; a < p->n_scalars; ++a)
        if (!(p->diffusivity[a] >= 0.0) || !std::isfinite(p->diffusivity[a]) || !std::isfinite(p->scalar_source[a]))
            return OASIS_EINVAL;
    Tuning t;
    return Tuning::from(&p->tuning, &t);
}

extern "C" int oasis_ipcs_workspace_size(const oasis_mesh *mesh, int32_t nnz, const oasis_ipcs_params *par,
                                         size_t *bytes) {
    if (!mesh || !bytes || nnz <= 0 || (mesh->dim != 2 && mesh->dim != 3) || mesh->n_dof <= 0) return OASIS_EINVAL;
    OASIS_TRY(check_params(par));
    Carver c(nullptr, 0);
    oasis_ipcs h;
    carve_ipcs(c, mesh->dim, mesh->n_dof, mesh->n_cell, mesh->n_vert, nnz, par->precision == OASIS_F32,
               par->velocity_update == OASIS_UPDATE_CONSISTENT, par->n_scalars, par->convection == OASIS_CONV_ABE,
               par->velocity_update == OASIS_UPDATE_GRADIENT, par->assembly != OASIS_ASSEMBLE_COLORS, h);
    *bytes = c.bytes();
    return OASIS_OK;
}

static inline int gvec(int n) { return grid_for(n, kBlock, 8192); }

// The row kernels' mesh copy: vertices renumbered in dof order and cells
// sorted by their lowest dof (both stable counting sorts on the host, once),
// so that the cells a row walks, and their vertices, sit near each other in
// memory whatever order the caller's arrays have.  Synchronises.
static int locality_mesh(hipStream_t s, const oasis_mesh *m, int *rcells, int *rv2d, double *rcoords,
                         oasis_mesh *out) {
    const int nv = m->n_vert, nc = m->n_cell, D = m->dim, NV = D + 1, n = m->n_dof;
    std::vector<int> cells((size_t)nc * NV), v2d(nv);
    std::vector<double> X((size_t)nv * D);
    OASIS_TRY_HIP(hipMemcpyAsync(cells.data(), m->cells, cells.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipMemcpyAsync(v2d.data(), m->vert2dof, v2d.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipMemcpyAsync(X.data(), m->coords, X.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    // vertices by dof (stable)
    std::vector<int> cnt(n + 1, 0), vnew(nv);
    for (int v = 0; v < nv; ++v) {
        if (v2d[v] < 0 || v2d[v] >= n) return OASIS_EINVAL;
        ++cnt[v2d[v] + 1];
    }
    for (int d = 0; d < n; ++d) cnt[d + 1] += cnt[d];
    std::vector<int> v2dr(nv);
    std::vector<double> Xr((size_t)nv * D);
    for (int v = 0; v < nv; ++v) {
        const int q = cnt[v2d[v]]++;
        vnew[v] = q;
        v2dr[q] = v2d[v];
        for (int c = 0; c < D; ++c) Xr[(size_t)q * D + c] = X[(size_t)v * D + c];
    }
    // cells by their lowest dof (stable), vertex ids renumbered
    std::fill(cnt.begin(), cnt.end(), 0);
    std::vector<int> key(nc);
    for (int e = 0; e < nc; ++e) {
        int k = n;
        for (int a = 0; a < NV; ++a) {
            const int v = cells[(size_t)e * NV + a];
            if (v < 0 || v >= nv) return OASIS_EINVAL;
            k = std::min(k, v2d[v]);
        }
        key[e] = k;
        ++cnt[k + 1];
    }
    for (int d = 0; d < n; ++d) cnt[d + 1] += cnt[d];
    std::vector<int> cr((size_t)nc * NV);
    for (int e = 0; e < nc; ++e) {
        const int q = cnt[key[e]]++;
        for (int a = 0; a < NV; ++a) cr[(size_t)q * NV + a] = vnew[cells[(size_t)e * NV + a]];
    }
    OASIS_TRY_HIP(hipMemcpyAsync(rcells, cr.data(), cr.size() * sizeof(int), hipMemcpyHostToDevice, s));
    OASIS_TRY_HIP(hipMemcpyAsync(rv2d, v2dr.data(), v2dr.size() * sizeof(int), hipMemcpyHostToDevice, s));
    OASIS_TRY_HIP(hipMemcpyAsync(rcoords, Xr.data(), Xr.size() * sizeof(double), hipMemcpyHostToDevice, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    *out = *m;
    out->cells = rcells;
    out->vert2dof = rv2d;
    out->coords = rcoords;
    out->n_colors = 0;
    out->color_ptr = nullptr;
    out->color_cells = nullptr;
    return OASIS_OK;
}

extern "C" int oasis_ipcs_create(void *stream, const oasis_mesh *mesh, const int32_t *row_ptr,
                                 const int32_t *col_idx, int32_t nnz, const oasis_ipcs_params *par,
                                 void *ws, size_t ws_bytes, oasis_ipcs **out) {
    if (!out) return OASIS_EINVAL;
    *out = nullptr;
    OASIS_TRY(check_mesh_colored(mesh));
    OASIS_TRY(check_params(par));
    if (!row_ptr || !col_idx || nnz <= 0 || !ws || !aligned(ws, 256)) return OASIS_EINVAL;
    hipStream_t s = as_stream(stream);
    oasis_ipcs *h = new (std::nothrow) oasis_ipcs();
    if (!h) return OASIS_EINVAL;
    h->mesh = *mesh;
    h->color_ptr.assign(mesh->color_ptr, mesh->color_ptr + mesh->n_colors + 1);
    h->mesh.color_ptr = h->color_ptr.data();
    h->dim = mesh->dim;
    h->n = mesh->n_dof;
    h->nnz = nnz;
    h->rp = row_ptr;
    h->ci = col_idx;
    h->par = *par;
    (void)Tuning::from(&par->tuning, &h->tun);
    h->mixed = par->precision == OASIS_F32;
    h->inner = par->inner_iters > 0 ? par->inner_iters : 1;
    h->consistent = par->velocity_update == OASIS_UPDATE_CONSISTENT;
    h->nsc = par->n_scalars;
    h->abe = par->convection == OASIS_CONV_ABE;
    h->gradient = par->velocity_update == OASIS_UPDATE_GRADIENT;
    Carver c(ws, ws_bytes);
    carve_ipcs(c, h->dim, h->n, mesh->n_cell, mesh->n_vert, nnz, h->mixed, h->consistent, h->nsc, h->abe,
               h->gradient, par->assembly != OASIS_ASSEMBLE_COLORS, *h);
    h->cg.tun = h->cg32.tun = h->cgM.tun = h->tun;
    h->bi.tun = h->bi32.tun = h->tun;
    stage_alloc(h->stage);
    h->cg.stage = h->cg32.stage = h->cgM.stage = h->stage;
    h->bi.stage = h->bi32.stage = h->ir.stage = h->stage;
    auto fail = [&](int rc) {
        delete h;
        return rc;
    };
    if (!c.ok) return fail(OASIS_EWORKSPACE);
    for (int k = 0; k < 6; ++k)
        if (hipEventCreate(&h->ev[k]) != hipSuccess) return fail(OASIS_EHIP);
    const int n = h->n, D = h->dim;
    int rc = OASIS_OK;
    auto step = [&](int r) {
        if (rc == OASIS_OK && r != OASIS_OK) rc = r;
    };
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, s, 16, h->flag, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(gvec(n)), dim3(kBlock), 0, s, n, h->bc_index, -1);
    if (par->n_bc > 0)
        hipLaunchKernelGGL(k_bc_index, dim3(gvec(par->n_bc)), dim3(kBlock), 0, s, par->n_bc, n, par->bc_dofs,
                           h->bc_index, h->flag + 2);
    P3 none{};
    // preassembled matrices (Sec. 5: assembled once)
    step(scale_copy(s, nnz, h->M, nullptr, 0.0));
    step(assemble_colored(s, &h->mesh, row_ptr, col_idx, h->M, OASIS_FORM_MASS, 1.0, none, none, 0, 0, h->flag));
    step(scale_copy(s, nnz, h->B, nullptr, 0.0));
    step(assemble_colored(s, &h->mesh, row_ptr, col_idx, h->B, OASIS_FORM_STIFF, 1.0, none, none, 0, 0, h->flag));
    for (int k = 0; k < D; ++k) {
        step(scale_copy(s, nnz, h->dP[k], nullptr, 0.0));
        step(assemble_colored(s, &h->mesh, row_ptr, col_idx, h->dP[k], OASIS_FORM_GRAD_X + k, 1.0, none, none,
                              0, 0, h->flag));
    }
    if (rc != OASIS_OK) return fail(rc);
    // K currently in B: diagonal, scaled copy, then B = M/dt + nu K / 2
    hipLaunchKernelGGL((k_diag<double>), dim3(gvec(n)), dim3(kBlock), 0, s, n, row_ptr, col_idx, h->B, h->dtmp);
    hipLaunchKernelGGL(k_diag_vectors, dim3(gvec(n)), dim3(kBlock), 0, s, n, h->dtmp, 0, h->sK, h->wK, h->wK32,
                       h->flag + 1);
    hipLaunchKernelGGL(k_scale_matrix, dim3(gvec(n)), dim3(kBlock), 0, s, n, row_ptr, col_idx, h->B, h->sK, kScaleSym,
                       h->Ks, h->Ks32);
    // scalars: M/dt + D K/2 each (before B takes its own combination)
    for (int a = 0; a < h->nsc; ++a)
        hipLaunchKernelGGL(k_lincomb, dim3(gvec(nnz)), dim3(kBlock), 0, s, (long long)nnz, h->Bs[a], h->M,
                           1.0 / par->dt, h->B, 0.5 * par->diffusivity[a]);
    hipLaunchKernelGGL(k_lincomb, dim3(gvec(nnz)), dim3(kBlock), 0, s, (long long)nnz, h->B, h->M,
                       1.0 / par->dt, h->B, 0.5 * par->nu);
    // consistent update: M with the Dirichlet dofs eliminated, symmetrically scaled
    if (h->consistent) {
        hipLaunchKernelGGL(k_mass_bc, dim3(gvec(n)), dim3(kBlock), 0, s, n, row_ptr, col_idx, h->M, h->bc_index,
                           h->Ms);
        hipLaunchKernelGGL((k_diag<double>), dim3(gvec(n)), dim3(kBlock), 0, s, n, row_ptr, col_idx, h->Ms,
                           h->dtmp);
        hipLaunchKernelGGL(k_diag_vectors, dim3(gvec(n)), dim3(kBlock), 0, s, n, h->dtmp, 0, h->sM, h->wM,
                           static_cast<float *>(nullptr), h->flag + 1);
        hipLaunchKernelGGL(k_scale_matrix, dim3(gvec(n)), dim3(kBlock), 0, s, n, row_ptr, col_idx, h->Ms, h->sM,
                           kScaleSym, h->Ms, static_cast<float *>(nullptr));
    }
    hipLaunchKernelGGL(k_row_sums, dim3(gvec(n)), dim3(kBlock), 0, s, n, row_ptr, h->M, h->ML);
    if (h->gradient)
        for (int k = 0; k < D; ++k)
            hipLaunchKernelGGL(k_row_div, dim3(gvec(n)), dim3(kBlock), 0, s, n, row_ptr, h->dP[k], h->ML, h->G[k]);
    if (hipGetLastError() != hipSuccess) return fail(OASIS_EHIP);
    // ELL copy of the pressure matrix for the CG product when its rows and
    // column offsets allow it (else the CSR product runs)
    {
        const int rc4 = ell_setup(s, n, row_ptr, col_idx, h->Ks, h->ecol, h->pid, h->ptab, h->eval, h->eval32,
                                  h->flag + 24, h->tun, &h->cols);
        if (rc4 != OASIS_OK) return fail(rc4);
        const bool fits = h->cols.any();
        h->ell = fits;
        if (fits && h->consistent) {
            // the mass matrix's ELL values on the same columns
            bool f2 = false;
            const int rc5 = csr_to_ell(s, n, row_ptr, col_idx, h->Ms, h->ecol, h->eM, nullptr, h->flag + 24, &f2);
            if (rc5 != OASIS_OK) return fail(rc5);
            if (f2) {
                h->cgM.cols = h->cols;
                h->cgM.eval = h->eM;
            }
        }
        if (fits && h->mixed) {
            h->cg32.cols = h->bi32.cols = h->cols;
            h->cg32.eval = h->eval32;
            h->bi32.eval = h->eA32;
        } else if (fits) {
            h->cg.cols = h->bi.cols = h->cols;
            h->cg.eval = h->eval;
            h->bi.eval = h->eA;
        }
    }
    // row-gather assembly: dof -> cell lists and the longest row
    h->assembly = par->assembly == OASIS_ASSEMBLE_COLORS ? OASIS_ASSEMBLE_COLORS : OASIS_ASSEMBLE_ROWS;
    if (h->assembly == OASIS_ASSEMBLE_ROWS) {
        std::vector<int> rph(n + 1);
        if (hipMemcpyAsync(rph.data(), row_ptr, (n + 1) * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(OASIS_EHIP);
        int maxrow = 0;
        for (int i = 0; i < n; ++i) maxrow = std::max(maxrow, rph[i + 1] - rph[i]);
        if (maxrow <= 16)
            h->maxc = 16;
        else if (maxrow <= 32)
            h->maxc = 32;
        else
            h->assembly = OASIS_ASSEMBLE_COLORS;
    }
    // dof -> incident cells: the row-gather assembly and the explicit convection
    if (h->assembly == OASIS_ASSEMBLE_ROWS || h->abe) {
        const int rc1 = locality_mesh(s, mesh, h->rcells, h->rv2d, h->rcoords, &h->rmesh);
        if (rc1 != OASIS_OK) return fail(rc1);
        const int rc2 = incidence_codes(s, &h->rmesh, h->iptr, h->inc, h->icnt, h->itmp, h->flag + 3);
        if (rc2 != OASIS_OK) return fail(rc2);
    }
    // the scaled pressure matrix has null vector s = sqrt(diag K) (K 1 = 0)
    // with it, the norm weights d = s^2 of the FP32 iterations are ||s||^2 v^2
    if (h->mixed && unit_vector_f32(s, n, h->sK, h->red, h->vnull32, &h->vscale) != OASIS_OK)
        return fail(OASIS_EHIP);
    int fl[3] = {0, 0, 0};
    if (hipMemcpyAsync(fl, h->flag, sizeof(fl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(OASIS_EHIP);
    if (fl[0] || fl[1] || fl[2]) return fail(OASIS_EINVAL);
    *out = h;
    return OASIS_OK;
}

extern "C" int oasis_ipcs_destroy(oasis_ipcs *h) {
    if (!h) return OASIS_EINVAL;
    for (auto &e : h->ev)
        if (e) (void)hipEventDestroy(e);
    delete h;
    return OASIS_OK;
}

extern "C" int oasis_ipcs_set_warmstart(oasis_ipcs *h, const float *params, const double *coords, void *ws,
                                        size_t ws_bytes) {
    if (!h) return OASIS_EINVAL;
    if (!params) {
        h->ws_params = nullptr;
        h->ws_coords = nullptr;
        h->ws_mem = nullptr;
        h->ws_bytes = 0;
        return OASIS_OK;
    }
    size_t need = 0;
    OASIS_TRY(oasis_mpnn_workspace_size(h->n, &need));
    if (!coords || !ws || ws_bytes < need) return ws_bytes < need ? OASIS_EWORKSPACE : OASIS_EINVAL;
    h->ws_params = params;
    h->ws_coords = coords;
    h->ws_mem = ws;
    h->ws_bytes = ws_bytes;
    return OASIS_OK;
}

extern "C" int oasis_ipcs_set_amg(oasis_ipcs *h, oasis_amg *amg) {
    if (!h) return OASIS_EINVAL;
    if (amg && !amg_handle_matches(amg, h->n, h->rp, h->Ks, h->sK)) return OASIS_EINVAL;
    h->amg = amg;
    return OASIS_OK;
}

extern "C" int oasis_ipcs_matrix(const oasis_ipcs *h, int32_t which, const double **val,
                                 const double **scaled_diag_sqrt) {
    if (!h || !val) return OASIS_EINVAL;
    if (scaled_diag_sqrt) *scaled_diag_sqrt = nullptr;
    switch (which) {
        case -1: *val = h->ML; return OASIS_OK;
        case OASIS_FORM_MASS: *val = h->M; return OASIS_OK;
        case OASIS_FORM_STIFF:
            *val = h->Ks;
            if (scaled_diag_sqrt) *scaled_diag_sqrt = h->sK;
            return OASIS_OK;
        case OASIS_FORM_GRAD_X: case OASIS_FORM_GRAD_Y: case OASIS_FORM_GRAD_Z:
            if (which - OASIS_FORM_GRAD_X >= h->dim) return OASIS_EINVAL;
            *val = h->dP[which - OASIS_FORM_GRAD_X];
            return OASIS_OK;
        case OASIS_INSPECT_A: *val = h->A; return OASIS_OK;
        case OASIS_INSPECT_DIAG_A: *val = h->dA; return OASIS_OK;
        case OASIS_INSPECT_RHS: case OASIS_INSPECT_RHS + 1: case OASIS_INSPECT_RHS + 2:
            if (which - OASIS_INSPECT_RHS >= h->dim) return OASIS_EINVAL;
            *val = h->bt[which - OASIS_INSPECT_RHS];
            return OASIS_OK;
        default: return OASIS_EINVAL;
    }
}

// gp: the pressure term is already in h->bt (k_asm_rows<.., true>); cs:
// the diagonal is already in h->dA, and the column scaling is done here
// (no k_colscale pass afterwards); r0 (with cs, mixed mode): also the
// refinement loop's first residual into h->ir, returning the number of
// partials written (0 otherwise)
// Blocks of kBlock threads that fill every CU once at `kern`'s occupancy,
// at most kMaxPartials: a partial-writing grid without a partly filled
// last round
template <class K>
static int one_round_grid(K kern) {
    int dev = 0, cu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kBlock, 0) != hipSuccess || per < 1 || cu < 1)
        return kMaxPartials / 4;
    return std::min(kMaxPartials, per * cu);
}

template <int D, int L>
static int launch_step_kernels_tent(hipStream_t s, oasis_ipcs *h, const oasis_state *st, const double *g,
                                    double *const *x, bool gp = false, bool cs = false, bool r0 = false) {
    const int n = h->n;
    P3 dP{}, U1{}, cv{};
    for (int k = 0; k < D; ++k) {
        dP.p[k] = h->dP[k];
        U1.p[k] = st->U1[k];
        cv.p[k] = h->abe ? h->cv[k] : nullptr;
    }
    r0 = r0 && cs && h->mixed;
    // the partials of the first residual: at most kMaxPartials blocks, and
    // then one round of resident blocks (on gfx950 six per CU: 1536; 2048
    // left a partly filled second round, 400 against 337 us)
    if (r0 && h->r0_grid == 0) {
        if constexpr (D == 3)
            h->r0_grid = gp ? one_round_grid(k_tent_rows<D, L, true, true>)
                            : one_round_grid(k_tent_rows<D, L, false, true>);
        else
            h->r0_grid = one_round_grid(k_tent_rows<D, L, false, true>);
    }
    const int grid = grid_for(n, kBlock / L, r0 ? h->r0_grid : 1 << 20);
    const bool e = h->ell && h->tun.ell();
    P3F r0o{};
    for (int k = 0; k < D && r0; ++k) r0o.p[k] = h->ir.r32[k];
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, n, h->rp, h->ci, h->M, h->A, dP, U1, cv, st->p,
                           h->ML, h->bc_index, g, h->par.n_bc, h->par.f[0], h->par.f[1], h->par.f[2],
                           2.0 / h->par.dt, h->bt[0], h->bt[1], D > 2 ? h->bt[2] : nullptr, x[0], x[1],
                           D > 2 ? x[2] : nullptr, h->dA, h->wA, h->wA32, h->mixed && !e ? h->A32 : nullptr,
                           e ? h->eA : nullptr, e ? h->eA32 : nullptr, r0o, r0 ? h->ir.part : nullptr);
    };
    if constexpr (D == 3) {
        if (gp && cs) {
            go(k_tent_rows<D, L, true, true>);
            return r0 ? grid : 0;
        }
    }
    if (cs)
        go(k_tent_rows<D, L, false, true>);
    else
        go(k_tent_rows<D, L, false, false>);
    return r0 ? grid : 0;
}

// A = Bsrc + C(u_bar)/2 by the row-gather kernel (u_bar already in h->ubar);
// with GP also the pressure term dP^k p into h->bt (3D, p in the records)
// and with cs the diagonal into h->dA
template <int D, int MAXC, bool GP>
static void launch_asm_kernel(hipStream_t s, oasis_ipcs *h, const double *Bsrc, bool cs) {
    hipLaunchKernelGGL((k_asm_rows<D, MAXC, GP>), dim3(grid_for(h->n, kBlock, 1 << 20)), dim3(kBlock), 0, s,
                       h->n, h->rp, h->ci, Bsrc, h->iptr, h->inc, h->rmesh.cells, h->rmesh.vert2dof,
                       h->rmesh.coords, h->ubar, h->A, GP ? h->bt[0] : nullptr, GP ? h->bt[1] : nullptr,
                       GP ? h->bt[2] : nullptr, h->bc_index, cs ? h->dA : nullptr);
}

// gp: only for 3D rows of at most 16 entries (with 32 slots the extra
// registers would halve the kernel's occupancy)
static bool asm_gradient(const oasis_ipcs *h) { return h->dim == 3 && h->maxc == 16; }

static void launch_asm(hipStream_t s, oasis_ipcs *h, const double *Bsrc, bool gp = false, bool cs = false) {
    if (h->dim == 3 && h->maxc == 16 && gp)
        launch_asm_kernel<3, 16, true>(s, h, Bsrc, cs);
    else if (h->dim == 3 && h->maxc == 16)
        launch_asm_kernel<3, 16, false>(s, h, Bsrc, cs);
    else if (h->dim == 3)
        launch_asm_kernel<3, 32, false>(s, h, Bsrc, cs);
    else if (h->maxc == 16)
        launch_asm_kernel<2, 16, false>(s, h, Bsrc, cs);
    else
        launch_asm_kernel<2, 32, false>(s, h, Bsrc, cs);
}

template <int D>
static int launch_asm_rows(hipStream_t s, oasis_ipcs *h, const oasis_state *st, const double *g, double *const *x) {
    const int n = h->n;
    P3 U1{}, U2{};
    for (int k = 0; k < D; ++k) {
        U1.p[k] = st->U1[k];
        U2.p[k] = st->U2[k];
    }
    // in 3D the records carry p, and the assembly also forms dP^k p
    const bool gp = asm_gradient(h);
    hipLaunchKernelGGL((k_ubar<D>), dim3(gvec(n)), dim3(kBlock), 0, s, n, U1, U2,
                       gp ? static_cast<const double *>(st->p) : nullptr, h->ubar);
    launch_asm(s, h, h->B, gp, true);
    // right-hand sides, Dirichlet rows, y0, the column scaling and (mixed
    // mode) the first refinement residual, 8 lanes per row
    return launch_step_kernels_tent<D, 8>(s, h, st, g, x, gp, true, true);
}

template <int D, int L>
static void launch_div(hipStream_t s, oasis_ipcs *h, double *const *x, int *gout) {
    P3 dP{}, UI{};
    for (int k = 0; k < D; ++k) {
        dP.p[k] = h->dP[k];
        UI.p[k] = x[k];
    }
    const int grid = grid_for(h->n, kBlock / L);
    *gout = grid;
    hipLaunchKernelGGL((k_div_rows<D, L>), dim3(grid), dim3(kBlock), 0, s, h->n, h->rp, h->ci, dP, UI,
                       -1.0 / h->par.dt, h->bphi, h->red);
}

template <int D, int L>
static void launch_update(hipStream_t s, oasis_ipcs *h, double *const *x, const double *phi, const double *g,
                          double *const *un) {
    P3 dP{}, UI{};
    for (int k = 0; k < D; ++k) {
        dP.p[k] = h->gradient ? h->G[k] : h->dP[k];
        UI.p[k] = x[k];
    }
    const int grid = grid_for(h->n, kBlock / L, 1 << 20);
    hipLaunchKernelGGL((k_update_rows<D, L>), dim3(grid), dim3(kBlock), 0, s, h->n, h->rp, h->ci, dP, UI, phi,
                       h->gradient ? static_cast<const double *>(nullptr) : h->ML, h->bc_index, g, h->par.n_bc,
                       h->par.dt, un[0], un[1], D > 2 ? un[2] : nullptr);
}

// One passive scalar: A_c = M/dt + D K/2 + C(u_bar)/2 by the step's
// assembly (into h->A: the velocity's matrix is no longer needed), the
// right-hand side (2M/dt - A_c) c^{n-1} + f M_L with the Dirichlet rows
// (k_tent_rows for one field without pressure gradient), column scaling,
// BiCGStab in the step's precision, unscaling into Cn.
static int scalar_solve(hipStream_t s, oasis_ipcs *h, oasis_state *st, int a, int D, const oasis_krylov_opts &o0,
                        oasis_step_stats &S, int *status) {
    const int n = h->n;
    if (!st->C1[a] || !st->Cn[a] || (h->par.n_bc > 0 && !st->C_bc[a])) return OASIS_EINVAL;
    if (h->assembly == OASIS_ASSEMBLE_ROWS) {
        launch_asm(s, h, h->Bs[a]);
        OASIS_TRY_LAUNCH();
    } else {
        P3 U1{}, U2{};
        for (int k = 0; k < D; ++k) {
            U1.p[k] = st->U1[k];
            U2.p[k] = st->U2[k];
        }
        OASIS_TRY(scale_copy(s, h->nnz, h->A, h->Bs[a], 1.0));
        OASIS_TRY(assemble_colored(s, &h->mesh, h->rp, h->ci, h->A, OASIS_FORM_CONV, 0.5, U1, U2, 1.5, -0.5,
                                   nullptr));
    }
    P3 none{}, C1{};
    C1.p[0] = st->C1[a];
    const int grid = grid_for(n, kBlock / 8, 1 << 20);
    hipLaunchKernelGGL((k_tent_rows<1, 8>), dim3(grid), dim3(kBlock), 0, s, n, h->rp, h->ci, h->M, h->A, none, C1,
                       none, static_cast<const double *>(nullptr), h->ML, h->bc_index, st->C_bc[a], h->par.n_bc,
                       h->par.scalar_source[a], 0.0, 0.0, 2.0 / h->par.dt, h->bt[0], static_cast<double *>(nullptr),
                       static_cast<double *>(nullptr), st->Cn[a], static_cast<double *>(nullptr),
                       static_cast<double *>(nullptr), h->dA, h->wA, h->wA32, static_cast<float *>(nullptr),
                       static_cast<double *>(nullptr), static_cast<float *>(nullptr), P3F{},
                       static_cast<double *>(nullptr));
    OASIS_TRY_LAUNCH();
    const bool e = h->ell && h->tun.ell();
    hipLaunchKernelGGL(k_colscale, dim3(grid_for(n, kBlock / kEll, 1 << 20)), dim3(kBlock), 0, s, n, h->rp, h->ci,
                       h->dA, h->A, h->mixed && !e ? h->A32 : nullptr, e ? h->eA : nullptr, e ? h->eA32 : nullptr);
    OASIS_TRY_LAUNCH();
    oasis_krylov_opts o = o0;
    o.rtol = h->par.rtol_u;
    const KOpts ko = kopts(&o);
    double *b[3] = {h->bt[0], nullptr, nullptr};
    double *x[3] = {st->Cn[a], nullptr, nullptr};
    SolveOut sc[3];
    int rc;
    if (h->mixed)
        rc = ir_bicgstab(s, n, 1, h->rp, h->ci, h->A, h->A32, h->wA, h->wA32, b, x, ko, h->bi32, h->ir, sc);
    else
        rc = bicgstab_solve<double>(s, n, 1, h->rp, h->ci, h->A, h->wA, b, x, ko.rtol, ko.maxit, 0, false, h->bi, sc);
    if (rc == OASIS_EHIP) return rc;
    hipLaunchKernelGGL(k_scale3, dim3(gvec(n)), dim3(kBlock), 0, s, n, h->dA, 2, st->Cn[a],
                       static_cast<double *>(nullptr), static_cast<double *>(nullptr));
    OASIS_TRY_LAUNCH();
    S.iters_c[a] = sc[0].iters;
    S.res_c[a] = sc[0].rel_res;
    *status = sc[0].status;
    return OASIS_OK;
}

// J(x) = -1/2 x^T (r + b) on the scaled pressure system (r = b - Ks x from
// the residual pass); synchronises
static int step_energy(hipStream_t s, oasis_ipcs *h, const double *x, double *J) {
    double wrr = 0, wbb = 0;
    OASIS_TRY(cg_residual(s, h->n, h->rp, h->ci, h->Ks, h->wK, h->bs, x, h->rtmp, h->cg, &wrr, &wbb));
    const int g = grid_for(h->n, kBlock);
    hipLaunchKernelGGL(k_energy_part, dim3(g), dim3(kBlock), 0, s, h->n, x, h->rtmp, h->bs, h->red);
    hipLaunchKernelGGL((k_sum_to<1>), dim3(1), dim3(kBlock), 0, s, h->red, g, h->red + kMaxPartials);
    OASIS_TRY_LAUNCH();
    double v = 0;
    OASIS_TRY(read_state(s, h->stage, h->red + kMaxPartials, &v, sizeof(v)));
    *J = -0.5 * v;
    return OASIS_OK;
}

extern "C" int oasis_ipcs_step(void *stream, oasis_ipcs *h, oasis_state *st, const double *bc_values,
                               const double *phi_guess, oasis_step_stats *stats) {
    if (!h || !st || !st->p || !st->phi) return OASIS_EINVAL;
    const int D = h->dim, n = h->n;
    for (int k = 0; k < D; ++k)
        if (!st->U1[k] || !st->U2[k] || !st->Un[k] || st->Un[k] == st->U1[k] || st->Un[k] == st->U2[k])
            return OASIS_EINVAL;
    if (h->par.n_bc > 0 && !bc_values) return OASIS_EINVAL;
    for (int a = 0; a < h->nsc; ++a)
        if (!st->C1[a] || !st->Cn[a] || st->Cn[a] == st->C1[a] || (h->par.n_bc > 0 && !st->C_bc[a]))
            return OASIS_EINVAL;
    hipStream_t s = as_stream(stream);
    oasis_step_stats loc{};
    oasis_step_stats &S = stats ? *stats : loc;
    S = oasis_step_stats{};
    OASIS_TRY_HIP(hipEventRecord(h->ev[0], s));
    P3 U1{}, U2{};
    for (int k = 0; k < D; ++k) {
        U1.p[k] = st->U1[k];
        U2.p[k] = st->U2[k];
    }
    double *x[3];
    for (int k = 0; k < D; ++k) x[k] = st->UI[k] ? st->UI[k] : h->ui[k];
    int r0_parts = 0;   // > 0: the tentative kernel left the first refinement residual in h->ir
    if (h->abe) {
        // 1+2 (eq:convection_ABE): A = M/dt + nu K/2, the explicit convection
        // vectors, right-hand sides, Dirichlet rows, diagonal; y0 = D U^{n-1}
        OASIS_TRY(scale_copy(s, h->nnz, h->A, h->B, 1.0));
        const int grid = grid_for(n, kBlock, 1 << 20);
        if (D == 3) {
            hipLaunchKernelGGL(k_uu<3>, dim3(gvec(n)), dim3(kBlock), 0, s, n, U1, U2, h->uu);
            hipLaunchKernelGGL(k_conv_rows<3>, dim3(grid), dim3(kBlock), 0, s, n, h->iptr, h->inc, h->rmesh.cells,
                               h->rmesh.vert2dof, h->rmesh.coords, h->uu, h->cv[0], h->cv[1], h->cv[2]);
            launch_step_kernels_tent<3, 8>(s, h, st, bc_values, x);
        } else {
            hipLaunchKernelGGL(k_uu<2>, dim3(gvec(n)), dim3(kBlock), 0, s, n, U1, U2, h->uu);
            hipLaunchKernelGGL(k_conv_rows<2>, dim3(grid), dim3(kBlock), 0, s, n, h->iptr, h->inc, h->rmesh.cells,
                               h->rmesh.vert2dof, h->rmesh.coords, h->uu, h->cv[0], h->cv[1],
                               static_cast<double *>(nullptr));
            launch_step_kernels_tent<2, 8>(s, h, st, bc_values, x);
        }
        OASIS_TRY_LAUNCH();
    } else if (h->assembly == OASIS_ASSEMBLE_ROWS) {
        // 1+2. rows gather A = B + C(u_bar)/2 and its diagonal, right-hand
        // sides, Dirichlet rows, column scaling
        if (D == 3)
            r0_parts = launch_asm_rows<3>(s, h, st, bc_values, x);
        else
            r0_parts = launch_asm_rows<2>(s, h, st, bc_values, x);
        OASIS_TRY_LAUNCH();
    } else {
        // 1. A = B + C(u_bar)/2, colour by colour
        OASIS_TRY(scale_copy(s, h->nnz, h->A, h->B, 1.0));
        OASIS_TRY(assemble_colored(s, &h->mesh, h->rp, h->ci, h->A, OASIS_FORM_CONV, 0.5, U1, U2, 1.5, -0.5,
                                   nullptr));
        // 2. right-hand sides, Dirichlet rows, diagonal; y0 = D U^{n-1}
        if (D == 3)
            launch_step_kernels_tent<3, 8>(s, h, st, bc_values, x);
        else
            launch_step_kernels_tent<2, 8>(s, h, st, bc_values, x);
        OASIS_TRY_LAUNCH();
    }
    // right Jacobi: the solves run on A D^{-1} in y = D x (ELL values for
    // the Krylov products when the pattern fits, else the FP32 CSR copy);
    // the row-gather path has scaled A already
    if (h->abe || h->assembly != OASIS_ASSEMBLE_ROWS) {
        const bool e = h->ell && h->tun.ell();
        hipLaunchKernelGGL(k_colscale, dim3(grid_for(n, kBlock / kEll, 1 << 20)), dim3(kBlock), 0, s, n, h->rp,
                           h->ci, h->dA, h->A, h->mixed && !e ? h->A32 : nullptr, e ? h->eA : nullptr,
                           e ? h->eA32 : nullptr);
        OASIS_TRY_LAUNCH();
    }
    OASIS_TRY_HIP(hipEventRecord(h->ev[1], s));
    oasis_krylov_opts o{};
    o.maxit = h->par.maxit > 0 ? h->par.maxit : 10000;
    // F32 velocity refinement: 3e-5 per inner solve, so that two passes
    // usually reach 1e-8 (1e-4 took three on the channel, 2.5% slower)
    o.inner_rtol = h->par.inner_rtol > 0 ? h->par.inner_rtol : 3e-5;
    int worst = OASIS_OK;
    auto note = [&](int status) {
        if (status != OASIS_OK && (worst == OASIS_OK || status < worst)) worst = status;
    };
    const int zero_start = h->par.pressure_start == OASIS_PSTART_ZERO ? 1 : 0;
    S.guess_used = 0;
    SolveOut su[3], sp;
    for (int it = 0; it < h->inner; ++it) {
        if (it > 0) {
            // 3'. p* grew by phi: b^k -= dP^k phi; start from the last U^I
            P3 dP{};
            for (int k = 0; k < D; ++k) dP.p[k] = h->dP[k];
            const int g8 = grid_for(n, kBlock / 8, 1 << 20);
            if (D == 3)
                hipLaunchKernelGGL((k_rhs_dp<3, 8>), dim3(g8), dim3(kBlock), 0, s, n, h->rp, h->ci, dP, st->phi,
                                   h->bc_index, h->bt[0], h->bt[1], h->bt[2]);
            else
                hipLaunchKernelGGL((k_rhs_dp<2, 8>), dim3(g8), dim3(kBlock), 0, s, n, h->rp, h->ci, dP, st->phi,
                                   h->bc_index, h->bt[0], h->bt[1], static_cast<double *>(nullptr));
            hipLaunchKernelGGL(k_scale3, dim3(gvec(n)), dim3(kBlock), 0, s, n, h->dA, 1, x[0], x[1],
                               D > 2 ? x[2] : nullptr);
            OASIS_TRY_LAUNCH();
        }
        // 3. tentative velocity
        o.rtol = h->par.rtol_u;
        KOpts ko = kopts(&o);
        SolveOut sui[3];
        int rc_u;
        if (h->mixed)
            rc_u = ir_bicgstab(s, n, D, h->rp, h->ci, h->A, h->A32, h->wA, h->wA32, h->bt, x, ko, h->bi32, h->ir,
                               sui, it == 0 ? r0_parts : 0);
        else
            rc_u = bicgstab_solve<double>(s, n, D, h->rp, h->ci, h->A, h->wA, h->bt, x, ko.rtol, ko.maxit, 0, false,
                                          h->bi, sui);
        if (rc_u == OASIS_EHIP) return rc_u;
        for (int k = 0; k < D; ++k) {
            su[k].iters += sui[k].iters;
            su[k].outer = std::max(su[k].outer, sui[k].outer);
            su[k].rel_res = sui[k].rel_res;
            note(sui[k].status);
        }
        hipLaunchKernelGGL(k_scale3, dim3(gvec(n)), dim3(kBlock), 0, s, n, h->dA, 2, x[0], x[1],
                           D > 2 ? x[2] : nullptr);
        OASIS_TRY_LAUNCH();
        if (it == 0) OASIS_TRY_HIP(hipEventRecord(h->ev[2], s));
        // 4. pressure correction
        int gd = 0;
        if (D == 3)
            launch_div<3, 8>(s, h, x, &gd);
        else
            launch_div<2, 8>(s, h, x, &gd);
        OASIS_TRY_LAUNCH();
        hipLaunchKernelGGL(k_bphi_finish, dim3(gvec(n)), dim3(kBlock), 0, s, n, h->red, gd, h->bphi, h->sK,
                           st->phi, it > 0 ? 1 : zero_start, h->bs, h->xs);
        OASIS_TRY_LAUNCH();
        if (st->b_phi) {
            hipLaunchKernelGGL(k_copy_d, dim3(gvec(n)), dim3(kBlock), 0, s, (long long)n, st->b_phi, h->bphi);
            OASIS_TRY_LAUNCH();
        }
        const double *guess = it == 0 ? phi_guess : nullptr;
        if (it == 0 && !guess && h->ws_params) {
            // learned warm start from the projected right-hand side and phi_prev
            oasis_csr Kc{n, h->nnz, h->rp, h->ci, h->Ks, OASIS_F64};
            OASIS_TRY(mpnn_infer(stream, &Kc, h->sK, D, h->ws_coords, h->bphi, st->phi, h->ws_params, h->dtmp,
                                 h->ws_mem, h->ws_bytes));
            guess = h->dtmp;
        }
        if (guess) {
            // compare the CG energies J = 1/2 x^T K x - b^T x of the guess and
            // of the plain start (J = 0 for phi_0 = 0): CG's error is measured
            // in the K-norm, and J(x) - J(x*) = 1/2 ||x - x*||_K^2, whereas
            // the residual norm weights the rough error modes by K^2.  The
            // scaled system has the same energies (x_s = s x, b_s = b / s).
            hipLaunchKernelGGL(k_vscale, dim3(gvec(n)), dim3(kBlock), 0, s, n, guess, h->sK, 1, h->xg);
            OASIS_TRY_LAUNCH();
            double j_guess = 0, j_plain = 0;
            OASIS_TRY(step_energy(s, h, h->xg, &j_guess));
            if (!zero_start) OASIS_TRY(step_energy(s, h, h->xs, &j_plain));
            if (std::isfinite(j_guess) && j_guess < j_plain) {
                hipLaunchKernelGGL(k_copy_d, dim3(gvec(n)), dim3(kBlock), 0, s, (long long)n, h->xs, h->xg);
                OASIS_TRY_LAUNCH();
                S.guess_used = 1;
            }
        }
        o.rtol = h->par.rtol_p;
        ko = kopts(&o);
        SolveOut spi;
        int rc_p;
        if (h->amg)
            // FP64 CG around the handle's cycle: the mixed CG (amg_pcg_mixed)
            // needs a cycle per residual replacement, which at the step's
            // tolerances costs more than its FP32 products save
            rc_p = amg_handle_solve(s, h->amg, h->wK, h->bs, h->xs, ko.rtol, ko.maxit, spi);
        else if (h->mixed)
            rc_p = cg_mixed_solve(s, n, h->rp, h->ci, h->Ks, h->Ks32, h->wK, h->wK32, h->vnull32, h->vscale, h->bs,
                                  h->xs, ko.rtol,
                                  h->par.pressure_delta > 0.0 ? h->par.pressure_delta : kPressureDelta, ko.maxit, 0,
                                  false, h->cg32, h->xlo, h->rhi, spi);
        else
            rc_p = cg_solve<double>(s, n, h->rp, h->ci, h->Ks, h->wK, h->bs, h->xs, ko.rtol, ko.maxit, 0, false,
                                    h->cg, spi);
        if (rc_p == OASIS_EHIP) return rc_p;
        sp.iters += spi.iters;
        sp.outer += spi.outer;
        sp.rel_res = spi.rel_res;
        note(spi.status);
        // 5. phi, p* += phi, normalisation
        const int gp = grid_for(n, kBlock);
        hipLaunchKernelGGL(k_phi_a, dim3(gp), dim3(kBlock), 0, s, n, h->xs, h->sK, st->phi, h->red);
        hipLaunchKernelGGL(k_phi_b, dim3(gp), dim3(kBlock), 0, s, n, h->red, gp, st->phi, st->p,
                           h->red + kMaxPartials);
        hipLaunchKernelGGL(k_phi_c, dim3(gp), dim3(kBlock), 0, s, n, h->red + kMaxPartials, gp, st->p);
        OASIS_TRY_LAUNCH();
    }
    OASIS_TRY_HIP(hipEventRecord(h->ev[3], s));
    // 6. velocity correction
    if (h->consistent) {
        P3 dP{}, UI{};
        for (int k = 0; k < D; ++k) {
            dP.p[k] = h->dP[k];
            UI.p[k] = x[k];
        }
        const int g8 = grid_for(n, kBlock / 8, 1 << 20);
        double *un[3] = {st->Un[0], st->Un[1], D > 2 ? st->Un[2] : nullptr};
        if (D == 3)
            hipLaunchKernelGGL((k_mass_rhs<3, 8>), dim3(g8), dim3(kBlock), 0, s, n, h->rp, h->ci, h->M, dP, UI,
                               st->phi, h->bc_index, bc_values, h->par.n_bc, h->par.dt, h->sM, h->bt[0], h->bt[1],
                               h->bt[2], un[0], un[1], un[2]);
        else
            hipLaunchKernelGGL((k_mass_rhs<2, 8>), dim3(g8), dim3(kBlock), 0, s, n, h->rp, h->ci, h->M, dP, UI,
                               st->phi, h->bc_index, bc_values, h->par.n_bc, h->par.dt, h->sM, h->bt[0], h->bt[1],
                               static_cast<double *>(nullptr), un[0], un[1], static_cast<double *>(nullptr));
        OASIS_TRY_LAUNCH();
        for (int k = 0; k < D; ++k) {
            SolveOut sm;
            const int rc = cg_solve<double>(s, n, h->rp, h->ci, h->Ms, h->wM, h->bt[k], un[k], h->par.rtol_u,
                                            o.maxit, 0, false, h->cgM, sm);
            if (rc == OASIS_EHIP) return rc;
            S.iters_m[k] = sm.iters;
            note(sm.status);
            hipLaunchKernelGGL(k_vscale, dim3(gvec(n)), dim3(kBlock), 0, s, n, un[k], h->sM, 2, un[k]);
            OASIS_TRY_LAUNCH();
        }
    } else {
        if (D == 3)
            launch_update<3, 8>(s, h, x, st->phi, bc_values, st->Un);
        else
            launch_update<2, 8>(s, h, x, st->phi, bc_values, st->Un);
        OASIS_TRY_LAUNCH();
    }
    OASIS_TRY_HIP(hipEventRecord(h->ev[4], s));
    // 7. passive scalars (eq:scalar_disc): the velocity's u_bar (still in
    // h->ubar, or formed here after an explicit-convection step), M/dt + D K/2
    // in place of B, no pressure gradient
    if (h->nsc > 0 && h->abe && h->assembly == OASIS_ASSEMBLE_ROWS) {
        if (D == 3)
            hipLaunchKernelGGL((k_ubar<3>), dim3(gvec(n)), dim3(kBlock), 0, s, n, U1, U2,
                               static_cast<const double *>(nullptr), h->ubar);
        else
            hipLaunchKernelGGL((k_ubar<2>), dim3(gvec(n)), dim3(kBlock), 0, s, n, U1, U2,
                               static_cast<const double *>(nullptr), h->ubar);
        OASIS_TRY_LAUNCH();
    }
    for (int a = 0; a < h->nsc; ++a) {
        int status = OASIS_OK;
        OASIS_TRY(scalar_solve(s, h, st, a, D, o, S, &status));
        note(status);
    }
    OASIS_TRY_HIP(hipEventRecord(h->ev[5], s));
    OASIS_TRY_HIP(hipEventSynchronize(h->ev[5]));
    float t[5];
    for (int k = 0; k < 5; ++k) OASIS_TRY_HIP(hipEventElapsedTime(&t[k], h->ev[k], h->ev[k + 1]));
    S.ms_assemble = t[0];
    S.ms_velocity = t[1];
    S.ms_pressure = t[2];
    S.ms_update = t[3];
    S.ms_scalars = t[4];
    S.ms_total = t[0] + t[1] + t[2] + t[3] + t[4];
    for (int k = 0; k < D; ++k) {
        S.iters_u[k] = su[k].iters;
        S.res_u[k] = su[k].rel_res;
        S.outer_u = std::max(S.outer_u, su[k].outer);
    }
    S.iters_p = sp.iters;
    S.res_p = sp.rel_res;
    S.outer_p = sp.outer;
    S.status = worst;
    return worst;
}

// ---------------------------------------------------------------------------
// stand-alone Krylov entry points

struct KrylovWs {
    double *val, *s, *w, *b, *x, *rhi;
    float *val32, *w32, *vnull32, *xlo;
    int *flag;
    short *ecol;        // ELL copy of the scaled matrix for the Krylov products
    unsigned short *pid;
    short *ptab;
    double *eval;       // (FP64 mode)
    float *eval32;      // (mixed mode)
    CGWork<double> cg;
    CGWork<float> cg32;
    BiWork<double> bi;
    BiWork<float> bi32;
    IRBufs ir;
    double *bt[3];
};

static void carve_krylov(Carver &c, int n, int nnz, int nrhs, bool mixed, KrylovWs &k) {
    std::memset(&k, 0, sizeof(k));
    k.val = c.take<double>(nnz);
    k.s = c.take<double>(n);
    k.w = c.take<double>(n);
    k.b = c.take<double>(n);
    k.x = c.take<double>(n);
    k.flag = c.take<int>(16);
    k.ecol = c.take<short>((size_t)n * kEll);
    k.pid = c.take<unsigned short>(n);
    k.ptab = c.take<short>((size_t)kMaxEllPatterns * kEll);
    if (mixed)
        k.eval32 = c.take<float>((size_t)n * kEll);
    else
        k.eval = c.take<double>((size_t)n * kEll);
    for (int q = 0; q < nrhs; ++q) k.bt[q] = c.take<double>(n);
    carve_cg<double>(c, n, k.cg);
    carve_bi<double>(c, n, nrhs, k.bi);
    if (mixed) {
        k.val32 = c.take<float>(nnz);
        k.w32 = c.take<float>(n);
        k.vnull32 = c.take<float>(n);
        k.xlo = c.take<float>(n);
        k.rhi = c.take<double>(n);
        carve_cg<float>(c, n, k.cg32);
        carve_bi<float>(c, n, nrhs, k.bi32);
        carve_ir(c, n, nrhs, k.ir);
    }
}

extern "C" int oasis_krylov_workspace_size(int32_t n, int32_t nnz, int32_t nrhs, const oasis_krylov_opts *opt,
                                           size_t *bytes) {
    if (n <= 0 || nnz <= 0 || nrhs < 1 || nrhs > 3 || !opt || !bytes) return OASIS_EINVAL;
    Carver c(nullptr, 0);
    KrylovWs k;
    carve_krylov(c, n, nnz, nrhs, opt->precision == OASIS_F32, k);
    *bytes = c.bytes();
    return OASIS_OK;
}

static void fill_stats(const SolveOut &o, int ell_storage, oasis_krylov_stats *st) {
    st->iters = o.iters;
    st->outer_iters = o.outer;
    st->status = o.status;
    st->restarts = o.replacements;
    st->rel_res = o.rel_res;
    st->kernel_ms = o.kernel_ms;
    st->kernel_count = o.kernel_count;
    st->ell_patterns = ell_storage;
}

static int check_opts(const oasis_krylov_opts *o) {
    if (!o || !(o->rtol > 0) || o->maxit < 0) return OASIS_EINVAL;
    if (o->precision != OASIS_F64 && o->precision != OASIS_F32) return OASIS_EINVAL;
    Tuning t;
    return Tuning::from(&o->tuning, &t);
}

// The stand-alone PCG on a workspace ws (the caller's, or the library's
// no-allocation scratch array with `dict` false: the offset dictionary is
// built on the host, which the no-allocation entry point must not do).
static int pcg_run(void *stream, const oasis_csr *A, const double *b, double *x, const oasis_krylov_opts *opt,
                   void *ws, size_t ws_bytes, oasis_krylov_stats *stats, bool dict) {
    OASIS_TRY(check_csr(A));
    OASIS_TRY(check_opts(opt));
    if (A->dtype != OASIS_F64 || !b || !x || !ws || !stats || !aligned(ws, 256)) return OASIS_EINVAL;
    const bool mixed = opt->precision == OASIS_F32;
    const int n = A->n, nnz = A->nnz;
    Carver c(ws, ws_bytes);
    KrylovWs k;
    carve_krylov(c, n, nnz, 1, mixed, k);
    if (!c.ok) return OASIS_EWORKSPACE;
    Tuning tun;
    (void)Tuning::from(&opt->tuning, &tun);
    if (!dict && tun.storage == OASIS_STORAGE_AUTO) tun.storage = OASIS_STORAGE_ELL;
    k.cg.tun = k.cg32.tun = tun;
    k.bi.tun = k.bi32.tun = tun;
    hipStream_t s = as_stream(stream);
    const double *val = static_cast<const double *>(A->val);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, s, 16, k.flag, 0);
    hipLaunchKernelGGL((k_diag<double>), dim3(gvec(n)), dim3(kBlock), 0, s, n, A->row_ptr, A->col_idx, val, k.b);
    hipLaunchKernelGGL(k_diag_vectors, dim3(gvec(n)), dim3(kBlock), 0, s, n, k.b, 0, k.s, k.w, k.w32, k.flag);
    hipLaunchKernelGGL(k_scale_matrix, dim3(gvec(n)), dim3(kBlock), 0, s, n, A->row_ptr, A->col_idx, val, k.s,
                       kScaleSym, k.val, k.val32);
    hipLaunchKernelGGL(k_vscale, dim3(gvec(n)), dim3(kBlock), 0, s, n, b, k.s, 2, k.b);
    hipLaunchKernelGGL(k_vscale, dim3(gvec(n)), dim3(kBlock), 0, s, n, x, k.s, 1, k.x);
    OASIS_TRY_LAUNCH();
    int fl = 0;
    OASIS_TRY_HIP(hipMemcpyAsync(&fl, k.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    if (fl) return OASIS_EINVAL;
    int ell_storage = 0;
    {
        EllCols cols;
        OASIS_TRY(ell_setup(s, n, A->row_ptr, A->col_idx, k.val, k.ecol, k.pid, k.ptab, k.eval, k.eval32,
                            k.flag + 8, tun, &cols, &ell_storage));
        if (cols.any() && mixed) {
            k.cg32.cols = cols;
            k.cg32.eval = k.eval32;
        } else if (cols.any()) {
            k.cg.cols = cols;
            k.cg.eval = k.eval;
        }
    }
    const KOpts ko = kopts(opt);
    SolveOut so;
    int rc;
    if (mixed) {
        const float *vn = nullptr;
        double vscale = 0.0;
        if (opt->flags & OASIS_KRYLOV_NULLSPACE_CONST) {
            OASIS_TRY(unit_vector_f32(s, n, k.s, k.ir.part, k.vnull32, &vscale));
            vn = k.vnull32;
        }
        rc = cg_mixed_solve(s, n, A->row_ptr, A->col_idx, k.val, k.val32, k.w, k.w32, vn, vscale, k.b, k.x, ko.rtol,
                            reliable_delta(opt->inner_rtol), ko.maxit, ko.check_every, ko.time, k.cg32, k.xlo,
                            k.rhi, so);
    }
    else
        rc = cg_solve<double>(s, n, A->row_ptr, A->col_idx, k.val, k.w, k.b, k.x, ko.rtol, ko.maxit, ko.check_every,
                              ko.time, k.cg, so);
    if (rc == OASIS_EHIP) return rc;
    hipLaunchKernelGGL(k_vscale, dim3(gvec(n)), dim3(kBlock), 0, s, n, k.x, k.s, 2, x);
    OASIS_TRY_LAUNCH();
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    fill_stats(so, ell_storage, stats);
    return rc;
}

extern "C" int oasis_pcg(void *stream, const oasis_csr *A, const double *b, double *x, const oasis_krylov_opts *opt,
                         void *ws, size_t ws_bytes, oasis_krylov_stats *stats) {
    return pcg_run(stream, A, b, x, opt, ws, ws_bytes, stats, true);
}

// ---------------------------------------------------------------------------
// PCG without any allocation: the workspace is a file-scope device array.
// Host code never passes the array's name to a kernel or a copy: each
// device's copy of the array has its own address, obtained once per device
// with hipGetSymbolAddress and kept in scratch_addr.

constexpr size_t kScratchBytes = OASIS_PCG_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex scratch_mu;
static void *scratch_addr[kMaxDevices] = {};

// The address of the current device's scratch array (looked up on the first
// call on that device).
static int scratch_ptr(void **out) {
    int dev = 0;
    OASIS_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return OASIS_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return OASIS_EHIP;
        }
        scratch_addr[dev] = p;
    }
    *out = scratch_addr[dev];
    return OASIS_OK;
}

extern "C" int oasis_pcg_noalloc(void *stream, const oasis_csr *A, const double *b, double *x,
                                 const oasis_krylov_opts *opt, oasis_krylov_stats *stats) {
    OASIS_TRY(check_csr(A));
    OASIS_TRY(check_opts(opt));
    if (opt->flags & OASIS_KRYLOV_TIME) return OASIS_EINVAL;     // the timing mode creates events
    size_t need = 0;
    OASIS_TRY(oasis_krylov_workspace_size(A->n, A->nnz, 1, opt, &need));
    if (need > kScratchBytes) return OASIS_EUNSUPPORTED;
    void *ws = nullptr;
    OASIS_TRY(scratch_ptr(&ws));
    return pcg_run(stream, A, b, x, opt, ws, kScratchBytes, stats, false);
}

extern "C" int oasis_bicgstab(void *stream, const oasis_csr *A, int32_t nrhs, const double *b, double *x,
                              const oasis_krylov_opts *opt, void *ws, size_t ws_bytes, oasis_krylov_stats *stats) {
    OASIS_TRY(check_csr(A));
    OASIS_TRY(check_opts(opt));
    if (A->dtype != OASIS_F64 || nrhs < 1 || nrhs > 3 || !b || !x || !ws || !stats || !aligned(ws, 256))
        return OASIS_EINVAL;
    const bool mixed = opt->precision == OASIS_F32;
    const int n = A->n, nnz = A->nnz;
    Carver c(ws, ws_bytes);
    KrylovWs k;
    carve_krylov(c, n, nnz, nrhs, mixed, k);
    if (!c.ok) return OASIS_EWORKSPACE;
    Tuning tun;
    (void)Tuning::from(&opt->tuning, &tun);
    k.cg.tun = k.cg32.tun = tun;
    k.bi.tun = k.bi32.tun = tun;
    hipStream_t s = as_stream(stream);
    const double *val = static_cast<const double *>(A->val);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, s, 16, k.flag, 0);
    hipLaunchKernelGGL((k_diag<double>), dim3(gvec(n)), dim3(kBlock), 0, s, n, A->row_ptr, A->col_idx, val, k.b);
    hipLaunchKernelGGL(k_diag_vectors, dim3(gvec(n)), dim3(kBlock), 0, s, n, k.b, 1, k.s, k.w, k.w32, k.flag);
    // right Jacobi: BiCGStab on A D^{-1} y = b, x = D^{-1} y
    hipLaunchKernelGGL(k_scale_matrix, dim3(gvec(n)), dim3(kBlock), 0, s, n, A->row_ptr, A->col_idx, val, k.s,
                       kScaleCol, k.val, k.val32);
    OASIS_TRY_LAUNCH();
    int fl = 0;
    OASIS_TRY_HIP(hipMemcpyAsync(&fl, k.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    if (fl) return OASIS_EINVAL;     // x untouched
    int ell_storage = 0;
    {
        EllCols cols;
        OASIS_TRY(ell_setup(s, n, A->row_ptr, A->col_idx, k.val, k.ecol, k.pid, k.ptab, k.eval, k.eval32,
                            k.flag + 8, tun, &cols, &ell_storage));
        if (cols.any() && mixed) {
            k.bi32.cols = cols;
            k.bi32.eval = k.eval32;
        } else if (cols.any()) {
            k.bi.cols = cols;
            k.bi.eval = k.eval;
        }
    }
    double *xs[3] = {nullptr, nullptr, nullptr};
    for (int q = 0; q < nrhs; ++q) {
        OASIS_TRY_HIP(hipMemcpyAsync(k.bt[q], b + (size_t)q * n, (size_t)n * sizeof(double),
                                     hipMemcpyDeviceToDevice, s));
        xs[q] = x + (size_t)q * n;
    }
    hipLaunchKernelGGL(k_scale3, dim3(gvec(n)), dim3(kBlock), 0, s, n, k.s, 1, xs[0], xs[1], xs[2]);
    OASIS_TRY_LAUNCH();
    const KOpts ko = kopts(opt);
    SolveOut so[3];
    int rc;
    if (mixed)
        rc = ir_bicgstab(s, n, nrhs, A->row_ptr, A->col_idx, k.val, k.val32, k.w, k.w32, k.bt, xs, ko, k.bi32, k.ir,
                         so);
    else
        rc = bicgstab_solve<double>(s, n, nrhs, A->row_ptr, A->col_idx, k.val, k.w, k.bt, xs, ko.rtol, ko.maxit,
                                    ko.check_every, ko.time, k.bi, so);
    if (rc == OASIS_EHIP) return rc;
    hipLaunchKernelGGL(k_scale3, dim3(gvec(n)), dim3(kBlock), 0, s, n, k.s, 2, xs[0], xs[1], xs[2]);
    OASIS_TRY_LAUNCH();
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < nrhs; ++q) fill_stats(so[q], ell_storage, stats + q);
    return rc;
}
