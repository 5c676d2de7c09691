// Smoothed-aggregation AMG on the device: the V(1,1) cycle as the
// preconditioner of CG for the pressure correction.  The paper's channel
// runs precondition the pressure solve with algebraic multigrid (Sec. 6.2,
// channel performance paragraph); the hierarchy is built on the host once
// per matrix (amg_setup.hip) and uploaded into a caller workspace.
//
// Cycle on level l (b: right-hand side, w_i = omega_l / a_ii):
//   pre      t = b - A (w .* b)          (one Jacobi sweep from x = 0, then
//                                          its residual; x = w .* b is never
//                                          stored)
//   restrict b_{l+1} = P^T t
//   coarse   x_L = A_L^-1 b_L            (dense inverse)
//   prolong  t = w .* b + P x_{l+1}
//   post     x = t + w .* (b - A t)
// Level 0 runs on the ELL copy of the matrix (16-bit offsets, dictionary on
// structured meshes) when it fits, CSR otherwise; coarser levels on CSR.
// The cycle is in FP64 or FP32 (values and vectors); CG stays in FP64 and
// its dot products too, so the FP32 cycle is an inner approximation only.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <type_traits>

#include "amg.hpp"

namespace oasis {

namespace {

__device__ __forceinline__ bool stopped(const int *flag) {
    if (!flag) return false;
    __shared__ int v;
    if (threadIdx.x == 0) v = __atomic_load_n(flag, __ATOMIC_RELAXED);
    __syncthreads();
    const int r = v;
    __syncthreads();
    return r != 0;
}

// CSR row shapes of the coarse-level kernels: L lanes x 4 unrolled entries
// per row, L chosen per matrix from its mean row length (upload time), so
// that short rows (prolongator: ~5) do not issue 16 clamped loads each.
template <int L>
using AmgCfg = RowCfg<L, 4, 1>;

template <class F>
int with_lanes(int lanes, F &&f) {
    switch (lanes) {
        case 2: return f(AmgCfg<2>{});
        case 8: return f(AmgCfg<8>{});
        case 16: return f(AmgCfg<16>{});
        case 32: return f(AmgCfg<32>{});
        case 64: return f(AmgCfg<64>{});
        default: return f(AmgCfg<4>{});
    }
}

// y = w .* b: the one operand the pre-smoothing residual gathers
template <typename T, typename TB>
__global__ __launch_bounds__(kBlock) void k_amg_scale(int n, const T *__restrict__ wd, const TB *__restrict__ b,
                                                      T *__restrict__ y, const int *flag) {
    if (stopped(flag)) return;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = wd[i] * static_cast<T>(b[i]);
}

// pre-smoothing residual on the ELL copy: t = b - A y (straight-line row
// loop: the next row's offsets, values and b are fetched while this row's
// gathers are in flight)
template <typename T, typename TB, bool DICT, typename TE = T>
__global__ __launch_bounds__(kBlock) void k_amg_pre_ell(int n, EllCols cols, const TE *__restrict__ e,
                                                        const T *__restrict__ y, const TB *__restrict__ b,
                                                        T *__restrict__ t, const int *flag) {
    if (stopped(flag)) return;
    auto load = [&](int c) { return y[c]; };
    auto add = [&](const T &g, T v, T(&a)[1]) { a[0] += v * g; };
    auto own = [&](long long r) { return b[r]; };
    auto fin = [&](int row, int lane, T(&a)[1], const TB &o) {
        if (lane == 0) t[row] = static_cast<T>(o) - a[0];
    };
    ell_rows_pipe<T, 1, 2, DICT, T, TB>(n, cols, e, load, add, own, fin);
}

// pre-smoothing residual, CSR
template <typename T, typename TB, class C>
__global__ __launch_bounds__(kBlock) void k_amg_pre_csr(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                        const T *__restrict__ val, const T *__restrict__ y,
                                                        const TB *__restrict__ b, T *__restrict__ t,
                                                        const int *flag) {
    if (stopped(flag)) return;
    csr_rows<T, 1, C>(
        n, rp, ci, val,
        [&](int, int c, T v, bool ok, T(&a)[1]) {
            const T g = v * y[c];
            a[0] += ok ? g : T(0);
        },
        [&](int row, int lane, T(&a)[1]) {
            if (lane == 0) t[row] = static_cast<T>(b[row]) - a[0];
        });
}

// restriction b_c = R t (R = P^T as CSR), and y_c = w_c .* b_c when the
// next level smooths (wdc non-null)
template <typename T, class C>
__global__ __launch_bounds__(kBlock) void k_amg_restrict(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                         const T *__restrict__ val, const T *__restrict__ x,
                                                         T *__restrict__ bc, const T *__restrict__ wdc,
                                                         T *__restrict__ yc, const int *flag) {
    if (stopped(flag)) return;
    csr_rows<T, 1, C>(
        n, rp, ci, val,
        [&](int, int c, T v, bool ok, T(&a)[1]) {
            const T g = v * x[c];
            a[0] += ok ? g : T(0);
        },
        [&](int row, int lane, T(&a)[1]) {
            if (lane == 0) {
                bc[row] = a[0];
                if (wdc) yc[row] = wdc[row] * a[0];
            }
        });
}

// prolongation and correction: t = y + P xc (y = w .* b, the pre-smoothed
// iterate)
template <typename T, class C>
__global__ __launch_bounds__(kBlock) void k_amg_prolong(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                        const T *__restrict__ val, const T *__restrict__ xc,
                                                        const T *__restrict__ y, T *__restrict__ t, const int *flag) {
    if (stopped(flag)) return;
    csr_rows<T, 1, C>(
        n, rp, ci, val,
        [&](int, int c, T v, bool ok, T(&a)[1]) {
            const T g = v * xc[c];
            a[0] += ok ? g : T(0);
        },
        [&](int row, int lane, T(&a)[1]) {
            if (lane == 0) t[row] = y[row] + a[0];
        });
}

// post-smoothing x = t + w .* (b - A t), written as TO at out[i * os];
// with acc: per-thread partials (b.x, sum wgt b^2)
template <typename T, typename TB, typename TO>
__device__ __forceinline__ void amg_post_finish(int row, T ti, T wi, TB braw, T sum, TO *out, int os,
                                                const double *wgt, double *acc) {
    const T bi = static_cast<T>(braw);
    const T x = ti + wi * (bi - sum);
    out[static_cast<long long>(row) * os] = static_cast<TO>(x);
    if (wgt) {
        const double bd = static_cast<double>(braw);
        acc[0] += bd * static_cast<double>(x);
        acc[1] += wgt[row] * bd * bd;
    }
}

template <typename T, typename TB>
struct PostOwn {
    T t, w;
    TB b;
};

template <typename T, typename TB, typename TO, bool DICT, typename TE = T>
__global__ __launch_bounds__(kBlock) void k_amg_post_ell(int n, EllCols cols, const TE *__restrict__ e,
                                                         const T *__restrict__ wd, const TB *__restrict__ b,
                                                         const T *__restrict__ t, TO *__restrict__ out, int os,
                                                         const double *__restrict__ wgt, double *part,
                                                         const int *flag) {
    __shared__ double lds[2 * kBlock / kWave];
    if (stopped(flag)) return;
    double acc[2] = {0.0, 0.0};
    const double *w2 = part ? wgt : nullptr;
    using O = PostOwn<T, TB>;
    auto load = [&](int c) { return t[c]; };
    auto add = [&](const T &g, T v, T(&a)[1]) { a[0] += v * g; };
    auto own = [&](long long r) { return O{t[r], wd[r], b[r]}; };
    auto fin = [&](int row, int lane, T(&a)[1], const O &o) {
        if (lane == 0) amg_post_finish<T, TB, TO>(row, o.t, o.w, o.b, a[0], out, os, w2, acc);
    };
    ell_rows_pipe<T, 1, 2, DICT, T, O>(n, cols, e, load, add, own, fin);
    if (part) write_partials<2>(acc, part, lds);
}

template <typename T, typename TB, typename TO, class C>
__global__ __launch_bounds__(kBlock) void k_amg_post_csr(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                         const T *__restrict__ val, const T *__restrict__ wd,
                                                         const TB *__restrict__ b, const T *__restrict__ t,
                                                         TO *__restrict__ out, int os, const double *__restrict__ wgt,
                                                         double *part, const int *flag) {
    __shared__ double lds[2 * kBlock / kWave];
    if (stopped(flag)) return;
    double acc[2] = {0.0, 0.0};
    const double *w2 = part ? wgt : nullptr;
    csr_rows<T, 1, C>(
        n, rp, ci, val,
        [&](int, int c, T v, bool ok, T(&a)[1]) {
            const T g = v * t[c];
            a[0] += ok ? g : T(0);
        },
        [&](int row, int lane, T(&a)[1]) {
            if (lane == 0) amg_post_finish<T, TB, TO>(row, t[row], wd[row], b[row], a[0], out, os, w2, acc);
        });
    if (part) write_partials<2>(acc, part, lds);
}

// coarsest level: x = C b with the dense inverse C (row-major); one wave
// per row; with part, partials (b.x, sum wgt b^2) as the post kernel
template <typename T, typename TB, typename TO>
__global__ __launch_bounds__(kBlock) void k_amg_dense(int nc, const T *__restrict__ cinv, const TB *__restrict__ b,
                                                      TO *__restrict__ out, int os, const double *__restrict__ wgt,
                                                      double *part, const int *flag) {
    __shared__ double lds[2 * kBlock / kWave];
    if (stopped(flag)) return;
    const int lane = threadIdx.x & (kWave - 1);
    double acc[2] = {0.0, 0.0};
    for (int row = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; row < nc;
         row += gridDim.x * (kBlock / kWave)) {
        double s = 0.0;
        for (int j = lane; j < nc; j += kWave)
            s += static_cast<double>(cinv[static_cast<long long>(row) * nc + j]) * static_cast<double>(b[j]);
        s = wave_sum(s);
        if (lane == 0) {
            out[static_cast<long long>(row) * os] = static_cast<TO>(static_cast<T>(s));
            if (part && wgt) {
                const double bd = static_cast<double>(b[row]);
                acc[0] += bd * static_cast<double>(static_cast<T>(s));
                acc[1] += wgt[row] * bd * bd;
            }
        }
    }
    if (part) write_partials<2>(acc, part, lds);
}

// CG update: alpha = (r.z) / (p.q), x += alpha p, r -= alpha q (p from the
// (z, p) pairs written by the product kernel), and the cycle's first
// operand y0 = w0 .* r in the cycle's precision
template <typename T>
__global__ __launch_bounds__(kBlock) void k_apcg_update(int n, const RP<double> *__restrict__ nxt,
                                                        const double *__restrict__ q, double *__restrict__ x,
                                                        double *__restrict__ r, const T *__restrict__ wd0,
                                                        T *__restrict__ y0, const double *partIn, int nIn,
                                                        CGState *st, int it) {
    __shared__ double lds[2 * kBlock / kWave];
    if (stopped(&st->flag)) return;
    double v[2];
    read_partials<2>(partIn, nIn, v, lds);
    const double pq = v[0];
    if (!(pq > 0.0) || !finite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->flag = finite(pq) ? 2 : 3;
            st->it_done = it;
        }
        return;
    }
    const double a = st->rr[it & 1] / pq;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        x[i] += a * nxt[i].p;
        const double ri = r[i] - a * q[i];
        r[i] = ri;
        if (y0) y0[i] = wd0[i] * static_cast<T>(ri);
    }
}

// The FP32 form of k_apcg_update: alpha in FP64 from the partials, the
// iterate x += alpha p in FP64, the recursive residual r -= alpha q and the
// cycle's y0 = w0 .* r in FP32.
__global__ __launch_bounds__(kBlock) void k_apcg_update32(int n, const RP<float> *__restrict__ nxt,
                                                          const float *__restrict__ q, double *__restrict__ x,
                                                          float *__restrict__ r, const float *__restrict__ wd0,
                                                          float *__restrict__ y0, const double *partIn, int nIn,
                                                          CGState *st, int it) {
    __shared__ double lds[2 * kBlock / kWave];
    if (stopped(&st->flag)) return;
    double v[2];
    read_partials<2>(partIn, nIn, v, lds);
    const double pq = v[0];
    if (!(pq > 0.0) || !finite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->flag = finite(pq) ? 2 : 3;
            st->it_done = it;
        }
        return;
    }
    const double a = st->rr[it & 1] / pq;
    const float af = static_cast<float>(a);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        x[i] += a * static_cast<double>(nxt[i].p);
        const float ri = r[i] - af * q[i];
        r[i] = ri;
        if (y0) y0[i] = wd0[i] * ri;
    }
}

__global__ __launch_bounds__(kBlock) void k_amg_to_f32(int n, const double *__restrict__ a, float *__restrict__ b) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        b[i] = static_cast<float>(a[i]);
}

template <class C>
int csr_grid(int n) { return grid_for(n, rows_per_block<C>(), 1 << 20); }

// reps launches of `launch` back to back between two events on s
template <class Launch>
int time_repeats(hipStream_t s, int reps, Launch launch, SolveOut &out) {
    hipEvent_t e[2] = {nullptr, nullptr};
    int rc = OASIS_OK;
    for (auto &v : e)
        if (rc == OASIS_OK && hipEventCreate(&v) != hipSuccess) rc = OASIS_EHIP;
    if (rc == OASIS_OK && hipEventRecord(e[0], s) != hipSuccess) rc = OASIS_EHIP;
    for (int k = 0; k < reps && rc == OASIS_OK; ++k) rc = launch();
    float ms = 0.f;
    if (rc == OASIS_OK && (hipEventRecord(e[1], s) != hipSuccess || hipEventSynchronize(e[1]) != hipSuccess ||
                           hipEventElapsedTime(&ms, e[0], e[1]) != hipSuccess))
        rc = OASIS_EHIP;
    for (auto &v : e)
        if (v) (void)hipEventDestroy(v);
    if (rc == OASIS_OK) {
        out.kernel_ms = ms;
        out.kernel_count = reps;
    }
    return rc;
}
int ell_grid(int n, int cap) { return grid_for(n, kBlock / 2, cap); }

}  // namespace

template <typename T, typename TB, typename TO>
int amg_vcycle(hipStream_t s, const AmgCycle<T> &c, const TB *r, bool y0_ready, TO *z, int zs,
               const double *wgt, double *part, int *gpost, const int *flag, int grid_cap) {
    const int L = c.nlev;
    const bool ell0 = c.cols.any() && c.e;
    const bool dict = c.cols.pid != nullptr;
    if (L == 1) {
        const int g = std::min(grid_for(c.nc, kBlock / kWave, 1 << 20), part ? grid_cap : 1 << 20);
        hipLaunchKernelGGL((k_amg_dense<T, TB, TO>), dim3(g), dim3(kBlock), 0, s, c.nc, c.cinv, r, z, zs,
                           wgt, part, flag);
        OASIS_TRY_LAUNCH();
        if (gpost) *gpost = g;
        return OASIS_OK;
    }
    if (!y0_ready) {
        const AmgDevLevel<T> &v = c.lv[0];
        hipLaunchKernelGGL((k_amg_scale<T, TB>), dim3(grid_for(v.n, kBlock, 8192)), dim3(kBlock), 0, s, v.n,
                           v.wd, r, v.y, flag);
        OASIS_TRY_LAUNCH();
    }
    // down
    for (int l = 0; l + 1 < L; ++l) {
        const AmgDevLevel<T> &v = c.lv[l];
        if (l == 0 && ell0) {
            const int g = ell_grid(v.n, grid_cap);   // several rows per lane group: the row loop prefetches
            bool done = false;
            if constexpr (std::is_same<T, float>::value) {
                if (c.e16) {   // FP16-stored level-0 values
                    if (dict)
                        hipLaunchKernelGGL((k_amg_pre_ell<T, TB, true, _Float16>), dim3(g), dim3(kBlock), 0, s, v.n,
                                           c.cols, c.e16, v.y, r, v.t, flag);
                    else
                        hipLaunchKernelGGL((k_amg_pre_ell<T, TB, false, _Float16>), dim3(g), dim3(kBlock), 0, s,
                                           v.n, c.cols, c.e16, v.y, r, v.t, flag);
                    done = true;
                }
            }
            if (!done) {
                if (dict)
                    hipLaunchKernelGGL((k_amg_pre_ell<T, TB, true>), dim3(g), dim3(kBlock), 0, s, v.n, c.cols, c.e,
                                       v.y, r, v.t, flag);
                else
                    hipLaunchKernelGGL((k_amg_pre_ell<T, TB, false>), dim3(g), dim3(kBlock), 0, s, v.n, c.cols,
                                       c.e, v.y, r, v.t, flag);
            }
            OASIS_TRY_LAUNCH();
        } else {
            OASIS_TRY(with_lanes(v.alanes, [&](auto cfg) -> int {
                using C = decltype(cfg);
                if (l == 0)
                    hipLaunchKernelGGL((k_amg_pre_csr<T, TB, C>), dim3(csr_grid<C>(v.n)), dim3(kBlock), 0, s,
                                       v.n, v.rp, v.ci, v.val, v.y, r, v.t, flag);
                else
                    hipLaunchKernelGGL((k_amg_pre_csr<T, T, C>), dim3(csr_grid<C>(v.n)), dim3(kBlock), 0, s, v.n,
                                       v.rp, v.ci, v.val, v.y, v.b, v.t, flag);
                OASIS_TRY_LAUNCH();
                return OASIS_OK;
            }));
        }
        const AmgDevLevel<T> &nx = c.lv[l + 1];
        const bool smooth_next = l + 2 < L;
        OASIS_TRY(with_lanes(v.rlanes, [&](auto cfg) -> int {
            using C = decltype(cfg);
            hipLaunchKernelGGL((k_amg_restrict<T, C>), dim3(csr_grid<C>(nx.n)), dim3(kBlock), 0, s, nx.n, v.rrp,
                               v.rci, v.rval, v.t, nx.b, smooth_next ? nx.wd : nullptr,
                               smooth_next ? nx.y : nullptr, flag);
            OASIS_TRY_LAUNCH();
            return OASIS_OK;
        }));
    }
    // coarsest
    {
        const AmgDevLevel<T> &v = c.lv[L - 1];
        hipLaunchKernelGGL((k_amg_dense<T, T, T>), dim3(grid_for(c.nc, kBlock / kWave, 1 << 20)), dim3(kBlock), 0,
                           s, c.nc, c.cinv, v.b, v.x, 1, static_cast<const double *>(nullptr),
                           static_cast<double *>(nullptr), flag);
        OASIS_TRY_LAUNCH();
    }
    // up
    for (int l = L - 2; l >= 0; --l) {
        const AmgDevLevel<T> &v = c.lv[l];
        const AmgDevLevel<T> &nx = c.lv[l + 1];
        OASIS_TRY(with_lanes(v.planes, [&](auto cfg) -> int {
            using C = decltype(cfg);
            hipLaunchKernelGGL((k_amg_prolong<T, C>), dim3(csr_grid<C>(v.n)), dim3(kBlock), 0, s, v.n, v.prp, v.pci,
                               v.pval, nx.x, v.y, v.t, flag);
            OASIS_TRY_LAUNCH();
            return OASIS_OK;
        }));
        if (l == 0 && ell0) {
            const int g = ell_grid(v.n, part ? grid_cap : 1 << 20);
            bool done = false;
            if constexpr (std::is_same<T, float>::value) {
                if (c.e16) {
                    if (dict)
                        hipLaunchKernelGGL((k_amg_post_ell<T, TB, TO, true, _Float16>), dim3(g), dim3(kBlock), 0, s,
                                           v.n, c.cols, c.e16, v.wd, r, v.t, z, zs, wgt, part, flag);
                    else
                        hipLaunchKernelGGL((k_amg_post_ell<T, TB, TO, false, _Float16>), dim3(g), dim3(kBlock), 0,
                                           s, v.n, c.cols, c.e16, v.wd, r, v.t, z, zs, wgt, part, flag);
                    done = true;
                }
            }
            if (!done) {
                if (dict)
                    hipLaunchKernelGGL((k_amg_post_ell<T, TB, TO, true>), dim3(g), dim3(kBlock), 0, s, v.n,
                                       c.cols, c.e, v.wd, r, v.t, z, zs, wgt, part, flag);
                else
                    hipLaunchKernelGGL((k_amg_post_ell<T, TB, TO, false>), dim3(g), dim3(kBlock), 0, s, v.n,
                                       c.cols, c.e, v.wd, r, v.t, z, zs, wgt, part, flag);
            }
            OASIS_TRY_LAUNCH();
            if (gpost) *gpost = g;
        } else {
            OASIS_TRY(with_lanes(v.alanes, [&](auto cfg) -> int {
                using C = decltype(cfg);
                if (l == 0) {
                    const int g = std::min(csr_grid<C>(v.n), part ? grid_cap : 1 << 20);
                    hipLaunchKernelGGL((k_amg_post_csr<T, TB, TO, C>), dim3(g), dim3(kBlock), 0, s, v.n,
                                       v.rp, v.ci, v.val, v.wd, r, v.t, z, zs, wgt, part, flag);
                    if (gpost) *gpost = g;
                } else {
                    hipLaunchKernelGGL((k_amg_post_csr<T, T, T, C>), dim3(csr_grid<C>(v.n)), dim3(kBlock), 0, s, v.n,
                                       v.rp, v.ci, v.val, v.wd, v.b, v.t, v.x, 1,
                                       static_cast<const double *>(nullptr), static_cast<double *>(nullptr), flag);
                }
                OASIS_TRY_LAUNCH();
                return OASIS_OK;
            }));
        }
    }
    return OASIS_OK;
}

// Iterations to launch before the next poll: from the observed rate of
// log(wrr) per iteration, aiming just before convergence, within [1, 32]
// (an AMG iteration costs many kernels, so a late poll wastes more than an
// early one); 2 before any rate is known.
struct AmgPlan {
    int fixed;
    double rate = 0.0, w0 = 0.0;
    int it0 = 0, next = 2;
    // first: the first launch's size when the caller knows roughly how many
    // iterations a solve takes (0: 2)
    AmgPlan(int every, int first) : fixed(every) {
        if (fixed > 0)
            next = fixed;
        else if (first > 0)
            next = first;
    }
    void restart(double wrr, int it) {
        w0 = wrr;
        it0 = it;
        if (fixed <= 0) next = 2;
    }
    void observe(double wrr, int it_last, double target) {
        if (fixed > 0) return;
        if (it_last > it0 && wrr > 0.0 && w0 > 0.0) {
            const double r = std::log(wrr / w0) / (it_last - it0);
            if (r < 0.0) rate = r;
        }
        if (rate < 0.0 && wrr > 0.0 && target > 0.0) {
            const double k = std::log(target / wrr) / rate;
            next = static_cast<int>(std::min(32.0, std::max(1.0, std::floor(k))));
        } else {
            next = 2;
        }
    }
};

// The convergence test that the next product kernel would make, run at the
// end of a launched chunk so that the poll sees it at once: from the
// partials (r.z, sum wgt r^2) of the cycle's last kernel, flag 1 (or 3 on
// a non-finite value) at iteration `it`, and the residual recorded for the
// host's plan.  A flag already up is left alone.
__global__ __launch_bounds__(kBlock) void k_apcg_test(const double *part, int np, CGState *st, int it) {
    __shared__ double lds[2 * kBlock / kWave];
    if (stopped(&st->flag)) return;
    double v[2];
    read_partials<2>(part, np, v, lds);
    if (threadIdx.x == 0) {
        const double wrr = v[1];
        if (!finite(wrr) || !finite(v[0])) {
            st->flag = 3;
            st->it_done = it;
        } else if (wrr <= st->tol2) {
            st->flag = 1;
            st->it_done = it;
            st->wrr = wrr;
        } else {
            st->wrr_it = wrr;
            st->it_last = it;
        }
    }
}

template <typename T>
int amg_pcg_solve(hipStream_t s, int n, const int *rp, const int *ci, const double *val, const double *e64,
                  const AmgCycle<T> &c, const double *wgt, const double *b, double *x, double rtol, int maxit,
                  int check_every, bool time_kernel, double *r, CGWork<double> &w, SolveOut &out, int first_chunk) {
    out = SolveOut();
    const int cap = w.tun.grid_cap;
    const EllCols cols = (c.cols.any() && e64) ? c.cols : EllCols{};
    double *pv = w.partB;           // partials of the cycle's last kernel: (r.z, sum wgt r^2)
    double *pq = w.partA;           // partials of the product kernel: (p.q, 0)
    int gpost = 0, g1 = 0;
    auto zslot = [&](int at) { return reinterpret_cast<double *>(w.pair[at & 1]); };   // z in the pair's r
    auto start = [&](int mode, int at) -> int {
        OASIS_TRY(cg_residual_state(s, cap, n, rp, ci, val, cols, wgt, b, x, r, 1, pv, w.st, rtol * rtol,
                                    mode));
        return OASIS_OK;
    };
    const bool smooth0 = c.nlev > 1;
    // y0 = w0 .* r comes from the update kernel inside the loop, from the
    // cycle's own scaling kernel after an explicit residual
    auto precondition = [&](int at, bool y0_ready) -> int {
        return amg_vcycle<T>(s, c, r, y0_ready, zslot(at), 2, wgt, pv, &gpost, &w.st->flag, cap);
    };
    // The start residual is not read back: the first product kernel tests
    // it (converged, non-finite) like any other, and the first poll brings
    // its norms with the state.
    OASIS_TRY(start(0, 0));
    OASIS_TRY(precondition(0, false));
    CGState h;
    double wbb = 0.0, tol2 = 0.0;
    bool first = true;
    auto rel = [&](double wrr) { return wbb > 0.0 ? std::sqrt(wrr / wbb) : std::sqrt(wrr); };
    AmgPlan plan(check_every, first_chunk);
    int it = 0, restart_at = 0, rc = OASIS_OK;
    auto iterate = [&](int itj) -> int {
        OASIS_TRY(cg_product_launch(s, cap, n, rp, ci, val, cols, e64, w.pair[itj & 1], w.pair[(itj + 1) & 1],
                                    w.q, pv, gpost, 2, w.st, itj, itj == restart_at ? 1 : 0, pq, &g1));
        hipLaunchKernelGGL((k_apcg_update<T>), dim3(grid_for(n, kBlock, kMaxPartials)), dim3(kBlock), 0, s, n,
                           w.pair[(itj + 1) & 1], w.q, x, r, smooth0 ? c.lv[0].wd : nullptr,
                           smooth0 ? c.lv[0].y : nullptr, pq, g1, w.st, itj);
        OASIS_TRY_LAUNCH();
        return precondition(itj + 1, smooth0);
    };
    while (true) {
        const int m = std::min(plan.next, maxit - it);
        for (int j = 0; j < m; ++j) OASIS_TRY(iterate(it + j));
        it += m;
        if (m > 0) {
            hipLaunchKernelGGL(k_apcg_test, dim3(1), dim3(kBlock), 0, s, pv, gpost, w.st, it);
            OASIS_TRY_LAUNCH();
        }
        OASIS_TRY(read_state(s, w.stage, w.st, &h, sizeof(h)));
        if (first) {
            first = false;
            wbb = h.wbb;
            tol2 = h.tol2;
            if (h.flag == 0) plan.restart(h.wrr, 0);   // wrr: still the start residual's
        }
        if (h.flag == 0 && it < maxit) {
            plan.observe(h.wrr_it, h.it_last, tol2);
            continue;
        }
        if (h.flag == 2 || h.flag == 3) {
            out.iters = h.it_done;
            out.status = rc = h.flag == 2 ? OASIS_EBREAKDOWN : OASIS_ENAN;
            out.rel_res = NAN;
            break;
        }
        // converged candidate (or maxit): confirm on the true residual
        const int at = h.flag == 0 ? it : h.it_done;
        OASIS_TRY(start(1, at));
        OASIS_TRY(read_state(s, w.stage, w.st, &h, sizeof(h)));
        out.rel_res = rel(h.wrr);
        if (!std::isfinite(h.wrr)) {
            out.iters = at;
            out.status = rc = OASIS_ENAN;
            break;
        }
        if (h.wrr <= tol2) {
            out.iters = at;
            out.status = rc = OASIS_OK;
            break;
        }
        if (at >= maxit) {
            out.iters = at;
            out.status = rc = OASIS_ENOTCONV;
            if (time_kernel) {
                // repeat the cycle on the final residual maxit times (it
                // reads r and writes only the z slot, so x is unchanged)
                OASIS_TRY(time_repeats(s, maxit, [&] {
                    return amg_vcycle<T>(s, c, r, false, zslot(at), 2, wgt, pv, &gpost, nullptr, cap);
                }, out));
            }
            break;
        }
        // continue from the explicit residual with a fresh direction
        out.replacements += 1;
        OASIS_TRY(precondition(at, false));
        it = at;
        restart_at = at;
        plan.restart(h.wrr, at);
    }
    return rc;
}

int amg_pcg_mixed(hipStream_t s, int n, const int *rp, const int *ci, const double *val, const double *e64,
                  const AmgCycle<float> &c, const double *wgt, const double *b, double *x, double rtol,
                  double delta, int maxit, int check_every, double *r64, float *r32, CGWork<float> &w,
                  SolveOut &out) {
    out = SolveOut();
    const int cap = w.tun.grid_cap;
    const EllCols cols64 = (c.cols.any() && e64) ? c.cols : EllCols{};
    const bool ell32 = c.cols.any() && c.e;
    const AmgDevLevel<float> &l0 = c.lv[0];
    double *pv = w.partB;           // partials of the cycle's last kernel: (r.z, sum wgt r^2)
    double *pq = w.partA;           // partials of the product kernel: (p.q, 0)
    int gpost = 0, g1 = 0;
    auto zslot = [&](int at) { return reinterpret_cast<float *>(w.pair[at & 1]); };   // z in the pair's r
    const bool smooth0 = c.nlev > 1;
    // FP64 residual b - A x into r64 and the state (mode 0 also sets the
    // tolerance), its FP32 copy, and the next replacement armed at delta
    auto replace = [&](int mode) -> int {
        OASIS_TRY(cg_residual_state(s, cap, n, rp, ci, val, cols64, wgt, b, x, r64, 1, pv, w.st, rtol * rtol, mode,
                                    delta));
        hipLaunchKernelGGL(k_amg_to_f32, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, r64, r32);
        OASIS_TRY_LAUNCH();
        return OASIS_OK;
    };
    auto precondition = [&](int at, bool y0_ready) -> int {
        return amg_vcycle<float, float, float>(s, c, r32, y0_ready, zslot(at), 2, wgt, pv, &gpost, &w.st->flag,
                                               cap);
    };
    int restart_at = 0;
    auto iterate = [&](int itj) -> int {
        OASIS_TRY(cg_product_launch(s, cap, n, l0.rp, l0.ci, l0.val, ell32 ? c.cols : EllCols{},
                                    ell32 ? c.e : nullptr, w.pair[itj & 1], w.pair[(itj + 1) & 1], w.q, pv, gpost,
                                    2, w.st, itj, itj == restart_at ? 1 : 0, pq, &g1));
        hipLaunchKernelGGL(k_apcg_update32, dim3(grid_for(n, kBlock, kMaxPartials)), dim3(kBlock), 0, s, n,
                           w.pair[(itj + 1) & 1], w.q, x, r32, smooth0 ? l0.wd : nullptr, smooth0 ? l0.y : nullptr,
                           pq, g1, w.st, itj);
        OASIS_TRY_LAUNCH();
        return precondition(itj + 1, smooth0);
    };
    // as in amg_pcg_solve, the start residual is read back with the first poll
    OASIS_TRY(replace(0));
    OASIS_TRY(precondition(0, false));
    CGState h;
    double wbb = 0.0, tol2 = 0.0;
    bool first = true;
    auto rel = [&](double wrr) { return wbb > 0.0 ? std::sqrt(wrr / wbb) : std::sqrt(wrr); };
    AmgPlan plan(check_every, 0);
    int it = 0, rc = OASIS_OK;
    while (true) {
        const int m = std::min(plan.next, maxit - it);
        for (int j = 0; j < m; ++j) OASIS_TRY(iterate(it + j));
        it += m;
        OASIS_TRY(read_state(s, w.stage, w.st, &h, sizeof(h)));
        if (first) {
            first = false;
            wbb = h.wbb;
            tol2 = h.tol2;
            if (h.flag == 0) plan.restart(h.wrr, 0);
        }
        if (h.flag == 0 && it < maxit) {
            plan.observe(h.wrr_it, h.it_last, std::max(h.upd2, tol2));
            continue;
        }
        if (h.flag == 2 || h.flag == 3) {
            out.iters = h.it_done;
            out.status = rc = h.flag == 2 ? OASIS_EBREAKDOWN : OASIS_ENAN;
            out.rel_res = NAN;
            break;
        }
        // converged candidate, replacement due (flag 4) or maxit: the FP64
        // residual replaces the recursive one and decides
        const int at = h.flag == 0 ? it : h.it_done;
        OASIS_TRY(replace(1));
        OASIS_TRY(read_state(s, w.stage, w.st, &h, sizeof(h)));
        out.outer += 1;
        out.rel_res = rel(h.wrr);
        if (!std::isfinite(h.wrr)) {
            out.iters = at;
            out.status = rc = OASIS_ENAN;
            break;
        }
        if (h.wrr <= tol2) {
            out.iters = at;
            out.status = rc = OASIS_OK;
            break;
        }
        if (at >= maxit) {
            out.iters = at;
            out.status = rc = OASIS_ENOTCONV;
            break;
        }
        // continue from the replaced residual; the direction is kept
        out.replacements += 1;
        OASIS_TRY(precondition(at, false));
        it = at;
        plan.restart(h.wrr, at);
    }
    return rc;
}

template int amg_vcycle<float, float, float>(hipStream_t, const AmgCycle<float> &, const float *, bool, float *,
                                             int, const double *, double *, int *, const int *, int);
template int amg_vcycle<double>(hipStream_t, const AmgCycle<double> &, const double *, bool, double *, int,
                                const double *, double *, int *, const int *, int);
template int amg_vcycle<float>(hipStream_t, const AmgCycle<float> &, const double *, bool, double *, int,
                               const double *, double *, int *, const int *, int);
template int amg_pcg_solve<double>(hipStream_t, int, const int *, const int *, const double *, const double *,
                                   const AmgCycle<double> &, const double *, const double *, double *, double, int,
                                   int, bool, double *, CGWork<double> &, SolveOut &, int);
template int amg_pcg_solve<float>(hipStream_t, int, const int *, const int *, const double *, const double *,
                                  const AmgCycle<float> &, const double *, const double *, double *, double, int, int,
                                  bool, double *, CGWork<double> &, SolveOut &, int);

}  // namespace oasis
