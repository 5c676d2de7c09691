// Krylov solvers for the tentative velocity (BiCGStab + Jacobi) and the
// pressure correction (Jacobi-preconditioned CG), Sec. 6.2 of the paper.
//
// Both run on pre-scaled matrices so that the Jacobi preconditioner costs
// nothing inside the loop:
//   CG       : Ms = D^{-1/2} K D^{-1/2} (unit diagonal); same iterates as
//              CG with z = D^{-1} r in exact arithmetic.  With FP32 values
//              on the ELL copy an iteration is one pass (the single-
//              reduction recurrences, k_cg_sr); otherwise two (k_cg_p1*,
//              k_cg_p2).
//   BiCGStab : As = A D^{-1} (right Jacobi, iterate y = D x); its residual
//              is the true b - A x.  The residual norms take per-row
//              weights (1 here), so that other scalings can reuse the loop.
//
// Convergence is decided on the device.  Every kernel of an iteration
// first sums the partials of the previous kernel (fixed order, identical in
// all blocks), so scalars such as alpha and beta never leave the GPU; a
// kernel that detects convergence, breakdown or a non-finite value raises a
// flag that makes the remaining launched kernels return at once.  The host
// enqueues iterations in chunks and polls the small state block between
// chunks; on a convergence candidate it confirms with an explicit residual.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string_view>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "krylov.hpp"
#include "spmv.hpp"

namespace oasis {

// Producer grid cap (Tuning::grid_cap, default 512): every consumer block
// reads all partials of its producer (up to 9 per block in BiCGStab), so
// fewer, fuller producer blocks pay off, and a grid that is a whole number
// of blocks per CU (256 CUs) avoids a partly filled last round.  On the
// 1.6M-row channel the mixed velocity phase took 4.95 ms per step at 512 and
// 768 blocks, 5.23 at 1024, 5.45 at 640, 5.87 at 384, 6.63 at 2048; the
// FP32 Jacobi-CG pressure phase 66.6 ms at 512, 68.2 at 1024, 70.3 at 768.

// A flag written by an earlier kernel (or by block 0 of this one when it
// decides to stop, a decision every block reaches identically), read once
// per block so that the early return is uniform.
__device__ __forceinline__ int block_read_flag(const int *p) {
    __shared__ int v;
    if (threadIdx.x == 0) v = __atomic_load_n(p, __ATOMIC_RELAXED);
    __syncthreads();
    int r = v;
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// vector helpers

// a*b + c and c - a*b with a single rounding, so that a value formed once
// for a gathered column and once for the thread's own row is the same.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename T>
__device__ __forceinline__ T fmsub(T c, T a, T b) {
    return fmadd(-a, b, c);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int n, T *x, T v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(int n, T *__restrict__ y, const T *__restrict__ x) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = x[i];
}

// ---------------------------------------------------------------------------
// CG kernels

// r = b - Ms x (r[row * rs]: rs = 2 or 4 writes the r of an interleaved
// record); partials (r.r, sum wgt r^2, sum wgt b^2).  With an ELL copy's
// columns (cols.any()) the CSR values are read with those columns instead
// of the int32 column array.
template <typename T, class C>
__global__ __launch_bounds__(kBlock) void k_cg_init(int n, const int *__restrict__ rp,
                                                    const int *__restrict__ ci,
                                                    const T *__restrict__ val, EllCols cols,
                                                    const T *__restrict__ wgt,
                                                    const T *__restrict__ b,
                                                    const T *__restrict__ x, T *__restrict__ r, int rs,
                                                    double *part) {
    __shared__ double lds[3 * kBlock / kWave];
    double acc[3] = {0.0, 0.0, 0.0};
    auto gather = [&](int, int c, T v, bool ok, T(&a)[1]) {
        const T t = v * x[c];
        a[0] += ok ? t : T(0);
    };
    auto finish = [&](int row, int lane, T(&a)[1]) {
        if (lane == 0) {
            const T ri = b[row] - a[0];
            r[static_cast<long long>(row) * rs] = ri;
            const double rd = ri, bd = b[row], wd = wgt[row];
            acc[0] += rd * rd;
            acc[1] += wd * rd * rd;
            acc[2] += wd * bd * bd;
        }
    };
    if (cols.any())
        csr_cols_rows<T, 1, 2>(n, rp, val, cols, gather, finish);
    else
        csr_rows<T, 1, C>(n, rp, ci, val, gather, finish);
    write_partials<3>(acc, part, lds);
}

// mode 0: start of a solve (sets tol2); mode 1: explicit-residual check.
// upd_factor > 0 arms the next residual replacement at upd_factor * wrr.
__global__ __launch_bounds__(kBlock) void k_cg_finalize(const double *part, int nparts, CGState *st,
                                                        double rtol2, int mode, double upd_factor) {
    __shared__ double lds[3 * kBlock / kWave];
    double v[3];
    read_partials<3>(part, nparts, v, lds);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            st->tol2 = rtol2 * v[2];
            st->wbb = v[2];
        }
        st->wrr = v[1];
        st->upd2 = upd_factor * v[1];
        st->flag = 0;
        st->it_done = -1;
    }
}

// r_lo = (float) r_hi into the residual of a record of rs floats (the rest
// of the record is kept), x_lo = 0; partials (r.r, sum wgt r^2)
__global__ __launch_bounds__(kBlock) void k_cg_cast(int n, const double *__restrict__ rhi,
                                                    const float *__restrict__ wgt, float *__restrict__ rlo,
                                                    int rs, float *__restrict__ xlo, double *part) {
    __shared__ double lds[2 * kBlock / kWave];
    double acc[2] = {0.0, 0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float r = static_cast<float>(rhi[i]);
        rlo[i * rs] = r;
        xlo[i] = 0.f;
        const double rd = r;
        acc[0] += rd * rd;
        acc[1] += static_cast<double>(wgt[i]) * rd * rd;
    }
    write_partials<2>(acc, part, lds);
}

// Iteration part 1: convergence test on the incoming residual, direction
// p_new = r + beta p_old formed on the fly for the gathered operand (one
// gather of the (r, p_old) pair per entry), q = Ms p_new, partial p_new.q.
// partIn holds nIn blocks of `stride` values whose first two are
// (r.r, sum wgt r^2).
template <typename T, class C, int BS>
__global__ __launch_bounds__(BS) void k_cg_p1(int n, const int *__restrict__ rp,
                                                  const int *__restrict__ ci,
                                                  const T *__restrict__ val,
                                                  const RP<T> *__restrict__ cur,
                                                  RP<T> *__restrict__ nxt, T *__restrict__ q,
                                                  const double *partIn, int nIn, int stride, CGState *st,
                                                  int it, int beta_zero, const T *__restrict__ vnull,
                                                  double *partOut) {
    __shared__ double lds[2 * BS / kWave];
    if (block_read_flag(&st->flag)) return;
    double v[2];
    read_partials<2, BS>(partIn, nIn, v, lds, stride);
    const double rr = v[0], wrr = v[1];
    int flag = 0;
    if (!finite(wrr) || !finite(rr))
        flag = 3;
    else if (wrr <= st->tol2)
        flag = 1;
    else if (wrr <= st->upd2)
        flag = 4;
    if (flag) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->flag = flag;
            st->it_done = it;
            st->wrr = wrr;
        }
        return;
    }
    const double beta = beta_zero ? 0.0 : rr / st->rr[(it + 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rr[it & 1] = rr;
        st->wrr_it = wrr;
        st->it_last = it;
    }
    const T bt = static_cast<T>(beta);
    double acc[2] = {0.0, 0.0};
    auto finish = [&](int row, int lane, T(&a)[1]) {
        if (lane == 0) {
            const RP<T> me = cur[row];
            const T pn = beta_zero ? me.r : me.r + bt * me.p;
            nxt[row] = RP<T>{me.r, pn};    // k_cg_p2 updates r in place
            q[row] = a[0];
            acc[0] += static_cast<double>(pn) * static_cast<double>(a[0]);
            if (vnull) acc[1] += static_cast<double>(vnull[row]) * static_cast<double>(a[0]);
        }
    };
    // a fresh direction never uses p_old (it may hold stale values)
    if (beta_zero)
        csr_rows<T, 1, C, BS>(
            n, rp, ci, val,
            [&](int, int c, T vv, bool ok, T(&a)[1]) {
                const T t = vv * cur[c].r;
                a[0] += ok ? t : T(0);
            },
            finish);
    else
        csr_rows<T, 1, C, BS>(
            n, rp, ci, val,
            [&](int, int c, T vv, bool ok, T(&a)[1]) {
                const RP<T> g = cur[c];
                const T t = vv * (g.r + bt * g.p);
                a[0] += ok ? t : T(0);
            },
            finish);
    write_partials<2>(acc, partOut, lds);
}

// Iteration part 2: alpha = r.r / p.q, x += alpha p, r -= alpha q in the
// pair (r, p_new) written by part 1; partials (r.r, sum wgt r^2).
template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_cg_p2(int n, RP<T> *__restrict__ nxt,
                                                  const T *__restrict__ q, T *__restrict__ x,
                                                  const T *__restrict__ wgt, const double *partIn,
                                                  int nIn, CGState *st, int it,
                                                  const T *__restrict__ vnull, double *partOut) {
    __shared__ double lds[2 * BS / kWave];
    if (block_read_flag(&st->flag)) return;
    double v[2];
    read_partials<2, BS>(partIn, nIn, v, lds);
    const double pq = v[0];
    if (!(pq > 0.0) || !finite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->flag = finite(pq) ? 2 : 3;
            st->it_done = it;
        }
        return;
    }
    const T a = static_cast<T>(st->rr[it & 1] / pq);
    const T cv = static_cast<T>(v[1]);    // (v.q) for a unit null vector v
    double acc[2] = {0.0, 0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        RP<T> nx = nxt[i];
        const T xi = x[i] + a * nx.p;
        const T qi = vnull ? q[i] - cv * vnull[i] : q[i];
        const T ri = nx.r - a * qi;
        x[i] = xi;
        nx.r = ri;
        nxt[i] = nx;
        const double rd = ri;
        acc[0] += rd * rd;
        acc[1] += static_cast<double>(wgt[i]) * rd * rd;
    }
    write_partials<2>(acc, partOut, lds);
}

// Iteration part 1 on the ELL copy of the matrix: the same computation as
// k_cg_p1.  L lanes share a row (each holds E = kEll / L entries, fetched
// with 8-byte offset and 16-byte value loads), so that a lane has E pair
// gathers in flight.  The row loop is straight-line code as in k_cg_sr:
// every lane fetches the next row's offsets, values and own-row state from
// clamped row indices, the pattern id one row further ahead, over two
// register sets; DICT fixes the column storage and BZ (beta = 0) the
// direction update at compile time.
template <typename T, int BS, int L, bool DICT>
__global__ __launch_bounds__(BS) void k_cg_p1_ell(int n, EllCols cols,
                                                  const T *__restrict__ eval,
                                                  const RP<T> *__restrict__ cur,
                                                  RP<T> *__restrict__ nxt, T *__restrict__ q,
                                                  const double *partIn, int nIn, int stride, CGState *st,
                                                  int it, int beta_zero, const T *__restrict__ vnull,
                                                  double *partOut) {
    constexpr int E = kEll / L;
    static_assert(E % 4 == 0, "lanes per row must leave a multiple of 4 entries per lane");
    __shared__ double lds[2 * BS / kWave];
    if (block_read_flag(&st->flag)) return;
    double v[2];
    read_partials<2, BS>(partIn, nIn, v, lds, stride);
    const double rr = v[0], wrr = v[1];
    int flag = 0;
    if (!finite(wrr) || !finite(rr))
        flag = 3;
    else if (wrr <= st->tol2)
        flag = 1;
    else if (wrr <= st->upd2)
        flag = 4;
    if (flag) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->flag = flag;
            st->it_done = it;
            st->wrr = wrr;
        }
        return;
    }
    const double beta = beta_zero ? 0.0 : rr / st->rr[(it + 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rr[it & 1] = rr;
        st->wrr_it = wrr;
        st->it_last = it;
    }
    const T bt = static_cast<T>(beta);
    double acc[2] = {0.0, 0.0};
    const int lane = threadIdx.x & (L - 1);
    const RowRange<L, BS> range(n);
    long long row = range.first + range.gid;
    if (row < range.last) {
        const long long top = range.last - 1;
        auto clamp = [top](long long r) { return r < top ? r : top; };
        const T *vsrc = vnull ? vnull : eval;   // read unused without a null vector
        struct Stage {
            int c[E];
            T w[E];
            RP<T> me;
            T vr;
        };
        auto fetch = [&](Stage &S, long long r, int key) {
            ell_fetch_key<DICT, T, E>(r, key, lane, n, cols, eval, S.c, S.w);
            S.me = cur[r];
            S.vr = vsrc[r];
        };
        auto run = [&](auto bzc) {
            constexpr bool BZ = decltype(bzc)::value;
            auto step = [&](const Stage &S, Stage &N, int kin, int &kout) {
                RP<T> gv[E];
#pragma unroll
                for (int k = 0; k < E; ++k) gv[k] = cur[S.c[k]];
                T wv[E];
#pragma unroll
                for (int k = 0; k < E; ++k) wv[k] = S.w[k];
                fetch(N, clamp(row + range.ngroups), kin);
                kout = ell_key<DICT>(cols, clamp(row + 2 * range.ngroups));
                T a = T(0);
#pragma unroll
                for (int k = 0; k < E; ++k) a += wv[k] * (BZ ? gv[k].r : gv[k].r + bt * gv[k].p);
                a = group_sum<L>(a);
                if (lane == 0) {
                    const T pn = BZ ? S.me.r : S.me.r + bt * S.me.p;
                    nxt[row] = RP<T>{S.me.r, pn};
                    q[row] = a;
                    acc[0] += static_cast<double>(pn) * static_cast<double>(a);
                    if (vnull) acc[1] += static_cast<double>(S.vr) * static_cast<double>(a);
                }
            };
            Stage A, B;
            int ka, kb;
            fetch(A, row, ell_key<DICT>(cols, row));
            ka = ell_key<DICT>(cols, clamp(row + range.ngroups));
            for (;;) {
                step(A, B, ka, kb);
                row += range.ngroups;
                if (row >= range.last) break;
                step(B, A, kb, ka);
                row += range.ngroups;
                if (row >= range.last) break;
            }
        };
        if (beta_zero)
            run(std::true_type{});
        else
            run(std::false_type{});
    }
    write_partials<2>(acc, partOut, lds);
}

// Launch the ELL product kernel (two lanes per row, which measured faster
// than one or four); returns its grid.  The producer grid cap `cap`: the
// update kernel reads every block's partials, and 1024 blocks measured 59 us
// per FP64 product against 66 us with 2048 and 65 / 80 us with 768 / 512
// (1.6M rows).
template <typename T, int BS>
static int launch_p1_ell(hipStream_t s, int cap, int n, const EllCols &cols, const T *eval, const RP<T> *cur,
                         RP<T> *nxt, T *q, const double *partIn, int nIn, int stride, CGState *st, int it,
                         int beta_zero, const T *vnull, double *partOut, bool grid_only = false) {
    auto go = [&](auto kern, int rows_per_blk) {
        const int g = grid_for(n, rows_per_blk, cap * kBlock / BS);
        if (!grid_only)
            hipLaunchKernelGGL(kern, dim3(g), dim3(BS), 0, s, n, cols, eval, cur, nxt, q, partIn, nIn, stride, st,
                               it, beta_zero, vnull, partOut);
        return g;
    };
    const bool dict = cols.pid != nullptr;
    return dict ? go(k_cg_p1_ell<T, BS, 2, true>, BS / 2) : go(k_cg_p1_ell<T, BS, 2, false>, BS / 2);
}

// ---------------------------------------------------------------------------
// Single-reduction CG on the ELL copy (the recurrences of Chronopoulos and
// Gear).  With w = Ms r and s = Ms p carried as vectors, an iteration
//   p_i = r_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1},
//   x_{i+1} = x_i + alpha_i p_i, r_{i+1} = r_i - alpha_i s_i, w_{i+1} = Ms r_{i+1}
// is one pass over the matrix, and every scalar it needs comes from one set
// of partial sums written by the previous pass:
//   beta_i = (r_i.r_i) / (r_{i-1}.r_{i-1}),  alpha_i = (r_i.r_i) / (p_i.s_i),
//   p_i.s_i = r_i.w_i + beta_i (r_i.s_{i-1} + p_{i-1}.w_i) + beta_i^2 p_{i-1}.s_{i-1}.
// Row i's product gathers r_{i+1} of its columns, formed on the fly from the
// gathered record (r, w, s) with the same roundings as in the owning row.
// In exact arithmetic the iterates are those of Hestenes-Stiefel CG.
//
// With a null vector v (singular matrix) each row projects w and s,
// w - (v.w) v, in its own update; the gathered operand leaves that term out,
// whose product (v.w) Ms v is second order in the rounding of Ms.

// Partials per block: r.r, sum wgt r^2, r.w, r.s + p.w, p.s, v.w, v.s
// (of the record just written).
constexpr int kSr = 7;

template <typename T>
__device__ __forceinline__ void sr_partials(double (&acc)[kSr], const Q4<T> &o, double wd, double vd) {
    const double r = o.r, w = o.w, s = o.s, p = o.p;
    acc[0] += r * r;
    acc[1] += wd * r * r;
    acc[2] += r * w;
    acc[3] += r * s + p * w;
    acc[4] += p * s;
    acc[5] += vd * w;
    acc[6] += vd * s;
}

// One iteration (see above).  Convergence tests on the incoming residual
// as in k_cg_p1; a non-positive p.s is a breakdown.
template <typename T, int BS, int L, bool PROJ, bool DICT>
__global__ __launch_bounds__(BS) void k_cg_sr(int n, EllCols cols, const T *__restrict__ eval,
                                              const Q4<T> *__restrict__ cur, Q4<T> *__restrict__ nxt,
                                              T *__restrict__ x, const T *__restrict__ wgt,
                                              const T *__restrict__ vnull, double vscale, const double *partIn,
                                              int nIn, CGState *st, int it, int beta_zero, double *partOut) {
    constexpr int E = kEll / L;
    static_assert(E % 4 == 0, "lanes per row must leave a multiple of 4 entries per lane");
    __shared__ double lds[kSr * BS / kWave];
    if (block_read_flag(&st->flag)) return;
    double v[kSr];
    read_partials<kSr, BS>(partIn, nIn, v, lds);
    const double rr = v[0], wrr = v[1];
    int flag = 0;
    double beta = 0.0, ps = 0.0;
    if (!finite(wrr) || !finite(rr)) {
        flag = 3;
    } else if (wrr <= st->tol2) {
        flag = 1;
    } else if (wrr <= st->upd2) {
        flag = 4;
    } else {
        beta = beta_zero ? 0.0 : rr / st->rr[(it + 1) & 1];
        ps = v[2] + beta * (v[3] + beta * v[4]);
        if (!finite(ps))
            flag = 3;
        else if (!(ps > 0.0))
            flag = 2;
    }
    if (flag) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->flag = flag;
            st->it_done = it;
            st->wrr = wrr;
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rr[it & 1] = rr;
        st->wrr_it = wrr;
        st->it_last = it;
    }
    const T al = static_cast<T>(rr / ps), bt = static_cast<T>(beta);
    const T cw = static_cast<T>(v[5]), cs = static_cast<T>(v[6]);
    double acc[kSr];
#pragma unroll
    for (int k = 0; k < kSr; ++k) acc[k] = 0.0;
    const int lane = threadIdx.x & (L - 1);
    const RowRange<L, BS> range(n);
    long long row = range.first + range.gid;
    if (row < range.last) {
        // Software-pipelined, straight-line loop: while this row's gathers
        // are in flight, every lane fetches the next row's offsets and
        // values, its own-row state (record, x, null-vector entry, weight)
        // and the pattern id of the row after it.  Row indices of these
        // fetches are clamped into the range (the last iteration re-reads
        // a valid row and drops it), so no load sits behind a branch and
        // the owning lane's update waits on none of them.  The loop is
        // unrolled twice over two register sets, so that no loaded value
        // is copied across the back edge (a copy waits for its load).
        const long long top = range.last - 1;
        auto clamp = [top](long long r) { return r < top ? r : top; };
        const T *wsrc = wgt ? wgt : x;   // read unused when the weights come from vnull
        struct Stage {
            int c[E];
            T w[E];
            Q4<T> me;
            T xr, vr, wr;
        };
        auto fetch = [&](Stage &S, long long r, int key) {
            ell_fetch_key<DICT, T, E>(r, key, lane, n, cols, eval, S.c, S.w);
            S.me = cur[r];
            S.xr = x[r];
            S.vr = PROJ ? vnull[r] : T(0);
            S.wr = wsrc[r];
        };
        auto step = [&](const Stage &S, Stage &N, int kin, int &kout) {
            Q4<T> g[E];
#pragma unroll
            for (int k = 0; k < E; ++k) g[k] = cur[S.c[k]];
            fetch(N, clamp(row + range.ngroups), kin);
            kout = ell_key<DICT>(cols, clamp(row + 2 * range.ngroups));
            T a = T(0);
#pragma unroll
            for (int k = 0; k < E; ++k) a += S.w[k] * fmsub(g[k].r, al, fmadd(bt, g[k].s, g[k].w));
            a = group_sum<L>(a);
            if (lane == 0) {
                const Q4<T> &m = S.me;
                const T wp = PROJ ? fmsub(m.w, cw, S.vr) : m.w;
                const T sp = PROJ ? fmsub(m.s, cs, S.vr) : m.s;
                Q4<T> o;
                o.s = fmadd(bt, sp, wp);
                o.p = fmadd(bt, m.p, m.r);
                o.r = fmsub(m.r, al, o.s);
                o.w = a;
                x[row] = fmadd(al, o.p, S.xr);
                nxt[row] = o;
                const double vd = S.vr;
                sr_partials<T>(acc, o, wgt ? static_cast<double>(S.wr) : vscale * vd * vd, vd);
            }
        };
        Stage A, B;
        int ka, kb;
        fetch(A, row, ell_key<DICT>(cols, row));
        ka = ell_key<DICT>(cols, clamp(row + range.ngroups));
        for (;;) {
            step(A, B, ka, kb);
            row += range.ngroups;
            if (row >= range.last) break;
            step(B, A, kb, ka);
            row += range.ngroups;
            if (row >= range.last) break;
        }
    }
    write_partials<kSr>(acc, partOut, lds);
}

// Start of a single-reduction run on the residual in rec: w = Ms r and, with
// keep != 0, s = Ms p for the direction kept (p itself unchanged);
// otherwise s = p = 0.  The record is updated in place (the gathered fields
// r and, with keep, p are not written); the partials are those the first
// iteration reads.
template <typename T, int BS, int L>
__global__ __launch_bounds__(BS) void k_cg_sr_start(int n, EllCols cols,
                                                    const T *__restrict__ eval, Q4<T> *rec,
                                                    const T *__restrict__ wgt, const T *__restrict__ vnull,
                                                    double vscale, int keep, double *partOut) {
    constexpr int E = kEll / L;
    __shared__ double lds[kSr * BS / kWave];
    double acc[kSr];
#pragma unroll
    for (int k = 0; k < kSr; ++k) acc[k] = 0.0;
    const int lane = threadIdx.x & (L - 1);
    const RowRange<L, BS> range(n);
    for (long long row = range.first + range.gid; row < range.last; row += range.ngroups) {
        int c[E];
        T w[E];
        ell_fetch<T, E>(row, lane, n, cols, eval, c, w);
        T ar = T(0), ap = T(0);
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const Q4<T> g = rec[c[k]];
            ar += w[k] * g.r;
            ap += w[k] * g.p;
        }
        ar = group_sum<L>(ar);
        ap = group_sum<L>(ap);
        if (lane == 0) {
            Q4<T> o;
            o.r = rec[row].r;
            o.w = ar;
            o.s = keep ? ap : T(0);
            o.p = keep ? rec[row].p : T(0);
            rec[row].w = o.w;
            rec[row].s = o.s;
            if (!keep) rec[row].p = T(0);
            const double vd = vnull ? static_cast<double>(vnull[row]) : 0.0;
            sr_partials<T>(acc, o, wgt ? static_cast<double>(wgt[row]) : vscale * vd * vd, vd);
        }
    }
    write_partials<kSr>(acc, partOut, lds);
}

// Single-reduction CG on the ELL copy in rec / the workspace partials.
// Used by cg_run and cg_mixed_run when the ELL copy is present.
template <typename T>
struct SrLoop {
    static constexpr int BS = kBlock, L = 2;
    hipStream_t s;
    int n;
    EllCols cols;
    const T *eval;
    const T *wgt, *vnull;
    double vscale;
    CGWork<T> *w;
    int grid;
    // vscale > 0 (with vnull): the norm weights are vscale * vnull^2 and are
    // formed in the kernels instead of read from wgt
    SrLoop(hipStream_t s_, int n_, CGWork<T> &w_, const T *wgt_, const T *vnull_, double vscale_)
        : s(s_), n(n_), cols(w_.cols), eval(w_.eval), wgt(vnull_ && vscale_ > 0.0 ? nullptr : wgt_),
          vnull(vnull_), vscale(vnull_ && vscale_ > 0.0 ? vscale_ : 0.0), w(&w_) {
        // every block of an iteration reads all partials of the previous
        // one, kSr per block: the grid is capped by the tuning's grid_cap
        grid = grid_for(n, BS / L, std::min(kMaxPartials, w_.tun.grid_cap));
    }
    double *part(int it) const { return (it & 1) ? w->partA : w->partB; }
    // partials for iteration `at`, written into part(at)
    int start(int at, bool keep) {
        hipLaunchKernelGGL((k_cg_sr_start<T, BS, L>), dim3(grid), dim3(BS), 0, s, n, cols, eval, w->rec[at & 1],
                           wgt, vnull, vscale, keep ? 1 : 0, part(at));
        OASIS_TRY_LAUNCH();
        return OASIS_OK;
    }
    template <bool PROJ, bool DICT>
    void go(int it, int beta_zero, T *x) {
        hipLaunchKernelGGL((k_cg_sr<T, BS, L, PROJ, DICT>), dim3(grid), dim3(BS), 0, s, n, cols, eval,
                           w->rec[it & 1], w->rec[(it + 1) & 1], x, wgt, vnull, vscale, part(it), grid, w->st, it,
                           beta_zero, part(it + 1));
    }
    void iterate(int it, int beta_zero, T *x) {
        const bool dict = cols.pid != nullptr;
        if (vnull)
            dict ? go<true, true>(it, beta_zero, x) : go<true, false>(it, beta_zero, x);
        else
            dict ? go<false, true>(it, beta_zero, x) : go<false, false>(it, beta_zero, x);
    }
};

__global__ __launch_bounds__(kBlock) void k_max_row(int n, const int *__restrict__ rp, int *out) {
    int m = 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        m = max(m, rp[i + 1] - rp[i]);
    for (int o = kWave / 2; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, m);
}

__global__ __launch_bounds__(kBlock) void k_csr_to_ell(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                       const double *__restrict__ val, short *__restrict__ ecol,
                                                       double *__restrict__ eval, float *__restrict__ eval32,
                                                       int *misfit) {
    const long long half = n / 2;
    int bad = 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int s = rp[i], len = rp[i + 1] - s;
        bad |= len > kEll ? 1 : 0;
        for (int k = 0; k < kEll; ++k) {
            long long d = 0;
            double v = 0.0;
            if (k < len) {
                d = static_cast<long long>(ci[s + k]) - i;
                if (d >= half) d -= n;
                if (d < -half) d += n;
                v = val[s + k];
            }
            const bool ok = d >= -32768 && d <= 32767;
            bad |= ok ? 0 : 1;
            ecol[i * kEll + k] = static_cast<short>(ok ? d : 0);
            if (eval) eval[i * kEll + k] = v;
            if (eval32) eval32[i * kEll + k] = static_cast<float>(v);
        }
    }
    if (bad) atomicOr(misfit, 1);
}

int csr_max_row(hipStream_t s, int n, const int *rp, int *tmp, int *out) {
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(kBlock), 0, s, 1, tmp, 0);
    hipLaunchKernelGGL(k_max_row, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, n, rp, tmp);
    OASIS_TRY_LAUNCH();
    OASIS_TRY_HIP(hipMemcpyAsync(out, tmp, sizeof(int), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    return OASIS_OK;
}

int csr_to_ell(hipStream_t s, int n, const int *rp, const int *ci, const double *val, short *ecol,
               double *eval, float *eval32, int *tmp, bool *fits) {
    if (!ecol || (!eval && !eval32) || !tmp || !fits) return OASIS_EINVAL;
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(kBlock), 0, s, 1, tmp, 0);
    hipLaunchKernelGGL(k_csr_to_ell, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, rp, ci, val, ecol,
                       eval, eval32, tmp);
    OASIS_TRY_LAUNCH();
    int misfit = 1;
    OASIS_TRY_HIP(hipMemcpyAsync(&misfit, tmp, sizeof(int), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    *fits = misfit == 0;
    return OASIS_OK;
}

// Rows sharing an offset list share a dictionary entry; ids in order of
// first occurrence, so the dictionary is a function of the pattern alone.
int ell_dictionary(hipStream_t s, int n, const short *ecol, unsigned short *pid, short *ptab, int *npat,
                   bool enable) {
    if (!ecol || !pid || !ptab || !npat || n < 0) return OASIS_EINVAL;
    *npat = 0;
    if (!enable) return OASIS_OK;
    std::vector<short> off(static_cast<size_t>(n) * kEll);
    OASIS_TRY_HIP(hipMemcpyAsync(off.data(), ecol, off.size() * sizeof(short), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    const size_t rowb = kEll * sizeof(short);
    // worth it only while the table stays small against the rows it serves
    const int max_pat = std::min(kMaxEllPatterns, n / 8);
    std::unordered_map<std::string_view, int> ids;
    ids.reserve(2 * kMaxEllPatterns);
    std::vector<unsigned short> hp(static_cast<size_t>(n));
    std::vector<short> tab;
    for (int i = 0; i < n; ++i) {
        const short *r = off.data() + static_cast<size_t>(i) * kEll;
        const auto ins = ids.try_emplace(std::string_view(reinterpret_cast<const char *>(r), rowb),
                                         static_cast<int>(ids.size()));
        if (ins.second) {
            if (static_cast<int>(ids.size()) > max_pat) return OASIS_OK;
            tab.insert(tab.end(), r, r + kEll);
        }
        hp[i] = static_cast<unsigned short>(ins.first->second);
    }
    OASIS_TRY_HIP(hipMemcpyAsync(pid, hp.data(), hp.size() * sizeof(unsigned short), hipMemcpyHostToDevice, s));
    OASIS_TRY_HIP(hipMemcpyAsync(ptab, tab.data(), tab.size() * sizeof(short), hipMemcpyHostToDevice, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    *npat = static_cast<int>(ids.size());
    return OASIS_OK;
}

template <typename T>
void carve_cg(Carver &c, int n, CGWork<T> &w) {
    for (int k = 0; k < 2; ++k) {
        w.rec[k] = c.take<Q4<T>>(n);
        w.pair[k] = reinterpret_cast<RP<T> *>(w.rec[k]);
    }
    w.q = c.take<T>(n);
    w.partA = c.take<double>(kSr * kMaxPartials);
    w.partB = c.take<double>(kSr * kMaxPartials);
    w.st = c.take<CGState>(1);
}

// Single-reduction iterations on the ELL copy (Tuning::single).  Their
// gathered record is (r, w, s) rather than (r, p): with FP32 values the one
// pass beats the two (the update pass is gone), with FP64 values the wider
// gathers cost more than that pass.

// Kernel timing of a solve (time_kernel): when the solve has stopped at
// maxit, the last iteration's state (a residual just recomputed, the flag
// cleared, the previous direction and r.r in place) is a valid input for
// one more direction+product launch; `launch` repeats that launch `reps`
// times back to back between two events, so kernel_ms / kernel_count is
// the kernel's duration without per-launch dispatch gaps.  Each repeat does
// a full iteration's product work (same inputs, same outputs).
template <class Launch>
static int time_product(hipStream_t s, int reps, Launch launch, SolveOut &out) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    OASIS_TRY_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return OASIS_EHIP;
    }
    int rc = OASIS_OK;
    float ms = 0.f;
    if (hipEventRecord(e0, s) != hipSuccess) rc = OASIS_EHIP;
    for (int i = 0; i < reps && rc == OASIS_OK; ++i) {
        launch();
        if (hipGetLastError() != hipSuccess) rc = OASIS_EHIP;
    }
    if (rc == OASIS_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = OASIS_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == OASIS_OK) {
        out.kernel_ms = ms;
        out.kernel_count = reps;
    }
    return rc;
}

// Grids of the iteration kernels with BS-thread blocks (256: 1024-thread
// blocks keep the occupancy with a quarter of the partial sums but measured
// slower on the product kernel).  The elementwise update kernel is capped at
// the tuning's grid_cap: a streaming kernel needs fewer resident waves than
// the gather-bound product, and fewer blocks mean fewer partial sums for the
// product kernel to read.
template <int BS>
struct CgGrids {
    int p1, p2;
    template <class C>
    static CgGrids make(int n, int cap_update) {
        const int cap = kMaxPartials * kBlock / BS;
        const int cap2 = std::min(cap, cap_update * kBlock / BS);
        return CgGrids{grid_for(n, rows_per_block<C, BS>(), cap), grid_for(n, BS, cap2)};
    }
};

// Iterations to launch before the next host poll of the CG state.  With
// check_every > 0 that fixed number; otherwise estimated from the rate at
// which log(wrr) has fallen since the last restart of the recurrence, so
// that the poll comes just before the next event (a residual replacement
// at upd2, convergence at tol2): fewer polls than a fixed chunk, and few
// launches after the event that return at once.  Within [8, 256]; 32
// before any rate is known.
struct ChunkPlan {
    int fixed;
    double rate = 0.0;            // d log(wrr) / d iteration, < 0 once known
    double w0 = 0.0;
    int it0 = -1;
    int next = 32;
    explicit ChunkPlan(int check_every) : fixed(check_every) {
        if (fixed > 0) next = fixed;
    }
    void plan(double wrr, double target) {
        if (fixed > 0) return;
        if (!(rate < 0.0) || !(wrr > 0.0) || !(target > 0.0)) {
            next = 32;
            return;
        }
        const double k = std::log(target / wrr) / rate;
        next = static_cast<int>(std::min(256.0, std::max(8.0, 0.85 * k)));
    }
    // a new recurrence starts at iteration it from weighted residual wrr
    void restart(double wrr, int it, double target) {
        w0 = wrr;
        it0 = it;
        plan(wrr, target);
    }
    // state seen at a poll: the residual entering iteration it_last
    void observe(double wrr, int it_last, double target) {
        if (it0 >= 0 && it_last > it0 && wrr > 0.0 && w0 > 0.0) {
            const double r = std::log(wrr / w0) / (it_last - it0);
            if (r < 0.0) rate = r;
        }
        plan(wrr, target);
    }
};

template <typename T, class C, int BS>
static int cg_run(hipStream_t s, int n, const int *rp, const int *ci, const T *val, const T *wgt,
                  const T *b, T *x, double rtol, int maxit, int check_every, bool time_kernel,
                  CGWork<T> &w, SolveOut &out) {
    const int cap = w.tun.grid_cap;
    const int gi = grid_for(n, rows_per_block<C>(), cap);     // k_cg_init (kBlock threads)
    const CgGrids<BS> g = CgGrids<BS>::template make<C>(n, cap);
    const bool ell = w.cols.any() && w.eval && w.tun.ell();
    const bool sr = ell && w.tun.single(sizeof(T));
    SrLoop<T> loop(s, n, w, wgt, nullptr, 0.0);
    const int g1 = ell ? launch_p1_ell<T, BS>(s, cap, n, w.cols, w.eval, nullptr, nullptr, nullptr, nullptr, 0, 2,
                                              nullptr, 0, 0, nullptr, nullptr, true)
                       : g.p1;
    out = SolveOut();
    // explicit residual into the r of the record that iteration `at` reads
    auto residual = [&](int mode, int at) -> int {
        T *r = sr ? reinterpret_cast<T *>(w.rec[at & 1]) : reinterpret_cast<T *>(w.pair[at & 1]);
        hipLaunchKernelGGL((k_cg_init<T, C>), dim3(gi), dim3(kBlock), 0, s, n, rp, ci, val,
                           ell ? w.cols : EllCols{}, wgt, b, x, r, sr ? 4 : 2, w.partB);
        OASIS_TRY_LAUNCH();
        hipLaunchKernelGGL(k_cg_finalize, dim3(1), dim3(kBlock), 0, s, w.partB, gi, w.st,
                           rtol * rtol, mode, 0.0);
        OASIS_TRY_LAUNCH();
        return OASIS_OK;
    };
    OASIS_TRY(residual(0, 0));
    if (sr) OASIS_TRY(loop.start(0, false));
    CGState h;
    OASIS_TRY(read_state(s, w.stage, w.st, &h, sizeof(h)));
    ChunkPlan plan(check_every);
    plan.restart(h.wrr, 0, h.tol2);
    int it = 0, restart_at = 0;
    int rc = OASIS_OK;
    auto finish = [&](double wrr, double wbb) {
        out.rel_res = wbb > 0.0 ? std::sqrt(wrr / wbb) : std::sqrt(wrr);
    };
    while (true) {
        const int m = std::min(plan.next, maxit - it);
        for (int j = 0; j < m; ++j) {
            const int itj = it + j;
            // after a restart the incoming partials are k_cg_init's (3 per block)
            const bool fresh = itj == restart_at;
            if (sr) {
                loop.iterate(itj, fresh ? 1 : 0, x);
                OASIS_TRY_LAUNCH();
                continue;
            }
            const int nin = fresh ? gi : g.p2, stride = fresh ? 3 : 2;
            if (ell)
                launch_p1_ell<T, BS>(s, cap, n, w.cols, w.eval, w.pair[itj & 1], w.pair[(itj + 1) & 1], w.q,
                                     w.partB, nin, stride, w.st, itj, fresh ? 1 : 0, static_cast<const T *>(nullptr),
                                     w.partA);
            else
                hipLaunchKernelGGL((k_cg_p1<T, C, BS>), dim3(g1), dim3(BS), 0, s, n, rp, ci, val,
                                   w.pair[itj & 1], w.pair[(itj + 1) & 1], w.q, w.partB, nin, stride, w.st, itj,
                                   fresh ? 1 : 0, static_cast<const T *>(nullptr), w.partA);
            OASIS_TRY_LAUNCH();
            hipLaunchKernelGGL((k_cg_p2<T, BS>), dim3(g.p2), dim3(BS), 0, s, n, w.pair[(itj + 1) & 1], w.q, x,
                               wgt, w.partA, g1, w.st, itj, static_cast<const T *>(nullptr), w.partB);
            OASIS_TRY_LAUNCH();
        }
        it += m;
        OASIS_TRY(read_state(s, w.stage, w.st, &h, sizeof(h)));
        if (h.flag == 0) {
            if (it < maxit) {
                plan.observe(h.wrr_it, h.it_last, h.tol2);
                continue;
            }
            const double wbb = h.wbb, tol2 = h.tol2;
            OASIS_TRY(residual(1, it));
            OASIS_TRY(read_state(s, w.stage, w.st, &h, sizeof(h)));
            out.iters = it;
            finish(h.wrr, wbb);
            out.status = rc = (h.wrr <= tol2) ? OASIS_OK : OASIS_ENOTCONV;
            if (time_kernel && rc == OASIS_ENOTCONV && sr) {
                // repeat iteration `it` from the residual just recomputed; x
                // is left alone (the repeats advance a scratch copy)
                OASIS_TRY(loop.start(it, false));
                OASIS_TRY(time_product(s, maxit, [&] { loop.iterate(it, 1, w.q); }, out));
            } else if (time_kernel && rc == OASIS_ENOTCONV) {
                // repeat iteration `it` on the residual just recomputed (k_cg_init's partials)
                const int itj = it;
                OASIS_TRY(time_product(
                    s, maxit,
                    [&] {
                        if (ell)
                            launch_p1_ell<T, BS>(s, cap, n, w.cols, w.eval, w.pair[itj & 1], w.pair[(itj + 1) & 1],
                                                 w.q, w.partB, gi, 3, w.st, itj, 0, static_cast<const T *>(nullptr),
                                                 w.partA);
                        else
                            hipLaunchKernelGGL((k_cg_p1<T, C, BS>), dim3(g1), dim3(BS), 0, s, n, rp, ci, val,
                                               w.pair[itj & 1], w.pair[(itj + 1) & 1], w.q, w.partB, gi, 3, w.st,
                                               itj, 0, static_cast<const T *>(nullptr), w.partA);
                    },
                    out));
            }
            break;
        }
        if (h.flag == 1) {
            const int itd = h.it_done;
            const double wbb = h.wbb, tol2 = h.tol2;
            OASIS_TRY(residual(1, itd));
            OASIS_TRY(read_state(s, w.stage, w.st, &h, sizeof(h)));
            if (h.wrr <= tol2) {
                out.iters = itd;
                finish(h.wrr, wbb);
                out.status = rc = OASIS_OK;
                break;
            }
            // continue from the explicit residual with a fresh direction
            out.replacements += 1;
            it = itd;
            restart_at = itd;
            if (it >= maxit) {
                out.iters = it;
                finish(h.wrr, wbb);
                out.status = rc = OASIS_ENOTCONV;
                break;
            }
            if (sr) OASIS_TRY(loop.start(itd, false));
            plan.restart(h.wrr, itd, tol2);
            continue;
        }
        out.iters = h.it_done;
        out.status = rc = (h.flag == 2) ? OASIS_EBREAKDOWN : OASIS_ENAN;
        out.rel_res = NAN;
        break;
    }
    return rc;
}

template <typename T>
int cg_solve(hipStream_t s, int n, const int *rp, const int *ci, const T *val, const T *wgt,
             const T *b, T *x, double rtol, int maxit, int check_every, bool time_kernel,
             CGWork<T> &w, SolveOut &out) {
    return with_cfg([&](auto c) {
        return cg_run<T, decltype(c), kBlock>(s, n, rp, ci, val, wgt, b, x, rtol, maxit, check_every,
                                              time_kernel, w, out);
    });
}

__global__ __launch_bounds__(kBlock) void k_add_lo(int n, double *__restrict__ x, const float *__restrict__ e) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] += static_cast<double>(e[i]);
}

template <class C, int BS>
static int cg_mixed_run(hipStream_t s, int n, const int *rp, const int *ci, const double *val,
                        const float *val32, const double *wgt, const float *wgt32,
                        const float *vnull, double vscale, const double *b, double *x, double rtol, double delta,
                        int maxit, int check_every, bool time_kernel, CGWork<float> &w,
                        float *xlo, double *rhi, SolveOut &out) {
    const int cap = w.tun.grid_cap;
    const int gi = grid_for(n, rows_per_block<C>(), cap);     // k_cg_init (kBlock threads)
    const int gv = grid_for(n, kBlock, cap);                  // k_cg_cast, k_add_lo
    const CgGrids<BS> g = CgGrids<BS>::template make<C>(n, cap);
    const bool ell = w.cols.any() && w.eval && w.tun.ell();
    const bool sr = ell && w.tun.single(4);
    SrLoop<float> loop(s, n, w, wgt32, vnull, vscale);
    const int g1 = ell ? launch_p1_ell<float, BS>(s, cap, n, w.cols, w.eval, nullptr, nullptr, nullptr, nullptr, 0,
                                                  2, nullptr, 0, 0, nullptr, nullptr, true)
                       : g.p1;
    const double upd = delta * delta;
    out = SolveOut();
    // FP64 residual of the FP64 accumulator, then its FP32 copy (x_lo = 0)
    auto replace = [&](int mode) -> int {
        hipLaunchKernelGGL((k_cg_init<double, C>), dim3(gi), dim3(kBlock), 0, s, n, rp, ci, val,
                           ell ? w.cols : EllCols{}, wgt, b, x, rhi, 1, w.partB);
        OASIS_TRY_LAUNCH();
        hipLaunchKernelGGL(k_cg_finalize, dim3(1), dim3(kBlock), 0, s, w.partB, gi, w.st,
                           rtol * rtol, mode, upd);
        OASIS_TRY_LAUNCH();
        return OASIS_OK;
    };
    // into the r of the record that iteration `at` reads; its direction stays
    // (the single-reduction start then forms Ms r and Ms p of the record)
    auto cast = [&](int at, bool keep) -> int {
        float *r = sr ? reinterpret_cast<float *>(w.rec[at & 1]) : reinterpret_cast<float *>(w.pair[at & 1]);
        hipLaunchKernelGGL(k_cg_cast, dim3(gv), dim3(kBlock), 0, s, n, rhi, wgt32, r, sr ? 4 : 2, xlo, w.partB);
        OASIS_TRY_LAUNCH();
        if (sr) OASIS_TRY(loop.start(at, keep));
        return OASIS_OK;
    };
    auto fold = [&]() -> int {
        hipLaunchKernelGGL(k_add_lo, dim3(gv), dim3(kBlock), 0, s, n, x, xlo);
        OASIS_TRY_LAUNCH();
        return OASIS_OK;
    };
    OASIS_TRY(replace(0));
    CGState h;
    OASIS_TRY(read_state(s, w.stage, w.st, &h, sizeof(h)));
    const double wbb = h.wbb, tol2 = h.tol2;
    auto rel = [&](double wrr) { return wbb > 0.0 ? std::sqrt(wrr / wbb) : std::sqrt(wrr); };
    if (!std::isfinite(h.wrr)) {
        out.status = OASIS_ENAN;
        out.rel_res = NAN;
        return out.status;
    }
    if (h.wrr <= tol2) {
        out.rel_res = rel(h.wrr);
        return OASIS_OK;
    }
    OASIS_TRY(cast(0, false));
    ChunkPlan plan(check_every);
    plan.restart(h.wrr, 0, std::max(h.upd2, tol2));
    int it = 0, restart_at = 0, nin = gv;     // partials of k_cg_cast first, then of k_cg_p2
    int rc = OASIS_OK;
    while (true) {
        const int m = std::min(plan.next, maxit - it);
        for (int j = 0; j < m; ++j) {
            const int itj = it + j;
            if (sr) {
                loop.iterate(itj, itj == restart_at ? 1 : 0, xlo);
                OASIS_TRY_LAUNCH();
                continue;
            }
            const int ni = j == 0 ? nin : g.p2;
            if (ell)
                launch_p1_ell<float, BS>(s, cap, n, w.cols, w.eval, w.pair[itj & 1], w.pair[(itj + 1) & 1], w.q,
                                         w.partB, ni, 2, w.st, itj, itj == restart_at ? 1 : 0, vnull, w.partA);
            else
                hipLaunchKernelGGL((k_cg_p1<float, C, BS>), dim3(g1), dim3(BS), 0, s, n, rp, ci, val32,
                                   w.pair[itj & 1], w.pair[(itj + 1) & 1], w.q, w.partB, ni, 2, w.st, itj,
                                   itj == restart_at ? 1 : 0, vnull, w.partA);
            OASIS_TRY_LAUNCH();
            hipLaunchKernelGGL((k_cg_p2<float, BS>), dim3(g.p2), dim3(BS), 0, s, n, w.pair[(itj + 1) & 1], w.q,
                               xlo, wgt32, w.partA, g1, w.st, itj, vnull, w.partB);
            OASIS_TRY_LAUNCH();
        }
        it += m;
        nin = g.p2;
        OASIS_TRY(read_state(s, w.stage, w.st, &h, sizeof(h)));
        if (h.flag == 2 || h.flag == 3) {
            OASIS_TRY(fold());
            out.iters = h.it_done;
            out.status = rc = (h.flag == 2) ? OASIS_EBREAKDOWN : OASIS_ENAN;
            out.rel_res = NAN;
            break;
        }
        if (h.flag == 0 && it < maxit) {
            plan.observe(h.wrr_it, h.it_last, std::max(h.upd2, tol2));
            continue;
        }
        // replacement: fold x_lo into x, FP64 residual, test, FP32 copy
        const int at = h.flag == 0 ? it : h.it_done;
        OASIS_TRY(fold());
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
            if (time_kernel && sr) {
                // repeat iteration `at` from the replaced residual; x_lo is
                // left alone (the repeats advance a scratch copy)
                OASIS_TRY(cast(at, true));
                OASIS_TRY(time_product(s, maxit, [&] { loop.iterate(at, 0, w.q); }, out));
            } else if (time_kernel) {
                // repeat iteration `at` (FP32 pair in place, k_cg_init's partials)
                OASIS_TRY(time_product(
                    s, maxit,
                    [&] {
                        if (ell)
                            launch_p1_ell<float, BS>(s, cap, n, w.cols, w.eval, w.pair[at & 1],
                                                     w.pair[(at + 1) & 1], w.q, w.partB, gi, 3, w.st, at, 0, vnull,
                                                     w.partA);
                        else
                            hipLaunchKernelGGL((k_cg_p1<float, C, BS>), dim3(g1), dim3(BS), 0, s, n, rp, ci, val32,
                                               w.pair[at & 1], w.pair[(at + 1) & 1], w.q, w.partB, gi, 3, w.st, at,
                                               0, vnull, w.partA);
                    },
                    out));
            }
            break;
        }
        OASIS_TRY(cast(at, true));
        plan.restart(h.wrr, at, std::max(h.upd2, tol2));
        it = at;
        nin = gv;
    }
    return rc;
}

int cg_mixed_solve(hipStream_t s, int n, const int *rp, const int *ci, const double *val,
                   const float *val32, const double *wgt, const float *wgt32, const float *vnull,
                   double vscale, const double *b, double *x, double rtol, double delta, int maxit,
                   int check_every, bool time_kernel, CGWork<float> &w, float *xlo, double *rhi,
                   SolveOut &out) {
    return with_cfg([&](auto c) {
        return cg_mixed_run<decltype(c), kBlock>(s, n, rp, ci, val, val32, wgt, wgt32, vnull, vscale, b, x, rtol,
                                                 delta, maxit, check_every, time_kernel, w, xlo, rhi, out);
    });
}

template <typename T>
static int product_launch(hipStream_t s, int cap, int n, const int *rp, const int *ci, const T *val,
                          const EllCols &cols, const T *eval, const RP<T> *cur, RP<T> *nxt, T *q,
                          const double *partIn, int nIn, int stride, CGState *st, int it, int beta_zero,
                          double *partOut, int *grid) {
    if (cols.any() && eval) {
        *grid = launch_p1_ell<T, kBlock>(s, cap, n, cols, eval, cur, nxt, q, partIn, nIn, stride, st, it,
                                         beta_zero, static_cast<const T *>(nullptr), partOut);
    } else {
        using C = Cfg4x4x1;
        *grid = grid_for(n, rows_per_block<C>(), kMaxPartials);
        hipLaunchKernelGGL((k_cg_p1<T, C, kBlock>), dim3(*grid), dim3(kBlock), 0, s, n, rp, ci, val, cur, nxt,
                           q, partIn, nIn, stride, st, it, beta_zero, static_cast<const T *>(nullptr), partOut);
    }
    OASIS_TRY_LAUNCH();
    return OASIS_OK;
}

int cg_product_launch(hipStream_t s, int cap, int n, const int *rp, const int *ci, const double *val,
                      const EllCols &cols, const double *eval, const RP<double> *cur, RP<double> *nxt, double *q,
                      const double *partIn, int nIn, int stride, CGState *st, int it, int beta_zero,
                      double *partOut, int *grid) {
    return product_launch<double>(s, cap, n, rp, ci, val, cols, eval, cur, nxt, q, partIn, nIn, stride, st, it,
                                  beta_zero, partOut, grid);
}

int cg_product_launch(hipStream_t s, int cap, int n, const int *rp, const int *ci, const float *val,
                      const EllCols &cols, const float *eval, const RP<float> *cur, RP<float> *nxt, float *q,
                      const double *partIn, int nIn, int stride, CGState *st, int it, int beta_zero,
                      double *partOut, int *grid) {
    return product_launch<float>(s, cap, n, rp, ci, val, cols, eval, cur, nxt, q, partIn, nIn, stride, st, it,
                                 beta_zero, partOut, grid);
}

int cg_residual_state(hipStream_t s, int cap, int n, const int *rp, const int *ci, const double *val,
                      const EllCols &cols, const double *wgt, const double *b, const double *x, double *r, int rs,
                      double *part, CGState *st, double rtol2, int mode, double upd_factor) {
    using C = Cfg4x4x1;
    const int g = grid_for(n, rows_per_block<C>(), cap);
    hipLaunchKernelGGL((k_cg_init<double, C>), dim3(g), dim3(kBlock), 0, s, n, rp, ci, val, cols, wgt, b, x, r, rs,
                       part);
    OASIS_TRY_LAUNCH();
    hipLaunchKernelGGL(k_cg_finalize, dim3(1), dim3(kBlock), 0, s, part, g, st, rtol2, mode, upd_factor);
    OASIS_TRY_LAUNCH();
    return OASIS_OK;
}

int cg_residual(hipStream_t s, int n, const int *rp, const int *ci, const double *val,
                const double *wgt, const double *b, const double *x, double *r,
                CGWork<double> &w, double *wrr, double *wbb) {
    const int g1 = grid_for(n, rows_per_block<Cfg8x2x1>(), w.tun.grid_cap);
    hipLaunchKernelGGL((k_cg_init<double, Cfg8x2x1>), dim3(g1), dim3(kBlock), 0, s, n, rp, ci, val,
                       w.tun.ell() ? w.cols : EllCols{}, wgt, b, x, r, 1, w.partB);
    OASIS_TRY_LAUNCH();
    hipLaunchKernelGGL(k_cg_finalize, dim3(1), dim3(kBlock), 0, s, w.partB, g1, w.st, 1.0, 0, 0.0);
    OASIS_TRY_LAUNCH();
    CGState h;
    OASIS_TRY(read_state(s, w.stage, w.st, &h, sizeof(h)));
    *wrr = h.wrr;
    *wbb = h.wbb;
    return OASIS_OK;
}

// ---------------------------------------------------------------------------
// BiCGStab kernels (nr right-hand sides share every pass over the matrix)
//
// Events raised per right-hand side (any event pauses all of them):
//   1 converged candidate (||r|| test)      2 rho = 0 or omega = 0
//   3 non-finite value                      4 (r_hat, v) = 0
//   5 converged candidate at the s stage

template <typename T>
struct V3 {
    T *p[3];
};
template <typename T>
struct C3 {
    const T *p[3];
};

// r_k = b_k - As xsrc_k for k in mask_res; r_hat_k = r_k for k in mask_rhat;
// partials (r_hat.r, sum wgt r^2, sum wgt b^2) for every k.  The residual
// is the first half of the (r, u) pair; u is left as it is.
template <typename T, int NR, class C>
__global__ __launch_bounds__(kBlock) void k_bi_resid(int n, Mat<T> m,
                                                     const T *__restrict__ wgt, C3<T> b,
                                                     C3<T> xsrc, RW<T> *ru, V3<T> rhat, int mask_res,
                                                     int mask_rhat, double *part) {
    __shared__ double lds[9 * kBlock / kWave];
    double acc[3 * NR];
#pragma unroll
    for (int k = 0; k < 3 * NR; ++k) acc[k] = 0.0;
    // every right-hand side is gathered (no branch per k, so that the loads
    // of all of them are in flight together); finish uses only those in
    // mask_res.  The row's own inputs are read for every k as well.
    struct Own {
        T w, b[NR], r[NR], h[NR];
    };
    auto own = [&](long long row) {
        Own o;
        o.w = wgt[row];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            o.b[k] = b.p[k][row];
            o.r[k] = ru[row * NR + k].r;
            o.h[k] = rhat.p[k][row];
        }
        return o;
    };
    auto fin = [&](int row, int lane, T(&a)[NR], const Own &o) {
        if (lane != 0) return;
        const double wd = o.w;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            T rk;
            if ((mask_res >> k) & 1) {
                rk = o.b[k] - a[k];
                ru[(long long)row * NR + k].r = rk;
            } else {
                rk = o.r[k];
            }
            T hk;
            if ((mask_rhat >> k) & 1) {
                rhat.p[k][row] = rk;
                hk = rk;
            } else {
                hk = o.h[k];
            }
            const double rd = rk, bd = o.b[k];
            acc[3 * k + 0] += static_cast<double>(hk) * rd;
            acc[3 * k + 1] += wd * rd * rd;
            acc[3 * k + 2] += wd * bd * bd;
        }
    };
    if (m.eval) {
        struct G {
            T x[NR];
        };
        auto load = [&](int c) {
            G g;
#pragma unroll
            for (int k = 0; k < NR; ++k) g.x[k] = xsrc.p[k][c];
            return g;
        };
        auto add = [&](const G &g, T v, T(&a)[NR]) {
#pragma unroll
            for (int k = 0; k < NR; ++k) a[k] += v * g.x[k];
        };
        if (m.cols.pid)
            ell_rows_pipe<T, NR, 2, true, G, Own>(n, m.cols, m.eval, load, add, own, fin);
        else
            ell_rows_pipe<T, NR, 2, false, G, Own>(n, m.cols, m.eval, load, add, own, fin);
    } else {
        csr_rows<T, NR, C>(
            n, m.rp, m.ci, m.val,
            [&](int, int c, T v, bool ok, T(&a)[NR]) {
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    const T t = v * xsrc.p[k][c];
                    a[k] += ok ? t : T(0);
                }
            },
            [&](int row, int lane, T(&a)[NR]) {
                if (lane != 0) return;
                fin(row, lane, a, own(row));
            });
    }
    write_partials<3 * NR>(acc, part, lds);
}

template <int NR>
__global__ __launch_bounds__(kBlock) void k_bi_finalize(const double *part, int nparts, BiState *st,
                                                        double rtol2, int mode) {
    __shared__ double lds[9 * kBlock / kWave];
    double v[3 * NR];
    read_partials<3 * NR>(part, nparts, v, lds);
    if (threadIdx.x == 0) {
        for (int k = 0; k < NR; ++k) {
            if (mode == 0) {
                st[k].tol2 = rtol2 * v[3 * k + 2];
                st[k].wbb = v[3 * k + 2];
            }
            st[k].wrr = v[3 * k + 1];
        }
    }
}

__device__ __forceinline__ void bi_pause(BiGlobal *g, int phase, int it) {
    g->phase = phase;
    g->pause_it = it;
    g->pause = 1;
}

// part 1: tests on the incoming residual, p = r + beta u (u = p_old -
// omega v_old, formed by part 3), v = As p, partial r_hat.v.  Writes p and
// the (r, v) pairs that part 2 gathers; reads nothing it writes, so a
// relaunch after a pause recomputes the same values.
template <typename T, int NR, class C>
__global__ __launch_bounds__(kBlock) void k_bi_1(int n, Mat<T> m, const RW<T> *ru, C3<T> rhat,
                                                 V3<T> p, RW<T> *rv, const double *partIn, int nIn,
                                                 BiState *st, BiGlobal *glob, int it,
                                                 double *partOut) {
    __shared__ double lds[9 * kBlock / kWave];
    if (block_read_flag(&glob->pause)) return;
    double v[3 * NR];
    read_partials<3 * NR>(partIn, nIn, v, lds);
    const int prev = (it + 1) & 1;
    int ev[NR];
    int any = 0;
    int active = 0;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        ev[k] = 0;
        if (!st[k].active) continue;
        active |= 1 << k;
        const double rr = v[3 * k], wrr = v[3 * k + 1];
        if (!finite(rr) || !finite(wrr))
            ev[k] = 3;
        else if (wrr <= st[k].tol2)
            ev[k] = 1;
        else if (rr == 0.0 || st[k].omega[prev] == 0.0)
            ev[k] = 2;
        any |= ev[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < NR; ++k)
            if ((active >> k) & 1) {
                st[k].wrr_rec = v[3 * k + 1];
                st[k].it_rec = it;
            }
    }
    if (any) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            for (int k = 0; k < NR; ++k)
                if (ev[k]) st[k].event = ev[k];
            bi_pause(glob, 1, it);
        }
        return;
    }
    T beta[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const double rr = v[3 * k];
        beta[k] = static_cast<T>((rr / st[k].rho[prev]) * (st[k].alpha[prev] / st[k].omega[prev]));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < NR; ++k)
            if ((active >> k) & 1) st[k].rho[it & 1] = v[3 * k];
    }
    double acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = 0.0;
    // all right-hand sides, active or not: branch-free, so that the gathers
    // of one entry are issued together (finish discards the inactive ones)
    struct Own {
        RW<T> me[NR];
        T hk[NR];
    };
    auto fin = [&](int row, int lane, T(&a)[NR], const Own &o) {
        if (lane != 0) return;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (!((active >> k) & 1)) continue;
            p.p[k][row] = fmadd(beta[k], o.me[k].w, o.me[k].r);
            rv[(long long)row * NR + k] = RW<T>{o.me[k].r, a[k]};
            acc[k] += static_cast<double>(o.hk[k]) * static_cast<double>(a[k]);
        }
    };
    auto own = [&](long long row) {
        Own o;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            o.me[k] = ru[row * NR + k];
            o.hk[k] = rhat.p[k][row];
        }
        return o;
    };
    if (m.eval) {
        // ELL copy: the straight-line row loop with the own-row state prefetched
        struct G {
            RW<T> g[NR];
        };
        auto load = [&](int c) {
            G x;
#pragma unroll
            for (int k = 0; k < NR; ++k) x.g[k] = ru[(long long)c * NR + k];
            return x;
        };
        auto add = [&](const G &g, T vv, T(&a)[NR]) {
#pragma unroll
            for (int k = 0; k < NR; ++k) a[k] += vv * fmadd(beta[k], g.g[k].w, g.g[k].r);
        };
        if (m.cols.pid)
            ell_rows_pipe<T, NR, 2, true, G, Own>(n, m.cols, m.eval, load, add, own, fin);
        else
            ell_rows_pipe<T, NR, 2, false, G, Own>(n, m.cols, m.eval, load, add, own, fin);
    } else {
        csr_rows<T, NR, C>(
            n, m.rp, m.ci, m.val,
            [&](int, int c, T vv, bool ok, T(&a)[NR]) {
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    const RW<T> g = ru[(long long)c * NR + k];
                    const T t = vv * fmadd(beta[k], g.w, g.r);
                    a[k] += ok ? t : T(0);
                }
            },
            [&](int row, int lane, T(&a)[NR]) {
                if (lane != 0) return;
                fin(row, lane, a, own(row));
            });
    }
    write_partials<NR>(acc, partOut, lds);
}

// part 2: alpha = rho / (r_hat.v), s = r - alpha v, t = As s,
// partials (t.s, t.t, sum wgt s^2).  s itself is not stored: part 3 forms
// it again from the same (r, v) pair with the same rounding.
template <typename T, int NR, class C>
__global__ __launch_bounds__(kBlock) void k_bi_2(int n, Mat<T> m, const T *__restrict__ wgt,
                                                 const RW<T> *rv, V3<T> t, const double *partIn, int nIn,
                                                 BiState *st, BiGlobal *glob, int it,
                                                 double *partOut) {
    __shared__ double lds[9 * kBlock / kWave];
    if (block_read_flag(&glob->pause)) return;
    double v[NR];
    read_partials<NR>(partIn, nIn, v, lds);
    const int cur = it & 1;
    int ev[NR];
    int any = 0, active = 0;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        ev[k] = 0;
        if (!st[k].active) continue;
        active |= 1 << k;
        if (!finite(v[k]))
            ev[k] = 3;
        else if (v[k] == 0.0)
            ev[k] = 4;
        any |= ev[k];
    }
    if (any) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            for (int k = 0; k < NR; ++k)
                if (ev[k]) st[k].event = ev[k];
            bi_pause(glob, 2, it);
        }
        return;
    }
    T al[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) al[k] = static_cast<T>(st[k].rho[cur] / v[k]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < NR; ++k)
            if ((active >> k) & 1) st[k].alpha[cur] = st[k].rho[cur] / v[k];
    }
    double acc[3 * NR];
#pragma unroll
    for (int k = 0; k < 3 * NR; ++k) acc[k] = 0.0;
    // branch-free over the right-hand sides (see k_bi_1)
    struct Own {
        RW<T> mv[NR];
        T w;
    };
    auto fin = [&](int row, int lane, T(&a)[NR], const Own &o) {
        if (lane != 0) return;
        const double wd = o.w;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (!((active >> k) & 1)) continue;
            const RW<T> me = o.mv[k];
            const T sn = fmsub(me.r, al[k], me.w);
            t.p[k][row] = a[k];
            const double sd = sn, td = a[k];
            acc[3 * k + 0] += td * sd;
            acc[3 * k + 1] += td * td;
            acc[3 * k + 2] += wd * sd * sd;
        }
    };
    auto own = [&](long long row) {
        Own o;
#pragma unroll
        for (int k = 0; k < NR; ++k) o.mv[k] = rv[row * NR + k];
        o.w = wgt[row];
        return o;
    };
    if (m.eval) {
        struct G {
            RW<T> g[NR];
        };
        auto load = [&](int c) {
            G x;
#pragma unroll
            for (int k = 0; k < NR; ++k) x.g[k] = rv[(long long)c * NR + k];
            return x;
        };
        auto add = [&](const G &g, T w, T(&a)[NR]) {
#pragma unroll
            for (int k = 0; k < NR; ++k) a[k] += w * fmsub(g.g[k].r, al[k], g.g[k].w);
        };
        if (m.cols.pid)
            ell_rows_pipe<T, NR, 2, true, G, Own>(n, m.cols, m.eval, load, add, own, fin);
        else
            ell_rows_pipe<T, NR, 2, false, G, Own>(n, m.cols, m.eval, load, add, own, fin);
    } else {
        csr_rows<T, NR, C>(
            n, m.rp, m.ci, m.val,
            [&](int, int c, T w, bool ok, T(&a)[NR]) {
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    const RW<T> g = rv[(long long)c * NR + k];
                    const T tk = w * fmsub(g.r, al[k], g.w);
                    a[k] += ok ? tk : T(0);
                }
            },
            [&](int row, int lane, T(&a)[NR]) {
                if (lane != 0) return;
                fin(row, lane, a, own(row));
            });
    }
    write_partials<3 * NR>(acc, partOut, lds);
}

// part 3: s-stage test, omega = (t.s)/(t.t), s = r - alpha v,
// x += alpha p + omega s, r = s - omega t and u = p - omega v for the next
// direction; partials (r_hat.r, sum wgt r^2, 0)
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void k_bi_3(int n, const T *__restrict__ wgt, V3<T> x,
                                                 RW<T> *ru, C3<T> rhat, C3<T> p, const RW<T> *rv,
                                                 C3<T> t, const double *partIn, int nIn,
                                                 BiState *st, BiGlobal *glob, int it,
                                                 double *partOut) {
    __shared__ double lds[9 * kBlock / kWave];
    if (block_read_flag(&glob->pause)) return;
    double v[3 * NR];
    read_partials<3 * NR>(partIn, nIn, v, lds);
    const int cur = it & 1;
    int ev[NR];
    int any = 0, active = 0;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        ev[k] = 0;
        if (!st[k].active) continue;
        active |= 1 << k;
        if (v[3 * k + 2] <= st[k].tol2 && st[k].no_sexit_it != it) ev[k] = 5;
        any |= ev[k];
    }
    if (any) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            for (int k = 0; k < NR; ++k)
                if (ev[k]) {
                    st[k].event = ev[k];
                    st[k].wrr_rec = v[3 * k + 2];   // weighted |s|^2
                }
            bi_pause(glob, 3, it);
        }
        return;
    }
    T al[NR], om[NR];
    double omd[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const double ts = v[3 * k], tt = v[3 * k + 1];
        omd[k] = tt > 0.0 ? ts / tt : 0.0;
        om[k] = static_cast<T>(omd[k]);
        al[k] = static_cast<T>(st[k].alpha[cur]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < NR; ++k)
            if ((active >> k) & 1) st[k].omega[cur] = omd[k];
    }
    double acc[3 * NR];
#pragma unroll
    for (int k = 0; k < 3 * NR; ++k) acc[k] = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double wd = wgt[i];
        // loads for every right-hand side first (no branch per k, so they are
        // in flight together); stores and partials only for the active ones
        RW<T> g[NR];
        T pk[NR], tk[NR], xk[NR], hk[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            g[k] = rv[i * NR + k];
            pk[k] = p.p[k][i];
            tk[k] = t.p[k][i];
            xk[k] = x.p[k][i];
            hk[k] = rhat.p[k][i];
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const bool on = (active >> k) & 1;
            const T sk = fmsub(g[k].r, al[k], g[k].w);
            const T rk = fmsub(sk, om[k], tk[k]);
            if (on) {
                x.p[k][i] = xk[k] + al[k] * pk[k] + om[k] * sk;
                ru[i * NR + k] = RW<T>{rk, fmsub(pk[k], om[k], g[k].w)};
                const double rd = rk;
                acc[3 * k + 0] += static_cast<double>(hk[k]) * rd;
                acc[3 * k + 1] += wd * rd * rd;
            }
        }
    }
    write_partials<3 * NR>(acc, partOut, lds);
}

// xs_k = x_k + alpha_k p_k for k in mask (s-stage candidates)
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void k_bi_xs(int n, C3<T> x, C3<T> p, V3<T> xs,
                                                  const BiState *st, int it, int mask) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < NR; ++k)
            if ((mask >> k) & 1)
                xs.p[k][i] = x.p[k][i] + static_cast<T>(st[k].alpha[it & 1]) * p.p[k][i];
    }
}

// u = 0 in every (r, u) pair: the next direction is the residual itself
template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero_u(int n, RW<T> *ru, int nr, int k) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        ru[i * nr + k].w = T(0);
}

// The start from x = 0: x = 0, r = r_hat = b, u = 0, and the partials
// (r_hat.r, sum wgt r^2, sum wgt b^2) that k_bi_resid would give.
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void k_bi_start0(int n, const T *__restrict__ wgt, C3<T> b, V3<T> x,
                                                      RW<T> *ru, V3<T> rhat, double *part) {
    __shared__ double lds[9 * kBlock / kWave];
    double acc[3 * NR];
#pragma unroll
    for (int k = 0; k < 3 * NR; ++k) acc[k] = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double wd = wgt[i];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const T bk = b.p[k][i];
            x.p[k][i] = T(0);
            ru[i * NR + k] = RW<T>{bk, T(0)};
            rhat.p[k][i] = bk;
            const double bd = bk;
            acc[3 * k + 0] += bd * bd;
            acc[3 * k + 1] += wd * bd * bd;
            acc[3 * k + 2] += wd * bd * bd;
        }
    }
    write_partials<3 * NR>(acc, part, lds);
}

// k_bi_resid with no residual to recompute (mask_res = 0): r_hat_k = r_k
// for k in mask_rhat and the partials (r_hat.r, sum wgt r^2, sum wgt b^2)
// from the vectors as they are, without the product.
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void k_bi_parts(int n, const T *__restrict__ wgt, C3<T> b, const RW<T> *ru,
                                                     V3<T> rhat, int mask_rhat, double *part) {
    __shared__ double lds[9 * kBlock / kWave];
    double acc[3 * NR];
#pragma unroll
    for (int k = 0; k < 3 * NR; ++k) acc[k] = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double wd = wgt[i];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const T rk = ru[i * NR + k].r;
            T hk;
            if ((mask_rhat >> k) & 1) {
                rhat.p[k][i] = rk;
                hk = rk;
            } else {
                hk = rhat.p[k][i];
            }
            const double rd = rk, bd = b.p[k][i];
            acc[3 * k + 0] += static_cast<double>(hk) * rd;
            acc[3 * k + 1] += wd * rd * rd;
            acc[3 * k + 2] += wd * bd * bd;
        }
    }
    write_partials<3 * NR>(acc, part, lds);
}

template <typename T>
void carve_bi(Carver &c, int n, int nrhs, BiWork<T> &w) {
    std::memset(&w, 0, sizeof(w));
    w.ru = c.take<RW<T>>((size_t)n * nrhs);
    w.rv = c.take<RW<T>>((size_t)n * nrhs);
    for (int k = 0; k < nrhs; ++k) {
        w.p[k] = c.take<T>(n);
        w.rhat[k] = c.take<T>(n);
        w.t[k] = c.take<T>(n);
        w.xs[k] = c.take<T>(n);
    }
    w.part1 = c.take<double>(9 * kMaxPartials);
    w.part2 = c.take<double>(9 * kMaxPartials);
    w.part3 = c.take<double>(9 * kMaxPartials);
    BiBlock *blk = c.take<BiBlock>(1);
    w.st = blk ? blk->st : nullptr;
    w.glob = blk ? &blk->glob : nullptr;
}

template <typename T, int NR, class C>
static int bi_run(hipStream_t s, int n, const int *rp, const int *ci, const T *val, const T *wgt,
                  const T *const *b, T *const *x, double rtol, int maxit, int check_every,
                  bool time_kernel, BiWork<T> &w, SolveOut *out, bool inner) {
    const int g1 = grid_for(n, rows_per_block<C>(), w.tun.grid_cap);
    const int g2 = grid_for(n, kBlock, w.tun.grid_cap);
    const int gv = grid_for(n, kBlock, 4096);
    const bool ell = w.cols.any() && w.eval && w.tun.ell();
    const Mat<T> mat{rp, ci, val, ell ? w.cols : EllCols{}, ell ? w.eval : nullptr};
    C3<T> cb{}, cx{}, crh{}, ct{}, cp{};
    V3<T> vx{}, vrh{}, vt{}, vp{}, vxs{};
    for (int k = 0; k < NR; ++k) {
        cb.p[k] = b[k];
        cx.p[k] = x[k];
        vx.p[k] = x[k];
        crh.p[k] = vrh.p[k] = w.rhat[k];
        ct.p[k] = vt.p[k] = w.t[k];
        cp.p[k] = vp.p[k] = w.p[k];
        vxs.p[k] = w.xs[k];
    }
    BiBlock hb{};
    BiState(&hs)[3] = hb.st;
    BiGlobal &hg = hb.glob;
    for (int k = 0; k < 3; ++k) {
        hs[k] = BiState{};
        for (int q = 0; q < 2; ++q) hs[k].rho[q] = hs[k].alpha[q] = hs[k].omega[q] = 1.0;
        hs[k].active = k < NR ? 1 : 0;
        hs[k].no_sexit_it = -1;
        out[k < NR ? k : 0] = SolveOut();
    }
    // one copy each way: the states and the pause record share a block
    BiBlock *dblk = reinterpret_cast<BiBlock *>(w.st);
    auto push_state = [&]() -> int { return write_state(s, w.stage, dblk, &hb, sizeof(hb)); };
    auto pull_state = [&]() -> int { return read_state(s, w.stage, dblk, &hb, sizeof(hb)); };
    auto zero_dirs = [&](int k) -> int {
        hipLaunchKernelGGL((k_zero_u<T>), dim3(gv), dim3(kBlock), 0, s, n, w.ru, NR, k);
        OASIS_TRY_LAUNCH();
        return OASIS_OK;
    };
    auto resid = [&](int mask_res, int mask_rhat, C3<T> src) -> int {
        if (mask_res == 0)   // partials only (same grid, so finalize and k_bi_1 read g1 of them)
            hipLaunchKernelGGL((k_bi_parts<T, NR>), dim3(g1), dim3(kBlock), 0, s, n, wgt, cb, w.ru, vrh, mask_rhat,
                               w.part3);
        else
            hipLaunchKernelGGL((k_bi_resid<T, NR, C>), dim3(g1), dim3(kBlock), 0, s, n, mat, wgt,
                               cb, src, w.ru, vrh, mask_res, mask_rhat, w.part3);
        OASIS_TRY_LAUNCH();
        return OASIS_OK;
    };
    auto finalize = [&](int mode) -> int {
        hipLaunchKernelGGL((k_bi_finalize<NR>), dim3(1), dim3(kBlock), 0, s, w.part3, g1, w.st,
                           rtol * rtol, mode);
        OASIS_TRY_LAUNCH();
        return OASIS_OK;
    };
    const int all = (1 << NR) - 1;
    OASIS_TRY(push_state());
    if (inner) {
        // the grid of the product kernels, whose partial count finalize reads
        hipLaunchKernelGGL((k_bi_start0<T, NR>), dim3(g1), dim3(kBlock), 0, s, n, wgt, cb, vx, w.ru, vrh, w.part3);
        OASIS_TRY_LAUNCH();
    } else {
        for (int k = 0; k < NR; ++k) OASIS_TRY(zero_dirs(k));
        OASIS_TRY(resid(all, all, cx));
    }
    OASIS_TRY(finalize(0));
    // The start residuals are not read back here: k_bi_1 tests them like
    // any other, and the first poll brings the norms with the states.
    double wbb[3] = {0, 0, 0}, tol2[3] = {0, 0, 0};
    bool known = false;
    auto rel = [&](int k, double wrr) { return wbb[k] > 0 ? std::sqrt(wrr / wbb[k]) : std::sqrt(wrr); };
    // Iterations to launch before the next poll.  Each right-hand side's
    // convergence rate (log of the weighted residual per iteration, from
    // its last restart to the latest recursive residual k_bi_1 recorded)
    // predicts the iteration at which the slowest active one meets its
    // tolerance; the launch reaches one past it, within [1, chunk].  A
    // launch past the pause costs kernels that return at once, a short one
    // another poll.  Before any rate is known: `chunk`.
    double lref[3] = {0, 0, 0}, lrate[3] = {0, 0, 0};
    int itref[3] = {0, 0, 0};
    auto set_ref = [&](int k, double wrr, int at) {
        lref[k] = wrr > 0.0 ? std::log(wrr) : 0.0;
        itref[k] = at;
    };
    auto learn = [&]() {
        if (known) return;
        known = true;
        for (int k = 0; k < NR; ++k) {
            wbb[k] = hs[k].wbb;
            tol2[k] = hs[k].tol2;
            set_ref(k, hs[k].wrr, 0);   // wrr: the start residual's until a finalize(1)
        }
    };
    auto observe = [&]() {
        for (int k = 0; k < NR; ++k) {
            if (!hs[k].active || hs[k].it_rec <= itref[k] || !(hs[k].wrr_rec > 0.0) || !std::isfinite(hs[k].wrr_rec))
                continue;
            const double r = (std::log(hs[k].wrr_rec) - lref[k]) / (hs[k].it_rec - itref[k]);
            if (r < 0.0) lrate[k] = r;
        }
    };
    int restarted[3] = {0, 0, 0};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (time_kernel) {
        OASIS_TRY_HIP(hipEventCreate(&e0));
        OASIS_TRY_HIP(hipEventCreate(&e1));
    }
    const int chunk = check_every > 0 ? check_every : 8;
    auto plan = [&](int at) -> int {
        if (check_every > 0) return chunk;
        int last = at;   // the iteration whose k_bi_1 should see convergence
        for (int k = 0; k < NR; ++k) {
            if (!hs[k].active) continue;
            if (!(lrate[k] < 0.0) || !(tol2[k] > 0.0)) return chunk;
            // the latest known point: the recorded recursive residual, or
            // the reference set at the last (re)start
            double lw = lref[k];
            int itw = itref[k];
            if (hs[k].it_rec > itref[k] && hs[k].wrr_rec > 0.0 && std::isfinite(hs[k].wrr_rec)) {
                lw = std::log(hs[k].wrr_rec);
                itw = hs[k].it_rec;
            }
            const double need = (std::log(tol2[k]) - lw) / lrate[k];
            const int j = itw + static_cast<int>(std::ceil(std::max(0.0, need)));
            last = std::max(last, j);
        }
        return std::min(chunk, std::max(1, last - at + 2));
    };
    int it = 0, phase = 1;
    int next = chunk;
    int part3_count = g1;
    auto n_active = [&]() {
        int a = 0;
        for (int k = 0; k < NR; ++k) a += hs[k].active;
        return a;
    };
    auto restart = [&](int k, int pit, int &mask_rhat) -> int {
        if (restarted[k]) {
            hs[k].active = 0;
            out[k].status = OASIS_EBREAKDOWN;
            out[k].iters = pit;
            return OASIS_OK;
        }
        restarted[k] = 1;
        out[k].replacements += 1;
        OASIS_TRY(zero_dirs(k));
        const int prev = (pit + 1) & 1;
        hs[k].rho[prev] = hs[k].alpha[prev] = hs[k].omega[prev] = 1.0;
        mask_rhat |= 1 << k;
        set_ref(k, hs[k].wrr, pit);
        return OASIS_OK;
    };
    while (n_active() > 0) {
        // enqueue up to `chunk` iterations
        int launched = 0;
        while (launched < next && it < maxit) {
            if (phase == 1) {
                if (time_kernel) OASIS_TRY_HIP(hipEventRecord(e0, s));
                hipLaunchKernelGGL((k_bi_1<T, NR, C>), dim3(g1), dim3(kBlock), 0, s, n, mat,
                                   w.ru, crh, vp, w.rv, w.part3, part3_count, w.st, w.glob, it,
                                   w.part1);
                OASIS_TRY_LAUNCH();
                if (time_kernel) {
                    OASIS_TRY_HIP(hipEventRecord(e1, s));
                    OASIS_TRY_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    OASIS_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
                    out[0].kernel_ms += ms;
                    out[0].kernel_count += 1;
                }
                hipLaunchKernelGGL((k_bi_2<T, NR, C>), dim3(g1), dim3(kBlock), 0, s, n, mat,
                                   wgt, w.rv, vt, w.part1, g1, w.st, w.glob, it, w.part2);
                OASIS_TRY_LAUNCH();
            }
            hipLaunchKernelGGL((k_bi_3<T, NR>), dim3(g2), dim3(kBlock), 0, s, n, wgt, vx, w.ru, crh,
                               cp, w.rv, ct, w.part2, g1, w.st, w.glob, it, w.part3);
            OASIS_TRY_LAUNCH();
            part3_count = g2;
            phase = 1;
            ++it;
            ++launched;
        }
        OASIS_TRY(pull_state());
        learn();
        observe();
        if (!hg.pause) {
            if (it < maxit) {
                next = plan(it);
                continue;
            }
            // iteration cap: confirm with the explicit residual
            int mask = 0;
            for (int k = 0; k < NR; ++k)
                if (hs[k].active) mask |= 1 << k;
            OASIS_TRY(resid(mask, 0, cx));
            OASIS_TRY(finalize(1));
            OASIS_TRY(pull_state());
            for (int k = 0; k < NR; ++k) {
                if (!((mask >> k) & 1)) continue;
                out[k].iters = it;
                out[k].rel_res = rel(k, hs[k].wrr);
                out[k].status = hs[k].wrr <= tol2[k] ? OASIS_OK : OASIS_ENOTCONV;
                hs[k].active = 0;
            }
            break;
        }
        const int pit = hg.pause_it, ph = hg.phase;
        int mask_rhat = 0;
        if (ph == 1 || ph == 2) {
            int cands = 0;
            for (int k = 0; k < NR; ++k)
                if (hs[k].active && hs[k].event == 1) cands |= 1 << k;
            if (cands && inner) {
                // the recursive residual is trusted (the caller's FP64 residual decides)
                for (int k = 0; k < NR; ++k) {
                    if (!((cands >> k) & 1)) continue;
                    hs[k].active = 0;
                    out[k].status = OASIS_OK;
                    out[k].iters = pit;
                    out[k].rel_res = rel(k, hs[k].wrr_rec);
                }
                cands = 0;
            }
            // a check leaves in part3 the partials of every residual as it
            // now is (k_bi_resid sums all right-hand sides)
            const bool checked = cands != 0;
            if (cands) {
                OASIS_TRY(resid(cands, 0, cx));
                OASIS_TRY(finalize(1));
                OASIS_TRY(pull_state());
                for (int k = 0; k < NR; ++k) {
                    if (!((cands >> k) & 1)) continue;
                    if (hs[k].wrr <= tol2[k]) {
                        hs[k].active = 0;
                        out[k].status = OASIS_OK;
                        out[k].iters = pit;
                        out[k].rel_res = rel(k, hs[k].wrr);
                    } else {
                        out[k].replacements += 1;
                        set_ref(k, hs[k].wrr, pit);   // the explicit residual replaced the recursive one
                    }
                }
            }
            for (int k = 0; k < NR; ++k) {
                if (!hs[k].active) continue;
                if (hs[k].event == 3) {
                    hs[k].active = 0;
                    out[k].status = OASIS_ENAN;
                    out[k].iters = pit;
                    out[k].rel_res = NAN;
                } else if (hs[k].event == 2 || hs[k].event == 4) {
                    OASIS_TRY(restart(k, pit, mask_rhat));
                }
            }
            for (int k = 0; k < NR; ++k) hs[k].event = 0;
            hg = BiGlobal{};
            if (n_active() == 0) break;
            OASIS_TRY(push_state());
            // k_bi_1 of pit reads partials of the residuals as they now are:
            // those of k_bi_3 of pit - 1, of the check, or (r_hat reset on a
            // restart) of a partials pass
            if (mask_rhat) {
                OASIS_TRY(resid(0, mask_rhat, cx));
                part3_count = g1;
            } else if (checked) {
                part3_count = g1;
            }
            it = pit;
            phase = 1;
            next = plan(it);
        } else {
            int cands = 0;
            for (int k = 0; k < NR; ++k)
                if (hs[k].active && hs[k].event == 5) cands |= 1 << k;
            if (inner) {
                // x += alpha p in place, on the norm of s alone
                hipLaunchKernelGGL((k_bi_xs<T, NR>), dim3(gv), dim3(kBlock), 0, s, n, cx, cp, vx, w.st, pit, cands);
                OASIS_TRY_LAUNCH();
                for (int k = 0; k < NR; ++k) {
                    if (!((cands >> k) & 1)) continue;
                    hs[k].active = 0;
                    out[k].status = OASIS_OK;
                    out[k].iters = pit + 1;
                    out[k].rel_res = rel(k, hs[k].wrr_rec);
                }
                for (int k = 0; k < NR; ++k) hs[k].event = 0;
                hg = BiGlobal{};
                if (n_active() == 0) break;
                OASIS_TRY(push_state());
                it = pit;
                phase = 3;
                next = plan(it);
                continue;
            }
            hipLaunchKernelGGL((k_bi_xs<T, NR>), dim3(gv), dim3(kBlock), 0, s, n, cx, cp, vxs,
                               w.st, pit, cands);
            OASIS_TRY_LAUNCH();
            C3<T> src = cx;
            for (int k = 0; k < NR; ++k)
                if ((cands >> k) & 1) src.p[k] = w.xs[k];
            OASIS_TRY(resid(cands, 0, src));
            OASIS_TRY(finalize(1));
            OASIS_TRY(pull_state());
            for (int k = 0; k < NR; ++k) {
                if (!((cands >> k) & 1)) continue;
                if (hs[k].wrr <= tol2[k]) {
                    hipLaunchKernelGGL((k_copy<T>), dim3(gv), dim3(kBlock), 0, s, n, x[k], w.xs[k]);
                    OASIS_TRY_LAUNCH();
                    hs[k].active = 0;
                    out[k].status = OASIS_OK;
                    out[k].iters = pit + 1;
                    out[k].rel_res = rel(k, hs[k].wrr);
                } else {
                    hs[k].no_sexit_it = pit;
                    out[k].replacements += 1;
                }
            }
            for (int k = 0; k < NR; ++k) hs[k].event = 0;
            hg = BiGlobal{};
            if (n_active() == 0) break;
            OASIS_TRY(push_state());
            it = pit;
            phase = 3;
            next = plan(it);
        }
    }
    // no synchronisation here: callers go on in stream order (the
    // stand-alone entry point synchronises itself)
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    int worst = OASIS_OK;
    for (int k = 0; k < NR; ++k)
        if (out[k].status != OASIS_OK && (worst == OASIS_OK || out[k].status < worst)) worst = out[k].status;
    return worst;
}

template <typename T>
int bicgstab_solve(hipStream_t s, int n, int nrhs, const int *rp, const int *ci, const T *val,
                   const T *wgt, const T *const *b, T *const *x, double rtol, int maxit,
                   int check_every, bool time_kernel, BiWork<T> &w, SolveOut *out, bool inner) {
    return with_cfg([&](auto c) {
        using C = decltype(c);
        if (nrhs == 1)
            return bi_run<T, 1, C>(s, n, rp, ci, val, wgt, b, x, rtol, maxit, check_every, time_kernel, w, out,
                                   inner);
        if (nrhs == 2)
            return bi_run<T, 2, C>(s, n, rp, ci, val, wgt, b, x, rtol, maxit, check_every, time_kernel, w, out,
                                   inner);
        return bi_run<T, 3, C>(s, n, rp, ci, val, wgt, b, x, rtol, maxit, check_every, time_kernel, w, out,
                               inner);
    });
}

template void carve_cg<double>(Carver &, int, CGWork<double> &);
template void carve_cg<float>(Carver &, int, CGWork<float> &);
template void carve_bi<double>(Carver &, int, int, BiWork<double> &);
template void carve_bi<float>(Carver &, int, int, BiWork<float> &);
template int cg_solve<double>(hipStream_t, int, const int *, const int *, const double *,
                              const double *, const double *, double *, double, int, int, bool,
                              CGWork<double> &, SolveOut &);
template int cg_solve<float>(hipStream_t, int, const int *, const int *, const float *,
                             const float *, const float *, float *, double, int, int, bool,
                             CGWork<float> &, SolveOut &);
template int bicgstab_solve<double>(hipStream_t, int, int, const int *, const int *,
                                    const double *, const double *, const double *const *,
                                    double *const *, double, int, int, bool, BiWork<double> &,
                                    SolveOut *, bool);
template int bicgstab_solve<float>(hipStream_t, int, int, const int *, const int *, const float *,
                                   const float *, const float *const *, float *const *, double,
                                   int, int, bool, BiWork<float> &, SolveOut *, bool);

}  // namespace oasis
