// CSR row-group iteration used by every sparse product in the library.
//
// A group of L consecutive lanes owns R consecutive rows at a time.  Each
// lane takes the entries s + lane + p*L (p < P) of every one of its R rows;
// all R*P value/column loads and the dependent operand gathers are issued
// back to back from clamped (always valid) addresses, and out-of-row
// entries are discarded with a select, so a lane keeps R*P independent
// memory streams in flight instead of walking a data-dependent loop.  Rows
// longer than P*L finish in a short tail loop.  The L partial sums of a row
// are combined with a fixed-order xor butterfly (deterministic).  Rows are
// visited grid-stride so that a producer kernel can run at a bounded grid
// and emit one partial per block.
#pragma once

#include "internal.hpp"

namespace oasis {

template <int L_, int P_, int R_>
struct RowCfg {
    static constexpr int L = L_;   // lanes per row (divides 64)
    static constexpr int P = P_;   // unrolled entries per lane
    static constexpr int R = R_;   // rows per group in flight
};

// Compile-time switch for the XCD-aware row mapping below (a macro so that
// a build can compare both).
#ifndef OASIS_XCD_MAP
#define OASIS_XCD_MAP 1
#endif
__device__ __forceinline__ constexpr bool xcd_mapping() { return OASIS_XCD_MAP != 0; }

// Sum over the L lanes of a group (L divides 64); all lanes get the sum.
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
    return v;
}

// gather(j, col, val_j, ok, acc) adds the contribution of entry j when ok
// (j and col are valid indices even when !ok); finish(row, lane, acc) runs
// on all L lanes of the group after the butterfly (lane 0 writes).
//
// XCD-aware mapping: workgroups are dispatched to the 8 XCDs round-robin
// (block b runs on XCD b % 8), and each XCD has its own L2.  When the grid
// is a multiple of 8, the blocks of XCD k walk only the k-th contiguous
// eighth of the rows, so the operand entries they gather (rows plus a
// bandwidth-sized halo) stay in that XCD's L2 instead of every L2 holding
// the whole moving window.
constexpr int kXcds = 8;

// Rows [first, last) walked by lane group gid of ngroups (groups of L
// lanes), with the XCD-aware split when the grid allows it.
template <int L, int BS = kBlock>
struct RowRange {
    long long first = 0, last = 0, gid = 0, ngroups = 1;
    __device__ __forceinline__ explicit RowRange(int n) {
        constexpr int GPB = BS / L;                   // groups per block
        first = 0;
        last = n;
        if (xcd_mapping() && (gridDim.x % kXcds) == 0 && gridDim.x >= kXcds) {
            const int x = blockIdx.x % kXcds;
            const long long seg = (n + kXcds - 1) / kXcds;
            first = x * seg;
            last = first + seg < n ? first + seg : n;
            gid = static_cast<long long>(blockIdx.x / kXcds) * GPB + threadIdx.x / L;
            ngroups = static_cast<long long>(gridDim.x / kXcds) * GPB;
        } else {
            gid = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) / L;
            ngroups = (static_cast<long long>(gridDim.x) * blockDim.x) / L;
        }
    }
};

template <typename TA, int NR, class C, int BS = kBlock, class Gather, class Finish>
__device__ __forceinline__ void csr_rows(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                         const TA *__restrict__ val, Gather gather, Finish finish) {
    constexpr int L = C::L, P = C::P, R = C::R;
    const int lane = threadIdx.x & (L - 1);
    const RowRange<L, BS> rr(n);
    const long long first = rr.first, last = rr.last, gid = rr.gid, ngroups = rr.ngroups;
    for (long long row0 = first + gid * R; row0 < last; row0 += ngroups * R) {
        int s[R], e[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const long long row = row0 + r;
            const bool in = row < last;
            s[r] = in ? rp[row] : 0;
            e[r] = in ? rp[row + 1] : 0;
        }
        TA acc[R][NR];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < NR; ++k) acc[r][k] = TA(0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int j = s[r] + lane + p * L;
                const bool ok = j < e[r];
                const int jj = ok ? j : (e[r] > s[r] ? s[r] : 0);
                gather(jj, ci[jj], val[jj], ok, acc[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            for (int j = s[r] + P * L + lane; j < e[r]; j += L) gather(j, ci[j], val[j], true, acc[r]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int k = 0; k < NR; ++k) acc[r][k] = group_sum<L>(acc[r][k]);
            if (row0 + r < last) finish(static_cast<int>(row0 + r), lane, acc[r]);
        }
    }
}

// ELL storage for matrices whose rows have at most kEll entries (P1 meshes
// made of Kuhn-split hexahedra have at most 15): row i occupies entries
// [kEll i, kEll i + kEll) of a column and a value array, padded with
// (column i, value 0).  Columns are stored as 16-bit cyclic offsets
// d = (c - i) taken into [-n/2, n/2), which fit whenever the matrix's
// cyclic bandwidth is below 2^15 (the periodic channel's structured
// numbering: one x-y layer; after RCM: about 1.3 layers).  The product
// loops give each of L lanes of a row kEll / L consecutive entries,
// fetched with 8-byte offset and 16-byte value loads (no row pointers).
constexpr int kEll = 16;

// Column offsets of an ELL copy: per entry (ecol, n x kEll), or per row
// through a dictionary (pid: pattern id of each row; ptab: kEll offsets per
// pattern) when the rows share few distinct offset lists, as on structured
// meshes, where the offsets then cost 2 bytes per row instead of 32.
struct EllCols {
    const short *ecol = nullptr;
    const unsigned short *pid = nullptr;
    const short *ptab = nullptr;
    __host__ __device__ bool any() const { return ecol != nullptr || pid != nullptr; }
    __device__ __forceinline__ const short *offsets(long long row) const {
        return pid ? ptab + static_cast<int>(pid[row]) * kEll : ecol + row * kEll;
    }
};

__device__ __forceinline__ int ell_col(long long row, int d, int n) {
    int c = static_cast<int>(row) + d;
    c += c < 0 ? n : 0;
    c -= c >= n ? n : 0;
    return c;
}

__device__ __forceinline__ void load4(const float *__restrict__ p, float (&v)[4]) {
    const float4 t = *reinterpret_cast<const float4 *>(p);
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
}
// four FP16 values widened to FP32 (one 8-byte load)
struct alignas(8) Half4 {
    _Float16 h[4];
};
__device__ __forceinline__ void load4(const _Float16 *__restrict__ p, float (&v)[4]) {
    const Half4 t = *reinterpret_cast<const Half4 *>(p);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = static_cast<float>(t.h[k]);
}
__device__ __forceinline__ void load4(const double *__restrict__ p, double (&v)[4]) {
    const double2 a = reinterpret_cast<const double2 *>(p)[0];
    const double2 b = reinterpret_cast<const double2 *>(p)[1];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
}

// The csr_rows contract on the ELL copy, L lanes per row: gather(j, c, v,
// ok, acc) for each of the row's kEll stored entries (padding: c = row,
// v = 0, ok = true) and finish(row, lane, acc) on all L lanes after the
// butterfly.  Rows are walked grid-stride, so any grid covers them.
// Offsets (decoded to columns) and values of one lane's E entries of row
// `row` of an ELL copy.
// TS: the stored value type (TA, or FP16 widened to an FP32 TA)
template <typename TA, int E, typename TS = TA>
__device__ __forceinline__ void ell_fetch_at(const short *off, long long row, int lane, int n,
                                             const TS *__restrict__ eval, int (&c)[E], TA (&w)[E]) {
    const long long base = row * kEll + lane * E;
    off += lane * E;
#pragma unroll
    for (int g = 0; g < E / 4; ++g) {
        const short4 d = *reinterpret_cast<const short4 *>(off + 4 * g);
        c[4 * g] = ell_col(row, d.x, n);
        c[4 * g + 1] = ell_col(row, d.y, n);
        c[4 * g + 2] = ell_col(row, d.z, n);
        c[4 * g + 3] = ell_col(row, d.w, n);
        TA t[4];
        load4(eval + base + 4 * g, t);
#pragma unroll
        for (int k = 0; k < 4; ++k) w[4 * g + k] = t[k];
    }
}

template <typename TA, int E>
__device__ __forceinline__ void ell_fetch(long long row, int lane, int n, const EllCols &cols,
                                          const TA *__restrict__ eval, int (&c)[E], TA (&w)[E]) {
    ell_fetch_at<TA, E>(cols.offsets(row), row, lane, n, eval, c, w);
}

// The same fetch split in two for row loops that run the pattern-id load
// one row further ahead: ell_key reads a row's key (its pattern id; 0
// without a dictionary) and ell_fetch_key the row's offsets and values given
// that key.  DICT fixes the column storage at compile time, so that such a
// loop is straight-line code whose outstanding loads the compiler counts
// exactly (a run-time choice merges two paths and makes it wait for all).
template <bool DICT>
__device__ __forceinline__ int ell_key(const EllCols &cols, long long row) {
    if constexpr (DICT)
        return cols.pid[row];
    else
        return 0;
}

template <bool DICT, typename TA, int E, typename TS = TA>
__device__ __forceinline__ void ell_fetch_key(long long row, int key, int lane, int n, const EllCols &cols,
                                              const TS *__restrict__ eval, int (&c)[E], TA (&w)[E]) {
    const short *off = DICT ? cols.ptab + key * kEll : cols.ecol + row * kEll;
    ell_fetch_at<TA, E, TS>(off, row, lane, n, eval, c, w);
}

// The row loop is software-pipelined: the next row's offsets and values are
// fetched while this row's gathers are in flight.
template <typename TA, int NR, int L, int BS = kBlock, class Gather, class Finish>
__device__ __forceinline__ void ell_rows(int n, const EllCols &cols, const TA *__restrict__ eval,
                                         Gather gather, Finish finish) {
    constexpr int E = kEll / L;
    static_assert(E % 4 == 0, "lanes per row must leave a multiple of 4 entries per lane");
    const int lane = threadIdx.x & (L - 1);
    const RowRange<L, BS> rr(n);
    long long row = rr.first + rr.gid;
    int c[E];
    TA w[E];
    if (row < rr.last) ell_fetch<TA, E>(row, lane, n, cols, eval, c, w);
    for (; row < rr.last; row += rr.ngroups) {
        TA acc[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = TA(0);
#pragma unroll
        for (int k = 0; k < E; ++k) gather(0, c[k], w[k], true, acc);
        const long long nrow = row + rr.ngroups;
        if (nrow < rr.last) ell_fetch<TA, E>(nrow, lane, n, cols, eval, c, w);
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = group_sum<L>(acc[k]);
        finish(static_cast<int>(row), lane, acc);
    }
}

// ell_rows as straight-line code (the row loop of the CG iteration
// kernels): while a row's operand gathers are in flight, every lane fetches
// the next row's offsets, values and own(row), the inputs of the row's
// finish step, from row indices clamped into the lane group's range; the
// pattern id comes one row further ahead, and the loop alternates two
// register sets so that no loaded value is copied across the back edge.
// The gather is split in two: load(c) -> G reads the operand(s) of column c
// and add(g, v, acc) adds one entry's contribution (padding has value 0);
// finish(row, lane, acc, o) runs on all L lanes with o = own(row).
// The stored values may be FP16 (TS) for an FP32 TA; they are widened on load.
template <typename TA, int NR, int L, bool DICT, class G, class O, class TS, class Load, class Add, class Own,
          class Finish>
__device__ __forceinline__ void ell_rows_pipe(int n, const EllCols &cols, const TS *__restrict__ eval, Load load,
                                              Add add, Own own, Finish finish) {
    constexpr int E = kEll / L;
    static_assert(E % 4 == 0, "lanes per row must leave a multiple of 4 entries per lane");
    const int lane = threadIdx.x & (L - 1);
    const RowRange<L> rr(n);
    long long row = rr.first + rr.gid;
    if (row >= rr.last) return;
    const long long top = rr.last - 1;
    auto clamp = [top](long long r) { return r < top ? r : top; };
    struct Stage {
        int c[E];
        TA w[E];
        O o;
    };
    auto fetch = [&](Stage &S, long long r, int key) {
        ell_fetch_key<DICT, TA, E, TS>(r, key, lane, n, cols, eval, S.c, S.w);
        S.o = own(r);
    };
    auto step = [&](const Stage &S, Stage &N, int kin, int &kout) {
        G g[E];
#pragma unroll
        for (int k = 0; k < E; ++k) g[k] = load(S.c[k]);
        TA wv[E];
#pragma unroll
        for (int k = 0; k < E; ++k) wv[k] = S.w[k];
        const O o = S.o;
        fetch(N, clamp(row + rr.ngroups), kin);
        kout = ell_key<DICT>(cols, clamp(row + 2 * rr.ngroups));
        TA acc[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = TA(0);
#pragma unroll
        for (int k = 0; k < E; ++k) add(g[k], wv[k], acc);
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = group_sum<L>(acc[k]);
        finish(static_cast<int>(row), lane, acc, o);
    };
    Stage A, B;
    int ka, kb;
    fetch(A, row, ell_key<DICT>(cols, row));
    ka = ell_key<DICT>(cols, clamp(row + rr.ngroups));
    for (;;) {
        step(A, B, ka, kb);
        row += rr.ngroups;
        if (row >= rr.last) break;
        step(B, A, kb, ka);
        row += rr.ngroups;
        if (row >= rr.last) break;
    }
}

// The csr_rows contract for CSR values whose columns come from an ELL
// copy's column storage (the offset dictionary or per-entry offsets): slot
// k of row i is CSR entry rp[i] + k, so the values are read in CSR order
// and the int32 column array is not read at all.  L lanes per row, kEll / L
// slots per lane, loads from clamped addresses; slots past the row's
// length are passed with ok = false.
template <typename TA, int NR, int L, int BS = kBlock, class Gather, class Finish>
__device__ __forceinline__ void csr_cols_rows(int n, const int *__restrict__ rp, const TA *__restrict__ val,
                                              const EllCols &cols, Gather gather, Finish finish) {
    constexpr int E = kEll / L;
    static_assert(E % 4 == 0, "lanes per row must leave a multiple of 4 slots per lane");
    const int lane = threadIdx.x & (L - 1);
    const RowRange<L, BS> rr(n);
    for (long long row = rr.first + rr.gid; row < rr.last; row += rr.ngroups) {
        const int s = rp[row], len = rp[row + 1] - s;
        const short *off = cols.offsets(row) + lane * E;
        int c[E];
        TA w[E];
        bool ok[E];
#pragma unroll
        for (int g = 0; g < E / 4; ++g) {
            const short4 d = *reinterpret_cast<const short4 *>(off + 4 * g);
            c[4 * g] = ell_col(row, d.x, n);
            c[4 * g + 1] = ell_col(row, d.y, n);
            c[4 * g + 2] = ell_col(row, d.z, n);
            c[4 * g + 3] = ell_col(row, d.w, n);
        }
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int slot = lane * E + k;
            ok[k] = slot < len;
            w[k] = val[s + (ok[k] ? slot : 0)];
        }
        TA acc[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = TA(0);
#pragma unroll
        for (int k = 0; k < E; ++k) gather(s + lane * E + k, c[k], w[k], ok[k], acc);
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = group_sum<L>(acc[k]);
        finish(static_cast<int>(row), lane, acc);
    }
}

// A matrix on the shared CSR pattern with an optional ELL copy (columns
// and eval both set) that products use instead.
template <typename T>
struct Mat {
    const int *rp;
    const int *ci;
    const T *val;
    EllCols cols;
    const T *eval;
};

template <typename TA, int NR, class C, class Gather, class Finish>
__device__ __forceinline__ void mat_rows(int n, const Mat<TA> &m, Gather gather, Finish finish) {
    if (m.eval)
        ell_rows<TA, NR, 2>(n, m.cols, m.eval, gather, finish);
    else
        csr_rows<TA, NR, C>(n, m.rp, m.ci, m.val, gather, finish);
}

// Row-iteration shapes of the CSR kernels.
using Cfg4x4x1 = RowCfg<4, 4, 1>;
using Cfg8x2x1 = RowCfg<8, 2, 1>;

template <class C, int BS = kBlock>
constexpr int rows_per_block() { return (BS / C::L) * C::R; }

// Call f with the CSR row shape of the general kernels: 4 lanes x 4
// unrolled entries x 1 row per lane group (the fastest of 8x2x1, 4x4x1,
// 8x2x2, 16x1x2 and 16x1x4 on the P1 patterns here).
template <class F>
auto with_cfg(F &&f) {
    return f(Cfg4x4x1{});
}

}  // namespace oasis
