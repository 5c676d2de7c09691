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

template <typename TA, int NR, class C, class Gather, class Finish>
__device__ __forceinline__ void csr_rows(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                         const TA *__restrict__ val, Gather gather, Finish finish) {
    constexpr int L = C::L, P = C::P, R = C::R;
    constexpr int GPB = kBlock / L;                   // groups per block
    const int lane = threadIdx.x & (L - 1);
    long long first = 0, last = n, gid, ngroups;
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

// Row-iteration shapes compiled into the library (selected at run time).
using Cfg4x4x1 = RowCfg<4, 4, 1>;
using Cfg8x2x1 = RowCfg<8, 2, 1>;
using Cfg8x2x2 = RowCfg<8, 2, 2>;
using Cfg16x1x2 = RowCfg<16, 1, 2>;
using Cfg16x1x4 = RowCfg<16, 1, 4>;

// Selected shape (default 1): 0 = 8x2x1, 1 = 4x4x1, 2 = 8x2x2, 3 = 16x1x2, 4 = 16x1x4
int spmv_cfg();
// Upper bound on producer grids (partials read by every consumer block).
int partial_cap();

template <class C>
constexpr int rows_per_block() { return (kBlock / C::L) * C::R; }

// Dispatch a callable templated on the row shape.
template <class F>
auto with_cfg(F &&f) {
    switch (spmv_cfg()) {
        case 1: return f(Cfg4x4x1{});
        case 2: return f(Cfg8x2x2{});
        case 3: return f(Cfg16x1x2{});
        case 4: return f(Cfg16x1x4{});
        default: return f(Cfg8x2x1{});
    }
}

}  // namespace oasis
