// CSR row-group iteration used by every sparse product in the library.
//
// A group of L consecutive lanes owns one row at a time: the lanes stride
// over the row's entries (coalesced loads of val/col_idx), each multiplies
// by a gathered operand, and the L partial sums are combined with a
// fixed-order xor butterfly.  Rows are visited grid-stride, so a producer
// kernel can run at a bounded grid size and emit one partial per block.
#pragma once

#include "internal.hpp"

namespace oasis {

// Sum over the L lanes of a group (L divides 64); all lanes get the sum.
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
    return v;
}

// Visits every row once.  gather(j, col, val_j, acc) accumulates the
// contribution of entry j into the NR accumulators; finish(row, acc) is
// called by all L lanes of the group after the butterfly (lane == 0 is
// the designated writer).
template <typename TA, int NR, int L, class Gather, class Finish>
__device__ __forceinline__ void csr_rows(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                         const TA *__restrict__ val, Gather gather, Finish finish) {
    const int lane = threadIdx.x & (L - 1);
    const long long gid = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) / L;
    const long long ngroups = (static_cast<long long>(gridDim.x) * blockDim.x) / L;
    for (long long row = gid; row < n; row += ngroups) {
        const int s = rp[row];
        const int e = rp[row + 1];
        TA acc[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = TA(0);
        for (int j = s + lane; j < e; j += L) gather(j, ci[j], val[j], acc);
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = group_sum<L>(acc[k]);
        finish(static_cast<int>(row), lane, acc);
    }
}

// Rows per block-iteration for a given lanes-per-row choice.
template <int L>
constexpr int rows_per_block() { return kBlock / L; }

}  // namespace oasis
