// Internal helpers shared by the library's translation units: error
// plumbing, workspace carving, deterministic wave/block reductions and the
// "consumer reduces" pattern used to hand a global sum from one kernel to
// the next without atomics or cross-block fences.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "oasis.h"

namespace oasis {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kMaxPartials = 2048;   // producer kernels launch at most this many blocks

void set_hip_error(hipError_t e);

#define OASIS_TRY_HIP(call)                                  \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) {                              \
            ::oasis::set_hip_error(e_);                      \
            return OASIS_EHIP;                               \
        }                                                    \
    } while (0)

#define OASIS_TRY_LAUNCH() OASIS_TRY_HIP(hipGetLastError())

#define OASIS_TRY(expr)                  \
    do {                                 \
        int rc_ = (expr);                \
        if (rc_ != OASIS_OK) return rc_; \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Per-call storage and kernel-shape choices (oasis_tuning, validated).
struct Tuning {
    int storage = OASIS_STORAGE_AUTO;
    int grid_cap = kMaxPartials / 4;   // 512: two blocks per CU, one round
    int cg_form = OASIS_CG_FORM_AUTO;
    bool ell() const { return storage != OASIS_STORAGE_CSR; }
    bool dict() const { return storage == OASIS_STORAGE_AUTO; }
    // single-reduction CG iterations for values of tbytes bytes
    bool single(int tbytes) const {
        return cg_form == OASIS_CG_FORM_SINGLE || (cg_form == OASIS_CG_FORM_AUTO && tbytes == 4);
    }
    // EINVAL on out-of-range fields; a null pointer gives the defaults
    static int from(const oasis_tuning *t, Tuning *out) {
        Tuning v;
        if (t) {
            if (t->storage < OASIS_STORAGE_AUTO || t->storage > OASIS_STORAGE_CSR) return OASIS_EINVAL;
            if (t->cg_form < OASIS_CG_FORM_AUTO || t->cg_form > OASIS_CG_FORM_SINGLE) return OASIS_EINVAL;
            if (t->grid_cap != 0 && (t->grid_cap < 64 || t->grid_cap > kMaxPartials)) return OASIS_EINVAL;
            v.storage = t->storage;
            v.cg_form = t->cg_form;
            if (t->grid_cap) v.grid_cap = t->grid_cap;
        }
        *out = v;
        return OASIS_OK;
    }
};

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Sequential sub-allocation of a caller workspace.  With base == nullptr it
// only measures; the same sequence of take() calls is used for both.
struct Carver {
    char *base;
    size_t cap;
    size_t off = 0;
    bool ok = true;
    Carver(void *b, size_t c) : base(static_cast<char *>(b)), cap(c) {}
    template <class T>
    T *take(size_t count) {
        size_t a = (off + 255) & ~size_t(255);
        size_t need = a + count * sizeof(T);
        off = need;
        if (base == nullptr) return nullptr;
        if (need > cap) {
            ok = false;
            return nullptr;
        }
        return reinterpret_cast<T *>(base + a);
    }
    size_t bytes() const { return (off + 255) & ~size_t(255); }
};

// Blocks for `work` items at `per_block` each, at most `cap`; rounded up to
// a multiple of 8 (one share per XCD) once there are at least 8.
inline int grid_for(long long work, int per_block, int cap = kMaxPartials) {
    long long g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g >= 8) g = (g + 7) / 8 * 8;
    if (g > cap) g = cap / 8 * 8;
    return static_cast<int>(g);
}

// ---------------------------------------------------------------------------
// device reductions (fixed order => bitwise deterministic)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum NV values over the block; every thread receives the totals.
// lds must hold NV * (blockDim/64) doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k * nw + wid] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[k * nw + w];
        v[k] = s;
    }
    __syncthreads();
}

// Producer side: the block's NV partial sums go to part[blockIdx.x][NV].
template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double *part, double *lds) {
    block_sum<NV>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) part[blockIdx.x * NV + k] = v[k];
    }
}

// Consumer side: every block sums the nparts partials of the previous kernel
// in the same order, so all blocks hold identical totals.
// For up to three values per block the loads are unrolled so that a thread
// issues all of its (at most kMaxPartials / kBlock) loads at once: one
// cache round trip, not eight.  Wider partials are read two blocks at a
// time, in rounds that are kept apart so that the registers held in flight
// stay bounded (the kernel's register count, and so its occupancy, is the
// maximum over all of its code).  `stride` (>= NV) is the producer's values
// per block when the consumer needs only its first NV.
template <int NV, int BS = kBlock>
__device__ __forceinline__ void read_partials(const double *part, int nparts, double (&out)[NV],
                                              double *lds, int stride = NV) {
    constexpr int PER = kMaxPartials / BS;
    constexpr int U = NV <= 3 || PER < 2 ? PER : 2;
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = 0.0;
#pragma unroll 1
    for (int q0 = 0; q0 < PER; q0 += U) {
        double t[U][NV];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int i = threadIdx.x + (q0 + q) * BS;
#pragma unroll
            for (int k = 0; k < NV; ++k) t[q][k] = i < nparts ? part[i * stride + k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int k = 0; k < NV; ++k) out[k] += t[q][k];
    }
    block_sum<NV>(out, lds);
}

__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

// A small pinned, host-mapped block through which a solver's host loop
// reads its state back.  A one-block kernel copies the state into it and
// the host synchronises the stream: one kernel round trip, where a copy to
// pageable memory also stages through the runtime.  A handle owns one
// (stage_alloc at create, stage_free at destroy); without it (h null) reads
// are copies to the caller's host memory.  This is host memory: the
// library still allocates no device memory.
struct HostStage {
    void *h = nullptr;   // host address
    void *d = nullptr;   // the same memory as the device sees it
};
constexpr size_t kStageBytes = 1024;
void stage_alloc(HostStage &st);   // best effort: stays null on failure
void stage_free(HostStage &st);
// bytes (a multiple of 4) of device memory at dev into host memory at out;
// synchronises the stream
int read_state(hipStream_t s, const HostStage &st, const void *dev, void *out, size_t bytes);
// bytes (a multiple of 4) of host memory at src into device memory at dev,
// in stream order, without synchronising: through the block when there is
// one (the host fills it and a one-block kernel copies it over; the block
// is next written by a read_state, after this copy in stream order), else
// as an ordinary copy
int write_state(hipStream_t s, const HostStage &st, void *dev, const void *src, size_t bytes);

}  // namespace oasis
