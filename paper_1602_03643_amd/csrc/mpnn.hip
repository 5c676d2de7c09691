// Learned warm start for the pressure-correction solve (not in the paper):
// a message-passing network on the P1 mesh graph, trained and evaluated
// with the kernels below.
//
// Inputs per node (X, [N][6]): with r = b_phi - K phi_prev and D = diag K,
//   x0 = (D^-1 r) / sigma,  sigma = rms(D^-1 r)      (1 if zero)
//   x1 = (D^-1 b_phi) / rms(D^-1 b_phi)               (0 if zero)
//   x2 = phi_prev / rms(phi_prev)                      (0 if zero)
//   x3.. = coordinates mapped to [-1, 1] by the bounding box (0 if flat/absent)
// Network (32 features, 3 message-passing layers, residual):
//   h0 = relu(We x + ce)
//   a_l = Agg(h_l),  Agg(h)_i = sum_{j != i} w_ij h_j,  w_ij = -K_ij / K_ii
//   z_l = Ws_l h_l + Wn_l a_l + c_l,   h_{l+1} = h_l + relu(z_l)
//   delta = wd . h_3 + cd,   guess = phi_prev + sigma * delta
// Activations are stored in BF16; the dense layers run on MFMA
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation); aggregations accumulate
// in FP32.  With K held as Ks = S^-1 K S^-1 (S = diag(s), s = sqrt(diag K)),
// w_ij = -Ks_ij s_j / s_i, and the transposed aggregation used by the
// backward pass is AggT(y)_j = -s_j sum_{i != j} Ks_ji (y_i / s_i).
// Training loss: mean over nodes of (delta - (phi - phi_prev)/sigma)^2.
// All reductions are fixed-order (block partials, then one ordered sum).
#include <cmath>
#include <cstring>
#include <type_traits>

#include "internal.hpp"
#include "mpnn.hpp"
#include "spmv.hpp"

namespace oasis {

constexpr int kIn = OASIS_MPNN_IN;
constexpr int kHid = OASIS_MPNN_HID;
constexpr int kLayers = OASIS_MPNN_LAYERS;
constexpr int kNParam = OASIS_MPNN_NPARAM;
constexpr int kOffWe = 0, kOffCe = 192, kOffWs = 224, kOffWn = 3296, kOffC = 6368, kOffWd = 6464, kOffCd = 6496;
constexpr int kTile = 64;     // nodes per block tile (4 waves x 16)
constexpr int kGradBlocks = 256;

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
    // round to nearest even on the upper 16 bits
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(static_cast<unsigned>(b) << 16); }

__device__ __forceinline__ f4 mfma16(bf4 a, bf4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

struct MpWs {
    float *X;                          // [N][8]
    unsigned short *H[kLayers + 1];    // [N][32]
    unsigned short *Ag[kLayers];       // [N][32]
    unsigned short *Z[kLayers + 1];    // [N][32] pre-activations (z0 = encoder)
    float *delta;                      // [N]
    double *scal;                      // [16]: sigma, sig_u, sig_phi, lo[3], hi[3], eKe, tKt
    double *part;                      // [kMaxPartials][4]
    double *mm;                        // [kMaxPartials][6] min / max partials
    float *G;                          // [N][32]
    unsigned short *GZ, *Y;            // [N][32]
    float *gpart;                      // [kGradBlocks][kNParam]
    double *lpart;                     // [kGradBlocks]
    double *et;                        // [N][2] K-norm loss: (s e, s t)
    double *ke;                        // [N] K e
};

constexpr int kScalEKE = 9, kScalTKT = 10;

static void carve_mp(Carver &c, int n, MpWs &w) {
    w.X = c.take<float>((size_t)n * 8);
    for (int l = 0; l <= kLayers; ++l) {
        w.H[l] = c.take<unsigned short>((size_t)n * kHid);
        w.Z[l] = c.take<unsigned short>((size_t)n * kHid);
    }
    for (int l = 0; l < kLayers; ++l) w.Ag[l] = c.take<unsigned short>((size_t)n * kHid);
    w.delta = c.take<float>(n);
    w.scal = c.take<double>(16);
    w.part = c.take<double>(kMaxPartials * 4);
    w.mm = c.take<double>(kMaxPartials * 6);
    w.G = c.take<float>((size_t)n * kHid);
    w.GZ = c.take<unsigned short>((size_t)n * kHid);
    w.Y = c.take<unsigned short>((size_t)n * kHid);
    w.gpart = c.take<float>((size_t)kGradBlocks * kNParam);
    w.lpart = c.take<double>(kGradBlocks);
    w.et = c.take<double>((size_t)n * 2);
    w.ke = c.take<double>(n);
}

// ---------------------------------------------------------------------------
// features

// Rows 0..2 of m become their minimum, rows 3..5 their maximum, in column
// 0 (tree over the block; all threads take part).
__device__ __forceinline__ void block_minmax6(double (&m)[6][kBlock]) {
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const int t = threadIdx.x;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                m[k][t] = fmin(m[k][t], m[k][t + h]);
                m[3 + k][t] = fmax(m[3 + k][t], m[3 + k][t + h]);
            }
        }
        __syncthreads();
    }
}

// r = b - K phi_prev with K = S Ks S; X[:,0..2] = (r/d, b/d, phi_prev) raw,
// X[:,3..5] = coordinates; partials: sums of squares and coordinate min/max
template <class C>
__global__ __launch_bounds__(kBlock) void k_mp_feat1(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                     const double *__restrict__ Ks, const double *__restrict__ s,
                                                     const double *__restrict__ b, const double *__restrict__ phi,
                                                     const double *__restrict__ xyz, int dim, float *__restrict__ X,
                                                     double *part, double *mm) {
    __shared__ double lds[3 * kBlock / kWave];
    __shared__ double mml[6][kBlock];
    double acc[3] = {0.0, 0.0, 0.0};
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    csr_rows<double, 1, C>(
        n, rp, ci, Ks,
        [&](int, int c, double v, bool ok, double(&a)[1]) {
            const double t = v * s[c] * phi[c];
            a[0] += ok ? t : 0.0;
        },
        [&](int row, int lane, double(&a)[1]) {
            if (lane != 0) return;
            const double si = s[row], d = si * si;
            const double r = b[row] - si * a[0];
            const double t = r / d, u = b[row] / d, f = phi[row];
            float *x = X + (size_t)row * 8;
            x[0] = static_cast<float>(t);
            x[1] = static_cast<float>(u);
            x[2] = static_cast<float>(f);
            acc[0] += t * t;
            acc[1] += u * u;
            acc[2] += f * f;
            for (int k = 0; k < 3; ++k) {
                const double cv = k < dim ? xyz[(size_t)row * dim + k] : 0.0;
                x[3 + k] = static_cast<float>(cv);
                lo[k] = fmin(lo[k], cv);
                hi[k] = fmax(hi[k], cv);
            }
        });
    write_partials<3>(acc, part, lds);
    for (int k = 0; k < 3; ++k) {
        mml[k][threadIdx.x] = lo[k];
        mml[3 + k][threadIdx.x] = hi[k];
    }
    block_minmax6(mml);
    if (threadIdx.x < 6) mm[blockIdx.x * 6 + threadIdx.x] = mml[threadIdx.x][0];
}

// One block: sums of squares and bounding box from the per-block partials
// into scal = (rms t, rms u, rms phi_prev, lo[3], hi[3]); rms t = 1 if zero.
__global__ __launch_bounds__(kBlock) void k_mp_feat_reduce(int n, int np, const double *part, const double *mm,
                                                           double *scal) {
    __shared__ double lds[3 * kBlock / kWave];
    __shared__ double mml[6][kBlock];
    double v[3];
    read_partials<3>(part, np, v, lds);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < np; b += blockDim.x)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], mm[b * 6 + k]);
            hi[k] = fmax(hi[k], mm[b * 6 + 3 + k]);
        }
    for (int k = 0; k < 3; ++k) {
        mml[k][threadIdx.x] = lo[k];
        mml[3 + k][threadIdx.x] = hi[k];
    }
    block_minmax6(mml);
    if (threadIdx.x == 0) {
        const double st = sqrt(v[0] / n);
        scal[0] = st > 0.0 ? st : 1.0;
        scal[1] = sqrt(v[1] / n);
        scal[2] = sqrt(v[2] / n);
    }
    if (threadIdx.x < 6) scal[3 + threadIdx.x] = mml[threadIdx.x][0];
}

// normalised features, encoder h0 = relu(We x + ce), from scal; the BF16
// rows of Z0 and H0 (64 bytes per node) are written as 16-byte stores
// STORE: keep the normalised features and the encoder's pre-activation
// for the backward pass (inference needs only H0).
template <bool STORE>
__global__ __launch_bounds__(kBlock) void k_mp_feat2(int n, const double *__restrict__ scal,
                                                     const float *__restrict__ P, float *__restrict__ X,
                                                     unsigned short *__restrict__ Z0, unsigned short *__restrict__ H0) {
    __shared__ float W[kHid * kIn + kHid];
    for (int k = threadIdx.x; k < kHid * kIn + kHid; k += blockDim.x) W[k] = P[kOffWe + k];
    __syncthreads();
    const double st = scal[0], su = scal[1], sf = scal[2];
    double lo[3], span[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = scal[3 + k];
        span[k] = scal[6 + k] - scal[3 + k];
    }
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        float4 *x4 = reinterpret_cast<float4 *>(X + i * 8);
        const float4 a = x4[0], b = x4[1];
        float xn[8];
        xn[0] = static_cast<float>(a.x / st);
        xn[1] = su > 0.0 ? static_cast<float>(a.y / su) : 0.f;
        xn[2] = sf > 0.0 ? static_cast<float>(a.z / sf) : 0.f;
        const float raw[3] = {a.w, b.x, b.y};
        for (int k = 0; k < 3; ++k)
            xn[3 + k] = span[k] > 0.0 ? static_cast<float>(2.0 * (raw[k] - lo[k]) / span[k] - 1.0) : 0.f;
        xn[6] = xn[7] = 0.f;
        if (STORE) {
            x4[0] = make_float4(xn[0], xn[1], xn[2], xn[3]);
            x4[1] = make_float4(xn[4], xn[5], 0.f, 0.f);
        }
        uint4 *z = reinterpret_cast<uint4 *>(Z0 + i * kHid);
        uint4 *h = reinterpret_cast<uint4 *>(H0 + i * kHid);
#pragma unroll
        for (int q = 0; q < kHid / 8; ++q) {
            unsigned zw[4], hw[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                float v2[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int o = q * 8 + p * 2 + e;
                    float acc = W[kHid * kIn + o];
#pragma unroll
                    for (int k = 0; k < kIn; ++k) acc += W[o * kIn + k] * xn[k];
                    v2[e] = acc;
                }
                zw[p] = static_cast<unsigned>(f2bf(v2[0])) | (static_cast<unsigned>(f2bf(v2[1])) << 16);
                hw[p] = static_cast<unsigned>(f2bf(fmaxf(v2[0], 0.f))) |
                        (static_cast<unsigned>(f2bf(fmaxf(v2[1], 0.f))) << 16);
            }
            if (STORE) z[q] = make_uint4(zw[0], zw[1], zw[2], zw[3]);
            h[q] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        }
    }
}

// ---------------------------------------------------------------------------
// message-passing layer: aggregation, dense MFMA layer, residual; the
// decoder is fused into the last layer

// Weighted neighbour sum over off-diagonal entries of one row, 8 features
// per lane: out = -(1/s_i) sum_{j != i} Ks_ij s_j v_j  (gathered 16-byte rows)
__device__ __forceinline__ void agg8(int i, int f0, const int *__restrict__ rp, const int *__restrict__ ci,
                                     const double *__restrict__ Ks, const double *__restrict__ s,
                                     const unsigned short *__restrict__ V, bool scale_by_j, float (&out)[8]) {
    float acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.f;
    // edges in chunks of U: all loads of a chunk come from clamped (valid)
    // addresses and are issued together, then the chunk is accumulated in
    // edge order (the same sums as one edge at a time)
    constexpr int U = 8;
    const int e0 = rp[i], len = rp[i + 1] - e0;
    for (int c0 = 0; c0 < len; c0 += U) {
        int j[U];
        double kv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + (c0 + u < len ? c0 + u : len - 1);
            j[u] = ci[e];
            kv[u] = Ks[e];
        }
        uint4 q[U];
        double sj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            q[u] = *reinterpret_cast<const uint4 *>(V + (size_t)j[u] * kHid + f0);
            sj[u] = scale_by_j ? s[j[u]] : 1.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (c0 + u >= len || j[u] == i) continue;
            const float w = static_cast<float>(scale_by_j ? kv[u] * sj[u] : kv[u]);
            const unsigned qq[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                acc[2 * k] += w * bf2f(static_cast<unsigned short>(qq[k] & 0xffffu));
                acc[2 * k + 1] += w * bf2f(static_cast<unsigned short>(qq[k] >> 16));
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] = acc[k];
}

// Edge weights of the forward aggregation: W_e = Ks_e s_{col(e)} rounded to
// FP32, the weight agg8 forms per gathered entry; computed once per forward
// pass for all layers (agg8w then reads 4 bytes per edge instead of the FP64
// value and a gathered FP64 scale).
__global__ __launch_bounds__(kBlock) void k_mp_edge_w(long long nnz, const int *__restrict__ ci,
                                                      const double *__restrict__ Ks, const double *__restrict__ s,
                                                      float *__restrict__ W) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nnz;
         e += (long long)gridDim.x * blockDim.x)
        W[e] = static_cast<float>(Ks[e] * s[ci[e]]);
}

// agg8 with scale_by_j on precomputed edge weights (the same sums, bit for
// bit: the same FP32 weights accumulated in the same order).
__device__ __forceinline__ void agg8w(int i, int f0, const int *__restrict__ rp, const int *__restrict__ ci,
                                      const float *__restrict__ W, const unsigned short *__restrict__ V,
                                      float (&out)[8]) {
    float acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.f;
    constexpr int U = 8;
    const int e0 = rp[i], len = rp[i + 1] - e0;
    for (int c0 = 0; c0 < len; c0 += U) {
        int j[U];
        float w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + (c0 + u < len ? c0 + u : len - 1);
            j[u] = ci[e];
            w[u] = W[e];
        }
        uint4 q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) q[u] = *reinterpret_cast<const uint4 *>(V + (size_t)j[u] * kHid + f0);
        // the diagonal and the clamped tail get weight 0 instead of a branch:
        // adding 0 * (a finite feature) to a sum that started at +0 leaves it
        // unchanged, so the sums are those of agg8
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float wu = (c0 + u >= len || j[u] == i) ? 0.f : w[u];
            const unsigned qq[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                acc[2 * k] += wu * bf2f(static_cast<unsigned short>(qq[k] & 0xffffu));
                acc[2 * k + 1] += wu * bf2f(static_cast<unsigned short>(qq[k] >> 16));
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] = acc[k];
}

// LDS B operand for z = [h | a] W^T: B[k][o] with k < 32 -> Ws[o][k], k >= 32 -> Wn[o][k-32]
__device__ __forceinline__ void load_layer_weights(const float *__restrict__ P, int l, unsigned short (*B)[kHid]) {
    for (int q = threadIdx.x; q < 2 * kHid * kHid; q += blockDim.x) {
        const int k = q / kHid, o = q - k * kHid;
        const float w = k < kHid ? P[kOffWs + l * kHid * kHid + o * kHid + k]
                                 : P[kOffWn + l * kHid * kHid + o * kHid + (k - kHid)];
        B[k][o] = f2bf(w);
    }
}

// STORE: keep the activations (aggregate, pre-activation, and the last
// layer's output) for the backward pass; inference needs only the hidden
// state that the next layer reads.  EW: the aggregation reads the edge
// weights W of k_mp_edge_w.
template <bool LAST, bool STORE, bool EW>
__global__ __launch_bounds__(kBlock) void k_mp_layer(int n, int l, const int *__restrict__ rp,
                                                     const int *__restrict__ ci, const double *__restrict__ Ks,
                                                     const double *__restrict__ s, const float *__restrict__ W,
                                                     const float *__restrict__ P,
                                                     const unsigned short *__restrict__ Hin,
                                                     unsigned short *__restrict__ Aout,
                                                     unsigned short *__restrict__ Zout,
                                                     unsigned short *__restrict__ Hout, float *__restrict__ delta,
                                                     double *__restrict__ guess, const double *__restrict__ phi_prev,
                                                     const double *scal) {
    __shared__ unsigned short B[2 * kHid][kHid];
    __shared__ unsigned short T[kTile][2 * kHid + 8];   // [h | a] per node, padded rows
    __shared__ float cvec[kHid], wd[kHid];
    load_layer_weights(P, l, B);
    if (threadIdx.x < kHid) {
        cvec[threadIdx.x] = P[kOffC + l * kHid + threadIdx.x];
        wd[threadIdx.x] = P[kOffWd + threadIdx.x];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const float cd = P[kOffCd];
    for (long long base = (long long)blockIdx.x * kTile; base < n; base += (long long)gridDim.x * kTile) {
        __syncthreads();
        // aggregation: 4 threads per node, 8 features each
        {
            const int ln = threadIdx.x >> 2, f0 = (threadIdx.x & 3) * 8;
            const long long i = base + ln;
            if (i < n) {
                const uint4 hq = *reinterpret_cast<const uint4 *>(Hin + (size_t)i * kHid + f0);
                const double si = s[i];
                float a[8];
                if constexpr (EW)
                    agg8w(static_cast<int>(i), f0, rp, ci, W, Hin, a);
                else
                    agg8(static_cast<int>(i), f0, rp, ci, Ks, s, Hin, true, a);
                const float inv = static_cast<float>(-1.0 / si);
                const unsigned hv[4] = {hq.x, hq.y, hq.z, hq.w};
                unsigned av[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const unsigned lo = f2bf(a[2 * k] * inv), hi = f2bf(a[2 * k + 1] * inv);
                    av[k] = lo | (hi << 16);
                    T[ln][f0 + 2 * k] = static_cast<unsigned short>(hv[k] & 0xffffu);
                    T[ln][f0 + 2 * k + 1] = static_cast<unsigned short>(hv[k] >> 16);
                    T[ln][kHid + f0 + 2 * k] = static_cast<unsigned short>(lo);
                    T[ln][kHid + f0 + 2 * k + 1] = static_cast<unsigned short>(hi);
                }
                if (STORE)
                    *reinterpret_cast<uint4 *>(Aout + (size_t)i * kHid + f0) = make_uint4(av[0], av[1], av[2], av[3]);
            } else {
                for (int k = 0; k < 8; ++k) {
                    T[ln][f0 + k] = 0;
                    T[ln][kHid + f0 + k] = 0;
                }
            }
        }
        __syncthreads();
        // dense: wave wv owns nodes [16 wv, 16 wv + 16) of the tile
        const int r0 = wv * 16;
        const int m = lane & 15, kq = (lane >> 4) * 4;
        f4 acc[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
                bf4 af, bfr;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    af[q] = static_cast<short>(T[r0 + m][kt * 16 + kq + q]);
                    bfr[q] = static_cast<short>(B[kt * 16 + kq + q][nt * 16 + m]);
                }
                acc[nt] = mfma16(af, bfr, acc[nt]);
            }
        }
        // epilogue: rows r0 + kq + q, column nt*16 + m
        float dpart[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int o = nt * 16 + m;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ln = r0 + kq + q;
                const long long i = base + ln;
                const float z = acc[nt][q] + cvec[o];
                const float hn = bf2f(T[ln][o]) + fmaxf(z, 0.f);
                if (i < n) {
                    if (STORE) Zout[(size_t)i * kHid + o] = f2bf(z);
                    if (STORE || !LAST) Hout[(size_t)i * kHid + o] = f2bf(hn);
                }
                if (LAST) dpart[q] += bf2f(f2bf(hn)) * wd[o];
            }
        }
        if (LAST) {
            // sum over the 16 lanes that share rows (xor over the low 4 lane bits)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float v = dpart[q];
                for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
                dpart[q] = v;
            }
            if (m == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const long long i = base + r0 + kq + q;
                    if (i < n) {
                        const float d = dpart[q] + cd;
                        if (delta) delta[i] = d;
                        if (guess) guess[i] = phi_prev[i] + scal[0] * static_cast<double>(d);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// backward

// decoder: g_delta = 2 (delta - t) / N (mean squared error) or, with ke
// given, 2 (K e)_i / t^T K t (K-norm loss; 0 when t^T K t = 0), G =
// g_delta wd; partials of the loss (mean squared error only), g_wd, g_cd
__global__ __launch_bounds__(kBlock) void k_mp_bwd_dec(int n, const unsigned short *__restrict__ H3,
                                                       const float *__restrict__ delta, const double *__restrict__ phi,
                                                       const double *__restrict__ phi_prev, const double *scal,
                                                       const double *__restrict__ ke,
                                                       const float *__restrict__ P, float *__restrict__ G,
                                                       float *gpart, double *lpart) {
    __shared__ float red[kBlock];
    __shared__ double lred[kBlock];
    float gwd[kHid];
    for (int o = 0; o < kHid; ++o) gwd[o] = 0.f;
    float gcd = 0.f;
    double loss = 0.0;
    const double sig = scal[0];
    const double tkt = ke ? scal[kScalTKT] : 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        float gd;
        if (ke) {
            gd = tkt > 0.0 ? static_cast<float>(2.0 * ke[i] / tkt) : 0.f;
        } else {
            const double t = (phi[i] - phi_prev[i]) / sig;
            const double e = static_cast<double>(delta[i]) - t;
            loss += e * e;
            gd = static_cast<float>(2.0 * e / n);
        }
        gcd += gd;
        for (int o = 0; o < kHid; ++o) {
            G[i * kHid + o] = gd * P[kOffWd + o];
            gwd[o] += gd * bf2f(H3[i * kHid + o]);
        }
    }
    // block sums in a fixed order
    for (int o = 0; o <= kHid; ++o) {
        red[threadIdx.x] = o < kHid ? gwd[o] : gcd;
        __syncthreads();
        for (int st = kBlock / 2; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) gpart[(size_t)blockIdx.x * kNParam + (o < kHid ? kOffWd + o : kOffCd)] = red[0];
        __syncthreads();
    }
    lred[threadIdx.x] = loss;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) lred[threadIdx.x] += lred[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = lred[0];
}

// layer l, part 1: gz = G * [z_l > 0]; Y = (gz Wn_l) / s; weight-gradient
// partials g_Ws_l = sum gz^T h_l, g_Wn_l = sum gz^T a_l, g_c_l = sum gz
__global__ __launch_bounds__(kBlock) void k_mp_bwd_gz(int n, int l, const double *__restrict__ s,
                                                      const float *__restrict__ P, const float *__restrict__ G,
                                                      const unsigned short *__restrict__ Zl,
                                                      const unsigned short *__restrict__ Hl,
                                                      const unsigned short *__restrict__ Al,
                                                      unsigned short *__restrict__ GZ, unsigned short *__restrict__ Y,
                                                      float *gpart) {
    __shared__ unsigned short Bn[kHid][kHid];     // Bn[o][k] = Wn_l[o][k]
    __shared__ unsigned short Tg[kTile][kHid + 8];
    __shared__ unsigned short Th[kTile][kHid + 8];
    __shared__ unsigned short Ta[kTile][kHid + 8];
    __shared__ float gcp[kBlock / kHid][kHid];
    for (int q = threadIdx.x; q < kHid * kHid; q += blockDim.x)
        Bn[q / kHid][q % kHid] = f2bf(P[kOffWn + l * kHid * kHid + q]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = (lane >> 4) * 4;
    // this wave's 16x16 block (o-tile, k-tile) of the weight gradients
    const int ot = wv >> 1, ktile = wv & 1;
    f4 gws = f4{0.f, 0.f, 0.f, 0.f}, gwn = f4{0.f, 0.f, 0.f, 0.f};
    float gc = 0.f;   // thread (ln = tid / 4 ... ) partial of g_c over its column
    for (long long base = (long long)blockIdx.x * kTile; base < n; base += (long long)gridDim.x * kTile) {
        __syncthreads();
        for (int q = threadIdx.x; q < kTile * kHid; q += blockDim.x) {
            const int ln = q / kHid, o = q - ln * kHid;
            const long long i = base + ln;
            unsigned short g = 0, h = 0, a = 0;
            if (i < n) {
                const float gv = bf2f(Zl[i * kHid + o]) > 0.f ? G[i * kHid + o] : 0.f;
                g = f2bf(gv);
                h = Hl[i * kHid + o];
                a = Al[i * kHid + o];
                GZ[i * kHid + o] = g;
            }
            Tg[ln][o] = g;
            Th[ln][o] = h;
            Ta[ln][o] = a;
        }
        __syncthreads();
        // g_c: thread t sums column t % 32 over rows t / 32, t / 32 + 8, ...
        {
            const int o = threadIdx.x & (kHid - 1);
            for (int ln = threadIdx.x / kHid; ln < kTile; ln += kBlock / kHid) gc += bf2f(Tg[ln][o]);
        }
        // Y = gz Wn / s for this wave's 16 nodes
        {
            const int r0 = wv * 16;
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kt = 0; kt < 2; ++kt) {
                    bf4 af, bfr;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        af[q] = static_cast<short>(Tg[r0 + m][kt * 16 + kq + q]);
                        bfr[q] = static_cast<short>(Bn[kt * 16 + kq + q][nt * 16 + m]);
                    }
                    acc = mfma16(af, bfr, acc);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const long long i = base + r0 + kq + q;
                    if (i < n) Y[i * kHid + nt * 16 + m] = f2bf(acc[q] / static_cast<float>(s[i]));
                }
            }
        }
        // weight gradients: rows o (gz features) x cols k (h or a features), K = nodes
#pragma unroll
        for (int kt = 0; kt < kTile / 16; ++kt) {
            bf4 af, bh, ba;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ln = kt * 16 + kq + q;
                af[q] = static_cast<short>(Tg[ln][ot * 16 + m]);
                bh[q] = static_cast<short>(Th[ln][ktile * 16 + m]);
                ba[q] = static_cast<short>(Ta[ln][ktile * 16 + m]);
            }
            gws = mfma16(af, bh, gws);
            gwn = mfma16(af, ba, gwn);
        }
    }
    // write this block's partials: C[o][k] at lane (row 4(l/16)+q, col l%16)
    float *gp = gpart + (size_t)blockIdx.x * kNParam;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int o = ot * 16 + kq + q, k = ktile * 16 + m;
        gp[kOffWs + l * kHid * kHid + o * kHid + k] = gws[q];
        gp[kOffWn + l * kHid * kHid + o * kHid + k] = gwn[q];
    }
    gcp[threadIdx.x / kHid][threadIdx.x & (kHid - 1)] = gc;
    __syncthreads();
    if (threadIdx.x < kHid) {
        float v = 0.f;
        for (int r = 0; r < kBlock / kHid; ++r) v += gcp[r][threadIdx.x];
        gp[kOffC + l * kHid + threadIdx.x] = v;
    }
}

// layer l, part 2: G <- G + gz Ws_l + AggT(Y),  AggT(Y)_i = -s_i sum_{j != i} Ks_ij Y_j
__global__ __launch_bounds__(kBlock) void k_mp_bwd_h(int n, int l, const int *__restrict__ rp,
                                                     const int *__restrict__ ci, const double *__restrict__ Ks,
                                                     const double *__restrict__ s, const float *__restrict__ P,
                                                     const unsigned short *__restrict__ GZ,
                                                     const unsigned short *__restrict__ Y, float *__restrict__ G) {
    __shared__ unsigned short Bs[kHid][kHid];     // Bs[o][k] = Ws_l[o][k]
    __shared__ unsigned short Tg[kTile][kHid + 8];
    __shared__ float Tagg[kTile][kHid + 1];
    for (int q = threadIdx.x; q < kHid * kHid; q += blockDim.x)
        Bs[q / kHid][q % kHid] = f2bf(P[kOffWs + l * kHid * kHid + q]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = (lane >> 4) * 4;
    for (long long base = (long long)blockIdx.x * kTile; base < n; base += (long long)gridDim.x * kTile) {
        __syncthreads();
        {
            const int ln = threadIdx.x >> 2, f0 = (threadIdx.x & 3) * 8;
            const long long i = base + ln;
            if (i < n) {
                float a[8];
                agg8(static_cast<int>(i), f0, rp, ci, Ks, s, Y, false, a);
                const float sc = static_cast<float>(-s[i]);
                for (int k = 0; k < 8; ++k) Tagg[ln][f0 + k] = a[k] * sc;
                for (int k = 0; k < 8; ++k) Tg[ln][f0 + k] = GZ[i * kHid + f0 + k];
            } else {
                for (int k = 0; k < 8; ++k) {
                    Tagg[ln][f0 + k] = 0.f;
                    Tg[ln][f0 + k] = 0;
                }
            }
        }
        __syncthreads();
        const int r0 = wv * 16;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) {
                bf4 af, bfr;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    af[q] = static_cast<short>(Tg[r0 + m][kt * 16 + kq + q]);
                    bfr[q] = static_cast<short>(Bs[kt * 16 + kq + q][nt * 16 + m]);
                }
                acc = mfma16(af, bfr, acc);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ln = r0 + kq + q, o = nt * 16 + m;
                const long long i = base + ln;
                if (i < n) G[i * kHid + o] += acc[q] + Tagg[ln][o];
            }
        }
    }
}

// encoder: g_z0 = G * [z0 > 0]; g_We = sum g_z0 x^T, g_ce = sum g_z0
__global__ __launch_bounds__(kBlock) void k_mp_bwd_enc(int n, const float *__restrict__ G,
                                                       const unsigned short *__restrict__ Z0,
                                                       const float *__restrict__ X, float *gpart) {
    __shared__ float red[kBlock];
    // thread handles column o = tid % 32 over nodes i = tid / 32 + 8 k
    const int o = threadIdx.x & (kHid - 1);
    float gw[kIn], gc = 0.f;
    for (int k = 0; k < kIn; ++k) gw[k] = 0.f;
    for (long long i = blockIdx.x * (long long)(kBlock / kHid) + threadIdx.x / kHid; i < n;
         i += (long long)gridDim.x * (kBlock / kHid)) {
        const float g = bf2f(Z0[i * kHid + o]) > 0.f ? G[i * kHid + o] : 0.f;
        gc += g;
        for (int k = 0; k < kIn; ++k) gw[k] += g * X[i * 8 + k];
    }
    float *gp = gpart + (size_t)blockIdx.x * kNParam;
    for (int k = 0; k <= kIn; ++k) {
        red[threadIdx.x] = k < kIn ? gw[k] : gc;
        __syncthreads();
        if (threadIdx.x < kHid) {
            float v = 0.f;
            for (int r = 0; r < kBlock / kHid; ++r) v += red[r * kHid + threadIdx.x];
            if (k < kIn)
                gp[kOffWe + threadIdx.x * kIn + k] = v;
            else
                gp[kOffCe + threadIdx.x] = v;
        }
        __syncthreads();
    }
}

// grad[p] = sum over blocks of gpart[b][p] (fixed order); loss
__global__ __launch_bounds__(kBlock) void k_mp_grad_reduce(const float *gpart, int nb, float *grad,
                                                           const double *lpart, double *loss_out, int n,
                                                           const double *scal, int knorm) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < kNParam; p += gridDim.x * blockDim.x) {
        float v = 0.f;
        for (int b = 0; b < nb; ++b) v += gpart[(size_t)b * kNParam + p];
        grad[p] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (knorm) {
            const double tkt = scal[kScalTKT];
            *loss_out = tkt > 0.0 ? scal[kScalEKE] / tkt : 0.0;
        } else {
            double l = 0.0;
            for (int b = 0; b < nb; ++b) l += lpart[b];
            *loss_out = l / n;
        }
    }
}

// K-norm loss, step 1: the pair (s_i e_i, s_i t_i) per node, e = delta - t,
// t = (phi - phi_prev) / sigma, s = sqrt(diag K), so that K = S Ks S gives
// e^T K e = (S e)^T Ks (S e)
__global__ __launch_bounds__(kBlock) void k_mp_kl_pair(int n, const float *__restrict__ delta,
                                                       const double *__restrict__ phi,
                                                       const double *__restrict__ phi_prev,
                                                       const double *__restrict__ s, const double *scal,
                                                       double *__restrict__ et) {
    const double sig = scal[0];
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double t = (phi[i] - phi_prev[i]) / sig;
        const double e = static_cast<double>(delta[i]) - t;
        et[2 * i] = s[i] * e;
        et[2 * i + 1] = s[i] * t;
    }
}

// step 2: Ks times both halves of the pair; ke_i = s_i (Ks S e)_i = (K e)_i;
// partials of e^T K e and t^T K t
template <class C>
__global__ __launch_bounds__(kBlock) void k_mp_kl_prod(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                       const double *__restrict__ Ks, const double *__restrict__ s,
                                                       const double *__restrict__ et, double *__restrict__ ke,
                                                       double *part) {
    __shared__ double lds[2 * kBlock / kWave];
    double acc[2] = {0.0, 0.0};
    csr_rows<double, 2, C>(
        n, rp, ci, Ks,
        [&](int, int c, double v, bool ok, double(&a)[2]) {
            const double2 p = *reinterpret_cast<const double2 *>(et + 2 * (size_t)c);
            a[0] += ok ? v * p.x : 0.0;
            a[1] += ok ? v * p.y : 0.0;
        },
        [&](int row, int lane, double(&a)[2]) {
            if (lane != 0) return;
            ke[row] = s[row] * a[0];
            acc[0] += et[2 * (size_t)row] * a[0];
            acc[1] += et[2 * (size_t)row + 1] * a[1];
        });
    write_partials<2>(acc, part, lds);
}

// step 3 (one block): scal[kScalEKE] = e^T K e, scal[kScalTKT] = t^T K t
__global__ __launch_bounds__(kBlock) void k_mp_kl_sum(int np, const double *part, double *scal) {
    __shared__ double lds[2 * kBlock / kWave];
    double v[2];
    read_partials<2>(part, np, v, lds);
    if (threadIdx.x == 0) {
        scal[kScalEKE] = v[0];
        scal[kScalTKT] = v[1];
    }
}

__global__ __launch_bounds__(kBlock) void k_mp_adam(float *p, const float *g, float *m, float *v, float lr, float b1,
                                                    float b2, float eps, float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kNParam; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

}  // namespace oasis

using namespace oasis;

extern "C" int oasis_mpnn_workspace_size(int32_t n, size_t *bytes) {
    if (n <= 0 || !bytes) return OASIS_EINVAL;
    Carver c(nullptr, 0);
    MpWs w;
    carve_mp(c, n, w);
    *bytes = c.bytes() + 256;   // + the loss scalar
    return OASIS_OK;
}

static int mp_check(const oasis_csr *Ks, const double *s, void *ws) {
    if (!Ks || Ks->dtype != OASIS_F64 || Ks->n <= 0 || !Ks->row_ptr || !Ks->col_idx || !Ks->val || !s || !ws)
        return OASIS_EINVAL;
    return OASIS_OK;
}

static int mp_forward(void *stream, const oasis_csr *Ks, const double *s, int32_t dim, const double *coords,
                      const double *b_phi, const double *phi_prev, const float *params, double *guess,
                      float *delta, void *ws, size_t ws_bytes, bool store) {
    OASIS_TRY(mp_check(Ks, s, ws));
    if (!b_phi || !phi_prev || !params || dim < 0 || dim > 3 || (dim > 0 && !coords)) return OASIS_EINVAL;
    const int n = Ks->n;
    Carver c(ws, ws_bytes);
    MpWs w;
    carve_mp(c, n, w);
    if (!c.ok) return OASIS_EWORKSPACE;
    hipStream_t st = as_stream(stream);
    const double *val = static_cast<const double *>(Ks->val);
    const int g1 = grid_for(n, rows_per_block<Cfg4x4x1>(), kMaxPartials);
    hipLaunchKernelGGL((k_mp_feat1<Cfg4x4x1>), dim3(g1), dim3(kBlock), 0, st, n, Ks->row_ptr, Ks->col_idx, val, s,
                       b_phi, phi_prev, coords, dim, w.X, w.part, w.mm);
    OASIS_TRY_LAUNCH();
    hipLaunchKernelGGL(k_mp_feat_reduce, dim3(1), dim3(kBlock), 0, st, n, g1, w.part, w.mm, w.scal);
    OASIS_TRY_LAUNCH();
    if (store)
        hipLaunchKernelGGL(k_mp_feat2<true>, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, n, w.scal,
                           params, w.X, w.Z[0], w.H[0]);
    else
        hipLaunchKernelGGL(k_mp_feat2<false>, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, n, w.scal,
                           params, w.X, w.Z[0], w.H[0]);
    OASIS_TRY_LAUNCH();
    // at most 1024 blocks, each walking tiles and loading the layer weights
    // once: 183 us per layer on the 1.6M-node mesh against 248 us with one
    // block per tile
    const int gt = (int)std::min<long long>((n + kTile - 1) / kTile, 1024);
    // the edge weights live in the gradient buffer (n x kHid floats, unused
    // until the backward pass) when the matrix has at most kHid entries per
    // row on average
    const long long nnz = Ks->nnz;
    const bool ew = nnz >= 0 && nnz <= static_cast<long long>(n) * kHid;
    if (ew) {
        hipLaunchKernelGGL(k_mp_edge_w, dim3((unsigned)std::min<long long>((nnz + kBlock - 1) / kBlock, 16384)),
                           dim3(kBlock), 0, st, nnz, Ks->col_idx, val, s, w.G);
        OASIS_TRY_LAUNCH();
    }
    for (int l = 0; l < kLayers; ++l) {
        const bool last = l == kLayers - 1;
        float *dl = delta ? delta : w.delta;
        auto go = [&](auto kern, float *d, double *g) {
            hipLaunchKernelGGL(kern, dim3(gt), dim3(kBlock), 0, st, n, l, Ks->row_ptr, Ks->col_idx, val, s, w.G,
                               params, w.H[l], w.Ag[l], w.Z[l + 1], w.H[l + 1], d, g, phi_prev, w.scal);
        };
        auto pick = [&](auto ewc) {
            constexpr bool E = decltype(ewc)::value;
            if (last)
                store ? go(k_mp_layer<true, true, E>, dl, guess) : go(k_mp_layer<true, false, E>, dl, guess);
            else
                store ? go(k_mp_layer<false, true, E>, nullptr, nullptr)
                      : go(k_mp_layer<false, false, E>, nullptr, nullptr);
        };
        if (ew)
            pick(std::true_type{});
        else
            pick(std::false_type{});
        OASIS_TRY_LAUNCH();
    }
    if (delta && store) {
        // keep the workspace copy for the backward pass
        OASIS_TRY_HIP(hipMemcpyAsync(w.delta, delta, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st));
    }
    return OASIS_OK;
}

extern "C" int oasis_mpnn_forward(void *stream, const oasis_csr *Ks, const double *s, int32_t dim,
                                  const double *coords, const double *b_phi, const double *phi_prev,
                                  const float *params, double *guess, float *delta, void *ws, size_t ws_bytes) {
    return mp_forward(stream, Ks, s, dim, coords, b_phi, phi_prev, params, guess, delta, ws, ws_bytes, true);
}

namespace oasis {
int mpnn_infer(void *stream, const oasis_csr *Ks, const double *s, int32_t dim, const double *coords,
               const double *b_phi, const double *phi_prev, const float *params, double *guess, void *ws,
               size_t ws_bytes) {
    return mp_forward(stream, Ks, s, dim, coords, b_phi, phi_prev, params, guess, nullptr, ws, ws_bytes, false);
}
}  // namespace oasis

extern "C" int oasis_mpnn_backward(void *stream, const oasis_csr *Ks, const double *s, const double *phi,
                                   const double *phi_prev, const float *params, float *grad, int32_t loss_kind,
                                   double *loss_out, void *ws, size_t ws_bytes) {
    OASIS_TRY(mp_check(Ks, s, ws));
    if (!phi || !phi_prev || !params || !grad) return OASIS_EINVAL;
    if (loss_kind != OASIS_MPNN_LOSS_MSE && loss_kind != OASIS_MPNN_LOSS_KNORM) return OASIS_EINVAL;
    const bool knorm = loss_kind == OASIS_MPNN_LOSS_KNORM;
    const int n = Ks->n;
    Carver c(ws, ws_bytes);
    MpWs w;
    carve_mp(c, n, w);
    double *dloss = c.take<double>(1);
    if (!c.ok) return OASIS_EWORKSPACE;
    hipStream_t st = as_stream(stream);
    const double *val = static_cast<const double *>(Ks->val);
    const int nb = kGradBlocks;
    if (knorm) {
        hipLaunchKernelGGL(k_mp_kl_pair, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, n, w.delta, phi,
                           phi_prev, s, w.scal, w.et);
        OASIS_TRY_LAUNCH();
        const int g1 = grid_for(n, rows_per_block<Cfg4x4x1>(), kMaxPartials);
        hipLaunchKernelGGL((k_mp_kl_prod<Cfg4x4x1>), dim3(g1), dim3(kBlock), 0, st, n, Ks->row_ptr, Ks->col_idx,
                           val, s, w.et, w.ke, w.part);
        OASIS_TRY_LAUNCH();
        hipLaunchKernelGGL(k_mp_kl_sum, dim3(1), dim3(kBlock), 0, st, g1, w.part, w.scal);
        OASIS_TRY_LAUNCH();
    }
    hipLaunchKernelGGL(k_mp_bwd_dec, dim3(nb), dim3(kBlock), 0, st, n, w.H[kLayers], w.delta, phi, phi_prev, w.scal,
                       knorm ? w.ke : static_cast<const double *>(nullptr), params, w.G, w.gpart, w.lpart);
    OASIS_TRY_LAUNCH();
    // at most 1024 blocks, each walking tiles and loading the layer weights
    // once: 183 us per layer on the 1.6M-node mesh against 248 us with one
    // block per tile
    const int gt = (int)std::min<long long>((n + kTile - 1) / kTile, 1024);
    for (int l = kLayers - 1; l >= 0; --l) {
        hipLaunchKernelGGL(k_mp_bwd_gz, dim3(nb), dim3(kBlock), 0, st, n, l, s, params, w.G, w.Z[l + 1], w.H[l],
                           w.Ag[l], w.GZ, w.Y, w.gpart);
        OASIS_TRY_LAUNCH();
        hipLaunchKernelGGL(k_mp_bwd_h, dim3(gt), dim3(kBlock), 0, st, n, l, Ks->row_ptr, Ks->col_idx, val, s, params,
                           w.GZ, w.Y, w.G);
        OASIS_TRY_LAUNCH();
    }
    hipLaunchKernelGGL(k_mp_bwd_enc, dim3(nb), dim3(kBlock), 0, st, n, w.G, w.Z[0], w.X, w.gpart);
    OASIS_TRY_LAUNCH();
    hipLaunchKernelGGL(k_mp_grad_reduce, dim3((kNParam + kBlock - 1) / kBlock), dim3(kBlock), 0, st, w.gpart, nb, grad,
                       w.lpart, dloss, n, w.scal, knorm ? 1 : 0);
    OASIS_TRY_LAUNCH();
    if (loss_out) {
        OASIS_TRY_HIP(hipMemcpyAsync(loss_out, dloss, sizeof(double), hipMemcpyDeviceToHost, st));
        OASIS_TRY_HIP(hipStreamSynchronize(st));
    }
    return OASIS_OK;
}

extern "C" int oasis_mpnn_adam(void *stream, float *params, const float *grad, float *m, float *v, int32_t t,
                               float lr, float beta1, float beta2, float eps) {
    if (!params || !grad || !m || !v || t < 1) return OASIS_EINVAL;
    const float c1 = 1.f - std::pow(beta1, (float)t), c2 = 1.f - std::pow(beta2, (float)t);
    hipLaunchKernelGGL(k_mp_adam, dim3((kNParam + kBlock - 1) / kBlock), dim3(kBlock), 0, as_stream(stream), params,
                       grad, m, v, lr, beta1, beta2, eps, c1, c2);
    OASIS_TRY_LAUNCH();
    return OASIS_OK;
}
