// Graph set-up on the device: the shared P1 sparsity pattern, greedy cell
// colouring for atomic-free assembly, colour classes, and the reverse
// Cuthill-McKee ordering.  All results are deterministic: integer atomics
// only count or claim, and every order-dependent list is re-sorted by a
// total key before use.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace oasis {

// ---------------------------------------------------------------------------
// exclusive scan of int32 (n <= 2^31 - 1 total), out[n] = total

constexpr int kScanTile = 1024;   // elements per block (256 threads x 4)

__global__ __launch_bounds__(kBlock) void k_scan_tiles(int n, const int *__restrict__ in,
                                                       int *__restrict__ out,
                                                       int *__restrict__ tile_sums) {
    __shared__ int sh[kScanTile];
    const int base = blockIdx.x * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += blockDim.x)
        sh[k] = (base + k < n) ? in[base + k] : 0;
    __syncthreads();
    // each thread scans 4 consecutive elements, then a Hillis-Steele pass over thread totals
    const int t = threadIdx.x;
    int a0 = sh[4 * t], a1 = sh[4 * t + 1], a2 = sh[4 * t + 2], a3 = sh[4 * t + 3];
    int tot = a0 + a1 + a2 + a3;
    __shared__ int ts[kBlock];
    ts[t] = tot;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        int v = (t >= o) ? ts[t - o] : 0;
        __syncthreads();
        ts[t] += v;
        __syncthreads();
    }
    int excl = ts[t] - tot;
    sh[4 * t] = excl;
    sh[4 * t + 1] = excl + a0;
    sh[4 * t + 2] = excl + a0 + a1;
    sh[4 * t + 3] = excl + a0 + a1 + a2;
    __syncthreads();
    for (int k = threadIdx.x; k < kScanTile; k += blockDim.x)
        if (base + k < n) out[base + k] = sh[k];
    if (t == kBlock - 1) tile_sums[blockIdx.x] = ts[t];
}

// single block: exclusive scan of the tile sums in place, total at [ntiles]
__global__ __launch_bounds__(1024) void k_scan_sums(int ntiles, int *sums) {
    __shared__ int carry;
    __shared__ int ts[1024];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < ntiles; base += 1024) {
        const int i = base + threadIdx.x;
        const int v = i < ntiles ? sums[i] : 0;
        ts[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int a = (threadIdx.x >= (unsigned)o) ? ts[threadIdx.x - o] : 0;
            __syncthreads();
            ts[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < ntiles) sums[i] = carry + ts[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += ts[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[ntiles] = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int n, int *out, const int *sums) {
    const int i = blockIdx.x * kScanTile;
    const int off = sums[blockIdx.x];
    for (int k = threadIdx.x; k < kScanTile; k += blockDim.x)
        if (i + k < n) out[i + k] += off;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[gridDim.x];
}

static size_t scan_ws_ints(int n) { return (size_t)(n + kScanTile - 1) / kScanTile + 1; }

// out has n+1 entries; in may equal out only if n == 0
static int exclusive_scan(hipStream_t s, int n, const int *in, int *out, int *tmp) {
    const int tiles = std::max(1, (n + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kBlock), 0, s, n, in, out, tmp);
    OASIS_TRY_LAUNCH();
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tiles, tmp);
    OASIS_TRY_LAUNCH();
    hipLaunchKernelGGL(k_scan_add, dim3(tiles), dim3(kBlock), 0, s, n, out, tmp);
    OASIS_TRY_LAUNCH();
    return OASIS_OK;
}

__global__ __launch_bounds__(kBlock) void k_fill_i(long long n, int *x, int v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

static int fill_i(hipStream_t s, long long n, int *x, int v) {
    if (n <= 0) return OASIS_OK;
    const int g = (int)std::min<long long>((n + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(k_fill_i, dim3(g), dim3(kBlock), 0, s, n, x, v);
    OASIS_TRY_LAUNCH();
    return OASIS_OK;
}

// ---------------------------------------------------------------------------
// dof -> incident cells, stored as codes cell * (dim+1) + local vertex,
// each list ascending

__global__ __launch_bounds__(kBlock) void k_inc_count(int ncell, int nv, int nvert, int ndof,
                                                      const int *__restrict__ cells,
                                                      const int *__restrict__ v2d, int *cnt,
                                                      int *err) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        int d[4];
        bool ok = true;
        for (int a = 0; a < nv; ++a) {
            const int v = cells[c * nv + a];
            if (v < 0 || v >= nvert) {
                ok = false;
                d[a] = -1;
                continue;
            }
            d[a] = v2d[v];
            if (d[a] < 0 || d[a] >= ndof) ok = false;
        }
        if (!ok) {
            atomicOr(err, 2);   // index out of range: the mesh is rejected
            continue;
        }
        for (int a = 0; a < nv; ++a) {
            for (int b = 0; b < a; ++b)
                if (d[a] == d[b]) atomicOr(err, 1);   // a cell must hold distinct dofs
            atomicAdd(&cnt[d[a]], 1);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_inc_fill(int ncell, int nv, const int *__restrict__ cells,
                                                     const int *__restrict__ v2d,
                                                     const int *__restrict__ ptr, int *fillc,
                                                     int *inc) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        for (int a = 0; a < nv; ++a) {
            const int d = v2d[cells[c * nv + a]];
            const int slot = atomicAdd(&fillc[d], 1);
            inc[ptr[d] + slot] = (int)(c * nv + a);   // cell and local vertex
        }
    }
}

// make every incidence list ascending (removes the fill order)
__global__ __launch_bounds__(kBlock) void k_inc_sort(int ndof, const int *__restrict__ ptr, int *inc) {
    for (long long d = blockIdx.x * (long long)blockDim.x + threadIdx.x; d < ndof;
         d += (long long)gridDim.x * blockDim.x) {
        const int s = ptr[d], e = ptr[d + 1];
        for (int i = s + 1; i < e; ++i) {
            const int v = inc[i];
            int j = i - 1;
            while (j >= s && inc[j] > v) {
                inc[j + 1] = inc[j];
                --j;
            }
            inc[j + 1] = v;
        }
    }
}

// distinct neighbour dofs of each dof, ascending; count only when col == nullptr
__global__ __launch_bounds__(kBlock) void k_row_pattern(int ndof, int nv, const int *__restrict__ cells,
                                                        const int *__restrict__ v2d,
                                                        const int *__restrict__ iptr,
                                                        const int *__restrict__ inc,
                                                        const int *__restrict__ rp, int *len,
                                                        int *col) {
    for (long long d = blockIdx.x * (long long)blockDim.x + threadIdx.x; d < ndof;
         d += (long long)gridDim.x * blockDim.x) {
        const int s = iptr[d], e = iptr[d + 1];
        int prev = -1, count = 0;
        int out = col ? rp[d] : 0;
        while (true) {
            int best = 0x7fffffff;
            for (int i = s; i < e; ++i) {
                const int c = inc[i] / nv;
                for (int a = 0; a < nv; ++a) {
                    const int q = v2d[cells[(long long)c * nv + a]];
                    if (q > prev && q < best) best = q;
                }
            }
            if (best == 0x7fffffff) break;
            if (col) col[out++] = best;
            ++count;
            prev = best;
        }
        if (!col) len[d] = count;
    }
}

struct GraphWs {
    int *iptr, *inc, *cnt, *tmp, *flag;
    int *round_of, *color_cnt, *pos;
};

static void carve_graph(Carver &c, const oasis_mesh *m, GraphWs &g) {
    const long long nv = m->dim + 1;
    const int nmax = std::max(m->n_dof, m->n_cell);
    g.iptr = c.take<int>((size_t)m->n_dof + 1);
    g.inc = c.take<int>((size_t)m->n_cell * nv);
    g.cnt = c.take<int>((size_t)nmax + 1);
    g.tmp = c.take<int>(scan_ws_ints(nmax) + 16);
    g.flag = c.take<int>(16);
    g.round_of = c.take<int>((size_t)m->n_cell);
    g.color_cnt = c.take<int>(256);
    g.pos = c.take<int>((size_t)nmax + 1);
}

static int check_mesh(const oasis_mesh *m) {
    if (!m || (m->dim != 2 && m->dim != 3) || m->n_vert <= 0 || m->n_cell <= 0 || m->n_dof <= 0)
        return OASIS_EINVAL;
    if (!m->coords || !m->cells || !m->vert2dof) return OASIS_EINVAL;
    return OASIS_OK;
}

static int build_incidence(hipStream_t s, const oasis_mesh *m, GraphWs &g) {
    const int nv = m->dim + 1;
    const int gc = grid_for(m->n_cell, kBlock, 8192);
    OASIS_TRY(fill_i(s, m->n_dof + 1, g.cnt, 0));
    OASIS_TRY(fill_i(s, 16, g.flag, 0));
    hipLaunchKernelGGL(k_inc_count, dim3(gc), dim3(kBlock), 0, s, m->n_cell, nv, m->n_vert, m->n_dof,
                       m->cells, m->vert2dof, g.cnt, g.flag);
    OASIS_TRY_LAUNCH();
    int err0 = 0;
    OASIS_TRY_HIP(hipMemcpyAsync(&err0, g.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    if (err0 & 2) return OASIS_EINVAL;
    OASIS_TRY(exclusive_scan(s, m->n_dof, g.cnt, g.iptr, g.tmp));
    OASIS_TRY(fill_i(s, m->n_dof + 1, g.cnt, 0));
    hipLaunchKernelGGL(k_inc_fill, dim3(gc), dim3(kBlock), 0, s, m->n_cell, nv, m->cells,
                       m->vert2dof, g.iptr, g.cnt, g.inc);
    OASIS_TRY_LAUNCH();
    hipLaunchKernelGGL(k_inc_sort, dim3(grid_for(m->n_dof, kBlock, 8192)), dim3(kBlock), 0, s,
                       m->n_dof, g.iptr, g.inc);
    OASIS_TRY_LAUNCH();
    int err = 0;
    OASIS_TRY_HIP(hipMemcpyAsync(&err, g.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    return err ? OASIS_EUNSUPPORTED : OASIS_OK;
}

// Incidence lists for an external user (the IPCS handle): iptr [n_dof+1],
// inc [n_cell*(dim+1)], scratch cnt [max(n_dof, n_cell)+1], tmp (scan).
int incidence_codes(hipStream_t s, const oasis_mesh *m, int *iptr, int *inc, int *cnt, int *tmp, int *flag) {
    GraphWs g{};
    g.iptr = iptr;
    g.inc = inc;
    g.cnt = cnt;
    g.tmp = tmp;
    g.flag = flag;
    return build_incidence(s, m, g);
}

size_t incidence_tmp_ints(int n) { return scan_ws_ints(n) + 16; }

// ---------------------------------------------------------------------------
// greedy first-fit colouring in decreasing priority (Jones-Plassmann rounds)

__global__ __launch_bounds__(kBlock) void k_color_round(int ncell, int nv, const int *__restrict__ cells,
                                                        const int *__restrict__ v2d,
                                                        const int *__restrict__ iptr,
                                                        const int *__restrict__ inc,
                                                        const int *__restrict__ pri, int *color,
                                                        int *round_of, int round, int *remaining,
                                                        int *overflow) {
    int left = 0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        if (__atomic_load_n(&color[c], __ATOMIC_RELAXED) >= 0) continue;
        const int my = pri[c];
        unsigned long long used0 = 0ull, used1 = 0ull;
        bool ready = true;
        for (int a = 0; a < nv && ready; ++a) {
            const int d = v2d[cells[c * nv + a]];
            for (int i = iptr[d]; i < iptr[d + 1]; ++i) {
                const int o = inc[i] / nv;
                if (o == c || pri[o] < my) continue;
                // a higher-priority neighbour counts only once coloured in an earlier round
                const int r = __atomic_load_n(&round_of[o], __ATOMIC_RELAXED);
                const int co = __atomic_load_n(&color[o], __ATOMIC_RELAXED);
                if (co < 0 || r >= round) {
                    ready = false;
                    break;
                }
                if (co < 64)
                    used0 |= 1ull << co;
                else
                    used1 |= 1ull << (co - 64);
            }
        }
        if (!ready) {
            ++left;
            continue;
        }
        int k;
        if (~used0)
            k = __builtin_ctzll(~used0);
        else if (~used1)
            k = 64 + __builtin_ctzll(~used1);
        else {
            atomicOr(overflow, 1);
            k = 127;
        }
        __atomic_store_n(&round_of[c], round, __ATOMIC_RELAXED);
        __atomic_store_n(&color[c], k, __ATOMIC_RELAXED);
    }
    if (left) atomicAdd(remaining, left);
}

__global__ __launch_bounds__(kBlock) void k_color_count(int ncell, const int *color, int *cnt) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x)
        atomicAdd(&cnt[color[c]], 1);
}

__global__ __launch_bounds__(kBlock) void k_flag_eq(int n, const int *a, int v, int *flags) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        flags[i] = a[i] == v ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_scatter_eq(int n, const int *a, int v, const int *pos,
                                                       int base, int *out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        if (a[i] == v) out[base + pos[i]] = (int)i;
}

// ---------------------------------------------------------------------------
// reverse Cuthill-McKee

struct RcmWs {
    int *pos, *dist, *claim, *lst[2], *grp, *cnt, *off, *fillc, *tmp, *ctr;
    long long *keyp;
};

static void carve_rcm(Carver &c, int n, RcmWs &r) {
    r.pos = c.take<int>(n);
    r.dist = c.take<int>(n);
    r.claim = c.take<int>(n);
    r.lst[0] = c.take<int>(n);
    r.lst[1] = c.take<int>(n);
    r.grp = c.take<int>(n);
    r.cnt = c.take<int>((size_t)n + 1);
    r.off = c.take<int>((size_t)n + 1);
    r.fillc = c.take<int>((size_t)n + 1);
    r.tmp = c.take<int>(scan_ws_ints(n) + 16);
    r.ctr = c.take<int>(16);
    r.keyp = c.take<long long>(kMaxPartials + 16);
}

__device__ __forceinline__ long long deg_key(const int *rp, int v) {
    return ((long long)(rp[v + 1] - rp[v]) << 32) | (unsigned)v;
}

// minimum (degree, index) over list[0..m) (or over unplaced vertices 0..n if list == nullptr)
__global__ __launch_bounds__(kBlock) void k_minkey(int m, const int *list, const int *rp,
                                                   const int *pos, long long *part) {
    __shared__ long long sh[kBlock];
    long long best = 0x7fffffffffffffffll;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m;
         i += (long long)gridDim.x * blockDim.x) {
        const int v = list ? list[i] : (int)i;
        if (!list && pos[v] >= 0) continue;
        const long long k = deg_key(rp, v);
        best = k < best ? k : best;
    }
    sh[threadIdx.x] = best;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o && sh[threadIdx.x + o] < sh[threadIdx.x]) sh[threadIdx.x] = sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kBlock) void k_minkey_final(int np, long long *part) {
    __shared__ long long sh[kBlock];
    long long best = 0x7fffffffffffffffll;
    for (int i = threadIdx.x; i < np; i += blockDim.x) best = part[i] < best ? part[i] : best;
    sh[threadIdx.x] = best;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o && sh[threadIdx.x + o] < sh[threadIdx.x]) sh[threadIdx.x] = sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[kMaxPartials] = sh[0];
}

// BFS level expansion over not-yet-placed vertices: claim with a CAS and append
__global__ __launch_bounds__(kBlock) void k_bfs_expand(int m, const int *front, const int *rp,
                                                       const int *ci, const int *pos, int *dist,
                                                       int level, int *next, int *nsize) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m;
         i += (long long)gridDim.x * blockDim.x) {
        const int u = front[i];
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            const int v = ci[j];
            if (v == u || pos[v] >= 0) continue;
            if (atomicCAS(&dist[v], -1, level) == -1) next[atomicAdd(nsize, 1)] = v;
        }
    }
}

// parent position (least position of a placed neighbour) and child counts
__global__ __launch_bounds__(kBlock) void k_cm_parent(int m, const int *lst, const int *rp,
                                                      const int *ci, const int *pos, int lb, int lm,
                                                      int *par, int *cnt) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m;
         i += (long long)gridDim.x * blockDim.x) {
        const int v = lst[i];
        int best = 0x7fffffff;
        for (int j = rp[v]; j < rp[v + 1]; ++j) {
            const int p = pos[ci[j]];
            if (p >= 0 && p < best) best = p;
        }
        // with a symmetric pattern the parent lies in the previous level; clamp otherwise
        if (best < lb || best >= lb + lm) best = lb;
        par[i] = best;
        atomicAdd(&cnt[best - lb], 1);
    }
}

__global__ __launch_bounds__(kBlock) void k_cm_group(int m, const int *lst, const int *par, int lb,
                                                     const int *off, int *fillc, int *grp) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m;
         i += (long long)gridDim.x * blockDim.x) {
        const int p = par[i] - lb;
        const int slot = atomicAdd(&fillc[p], 1);
        grp[off[p] + slot] = lst[i];
    }
}

// siblings (same parent) are ordered by (degree, index)
__global__ __launch_bounds__(kBlock) void k_cm_place(int m, const int *lst, const int *par, int lb,
                                                     const int *off, const int *cnt,
                                                     const int *grp, const int *rp, int base,
                                                     int *pos, int *order) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m;
         i += (long long)gridDim.x * blockDim.x) {
        const int v = lst[i];
        const int p = par[i] - lb;
        const long long kv = deg_key(rp, v);
        int rank = 0;
        for (int j = off[p]; j < off[p] + cnt[p]; ++j)
            if (deg_key(rp, grp[j]) < kv) ++rank;
        const int at = base + off[p] + rank;
        pos[v] = at;
        order[at] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_rcm_finish(int n, const int *pos, const int *cm,
                                                       int *perm, int *order) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        perm[i] = n - 1 - pos[i];
        order[i] = cm[n - 1 - i];
    }
}

__global__ __launch_bounds__(kBlock) void k_relabel(int count, const int *in, const int *perm, int *out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = perm[in[i]];
}

}  // namespace oasis

using namespace oasis;

// ---------------------------------------------------------------------------
// C ABI

extern "C" int oasis_graph_workspace_size(const oasis_mesh *mesh, size_t *bytes) {
    if (!bytes) return OASIS_EINVAL;
    OASIS_TRY(check_mesh(mesh));
    Carver c(nullptr, 0);
    GraphWs g;
    carve_graph(c, mesh, g);
    *bytes = c.bytes();
    return OASIS_OK;
}

extern "C" int oasis_p1_pattern(void *stream, const oasis_mesh *mesh, int32_t *row_ptr,
                                int32_t *col_idx, int64_t col_capacity, int32_t *nnz_out,
                                void *ws, size_t ws_bytes) {
    OASIS_TRY(check_mesh(mesh));
    if (!row_ptr || !nnz_out || !ws) return OASIS_EINVAL;
    hipStream_t s = as_stream(stream);
    Carver c(ws, ws_bytes);
    GraphWs g;
    carve_graph(c, mesh, g);
    if (!c.ok) return OASIS_EWORKSPACE;
    OASIS_TRY(build_incidence(s, mesh, g));
    const int nv = mesh->dim + 1;
    const int gd = grid_for(mesh->n_dof, kBlock, 8192);
    hipLaunchKernelGGL(k_row_pattern, dim3(gd), dim3(kBlock), 0, s, mesh->n_dof, nv, mesh->cells,
                       mesh->vert2dof, g.iptr, g.inc, (const int *)nullptr, g.cnt, (int *)nullptr);
    OASIS_TRY_LAUNCH();
    OASIS_TRY(exclusive_scan(s, mesh->n_dof, g.cnt, row_ptr, g.tmp));
    int nnz = 0;
    OASIS_TRY_HIP(hipMemcpyAsync(&nnz, row_ptr + mesh->n_dof, sizeof(int), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    *nnz_out = nnz;
    if (!col_idx) return OASIS_OK;
    if (col_capacity < nnz) return OASIS_EINVAL;
    hipLaunchKernelGGL(k_row_pattern, dim3(gd), dim3(kBlock), 0, s, mesh->n_dof, nv, mesh->cells,
                       mesh->vert2dof, g.iptr, g.inc, (const int *)row_ptr, (int *)nullptr,
                       col_idx);
    OASIS_TRY_LAUNCH();
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    return OASIS_OK;
}

extern "C" int oasis_color_cells(void *stream, const oasis_mesh *mesh, const int32_t *priority,
                                 int32_t *color, int32_t *n_colors_out, void *ws, size_t ws_bytes) {
    OASIS_TRY(check_mesh(mesh));
    if (!priority || !color || !n_colors_out || !ws) return OASIS_EINVAL;
    hipStream_t s = as_stream(stream);
    Carver c(ws, ws_bytes);
    GraphWs g;
    carve_graph(c, mesh, g);
    if (!c.ok) return OASIS_EWORKSPACE;
    OASIS_TRY(build_incidence(s, mesh, g));
    OASIS_TRY(fill_i(s, mesh->n_cell, color, -1));
    OASIS_TRY(fill_i(s, mesh->n_cell, g.round_of, 0x7fffffff));
    const int nv = mesh->dim + 1;
    const int gc = grid_for(mesh->n_cell, kBlock, 8192);
    int remaining = mesh->n_cell;
    for (int round = 0; remaining > 0; ++round) {
        if (round > 100000) return OASIS_EUNSUPPORTED;
        OASIS_TRY(fill_i(s, 2, g.flag, 0));
        hipLaunchKernelGGL(k_color_round, dim3(gc), dim3(kBlock), 0, s, mesh->n_cell, nv, mesh->cells,
                           mesh->vert2dof, g.iptr, g.inc, priority, color, g.round_of, round,
                           g.flag, g.flag + 1);
        OASIS_TRY_LAUNCH();
        int h[2];
        OASIS_TRY_HIP(hipMemcpyAsync(h, g.flag, sizeof(h), hipMemcpyDeviceToHost, s));
        OASIS_TRY_HIP(hipStreamSynchronize(s));
        if (h[1]) return OASIS_EUNSUPPORTED;
        remaining = h[0];
    }
    // number of colours = 1 + max colour
    OASIS_TRY(fill_i(s, 256, g.color_cnt, 0));
    hipLaunchKernelGGL(k_color_count, dim3(gc), dim3(kBlock), 0, s, mesh->n_cell, color, g.color_cnt);
    OASIS_TRY_LAUNCH();
    int cnt[128];
    OASIS_TRY_HIP(hipMemcpyAsync(cnt, g.color_cnt, sizeof(cnt), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    int nc = 0;
    for (int k = 0; k < 128; ++k)
        if (cnt[k]) nc = k + 1;
    *n_colors_out = nc;
    return OASIS_OK;
}

extern "C" int oasis_color_classes(void *stream, int32_t n_cell, const int32_t *color,
                                   int32_t n_colors, int32_t *color_ptr, int32_t *color_cells,
                                   void *ws, size_t ws_bytes) {
    if (n_cell <= 0 || n_colors <= 0 || n_colors > 128 || !color || !color_ptr || !color_cells || !ws)
        return OASIS_EINVAL;
    hipStream_t s = as_stream(stream);
    Carver c(ws, ws_bytes);
    int *flags = c.take<int>((size_t)n_cell + 1);
    int *posv = c.take<int>((size_t)n_cell + 1);
    int *tmp = c.take<int>(scan_ws_ints(n_cell) + 16);
    if (!c.ok) return OASIS_EWORKSPACE;
    const int gc = grid_for(n_cell, kBlock, 8192);
    int base = 0;
    color_ptr[0] = 0;
    for (int k = 0; k < n_colors; ++k) {
        hipLaunchKernelGGL(k_flag_eq, dim3(gc), dim3(kBlock), 0, s, n_cell, color, k, flags);
        OASIS_TRY_LAUNCH();
        OASIS_TRY(exclusive_scan(s, n_cell, flags, posv, tmp));
        hipLaunchKernelGGL(k_scatter_eq, dim3(gc), dim3(kBlock), 0, s, n_cell, color, k, posv, base,
                           color_cells);
        OASIS_TRY_LAUNCH();
        int cnt = 0;
        OASIS_TRY_HIP(hipMemcpyAsync(&cnt, posv + n_cell, sizeof(int), hipMemcpyDeviceToHost, s));
        OASIS_TRY_HIP(hipStreamSynchronize(s));
        base += cnt;
        color_ptr[k + 1] = base;
    }
    return base == n_cell ? OASIS_OK : OASIS_EINVAL;
}

extern "C" int oasis_rcm_workspace_size(int32_t n, size_t *bytes) {
    if (n <= 0 || !bytes) return OASIS_EINVAL;
    Carver c(nullptr, 0);
    RcmWs r;
    carve_rcm(c, n, r);
    *bytes = c.bytes();
    return OASIS_OK;
}

static int rcm_minkey(hipStream_t s, int m, const int *list, const int *rp, const int *pos,
                      long long *part, long long *out) {
    const int g = grid_for(m, kBlock);
    hipLaunchKernelGGL(k_minkey, dim3(g), dim3(kBlock), 0, s, m, list, rp, pos, part);
    OASIS_TRY_LAUNCH();
    hipLaunchKernelGGL(k_minkey_final, dim3(1), dim3(kBlock), 0, s, g, part);
    OASIS_TRY_LAUNCH();
    OASIS_TRY_HIP(hipMemcpyAsync(out, part + kMaxPartials, sizeof(long long), hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    return OASIS_OK;
}

// BFS over unplaced vertices from root; returns depth and the least-key vertex of the last level
static int rcm_levels(hipStream_t s, int n, const int *rp, const int *ci, RcmWs &r, int root,
                      int *depth, int *last_min) {
    OASIS_TRY(fill_i(s, n, r.dist, -1));
    int h0[2] = {0, 0};
    OASIS_TRY_HIP(hipMemcpyAsync(r.dist + root, h0, sizeof(int), hipMemcpyHostToDevice, s));
    OASIS_TRY_HIP(hipMemcpyAsync(r.lst[0], &root, sizeof(int), hipMemcpyHostToDevice, s));
    int cur = 0, m = 1, level = 0;
    while (true) {
        OASIS_TRY(fill_i(s, 1, r.ctr, 0));
        hipLaunchKernelGGL(k_bfs_expand, dim3(grid_for(m, kBlock, 8192)), dim3(kBlock), 0, s, m,
                           r.lst[cur], rp, ci, r.pos, r.dist, level + 1, r.lst[cur ^ 1], r.ctr);
        OASIS_TRY_LAUNCH();
        int nm = 0;
        OASIS_TRY_HIP(hipMemcpyAsync(&nm, r.ctr, sizeof(int), hipMemcpyDeviceToHost, s));
        OASIS_TRY_HIP(hipStreamSynchronize(s));
        if (nm == 0) break;
        cur ^= 1;
        m = nm;
        ++level;
    }
    long long key = 0;
    OASIS_TRY(rcm_minkey(s, m, r.lst[cur], rp, r.pos, r.keyp, &key));
    *depth = level;
    *last_min = (int)(key & 0xffffffffll);
    return OASIS_OK;
}

extern "C" int oasis_rcm(void *stream, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                         int32_t *perm, int32_t *order, void *ws, size_t ws_bytes) {
    if (n <= 0 || !row_ptr || !col_idx || !perm || !order || !ws) return OASIS_EINVAL;
    hipStream_t s = as_stream(stream);
    Carver c(ws, ws_bytes);
    RcmWs r;
    carve_rcm(c, n, r);
    if (!c.ok) return OASIS_EWORKSPACE;
    OASIS_TRY(fill_i(s, n, r.pos, -1));
    int placed = 0;
    while (placed < n) {
        long long key = 0;
        OASIS_TRY(rcm_minkey(s, n, nullptr, row_ptr, r.pos, r.keyp, &key));
        int root = (int)(key & 0xffffffffll);
        int depth = 0, x = 0;
        OASIS_TRY(rcm_levels(s, n, row_ptr, col_idx, r, root, &depth, &x));
        while (true) {
            int dx = 0, xx = 0;
            OASIS_TRY(rcm_levels(s, n, row_ptr, col_idx, r, x, &dx, &xx));
            if (dx > depth) {
                root = x;
                depth = dx;
                x = xx;
            } else {
                break;
            }
        }
        // Cuthill-McKee sequence of this component, level by level
        OASIS_TRY_HIP(hipMemcpyAsync(r.pos + root, &placed, sizeof(int), hipMemcpyHostToDevice, s));
        OASIS_TRY_HIP(hipMemcpyAsync(r.grp + placed, &root, sizeof(int), hipMemcpyHostToDevice, s));
        OASIS_TRY(fill_i(s, n, r.claim, -1));
        int lb = placed, le = placed + 1;
        OASIS_TRY_HIP(hipMemcpyAsync(r.claim + root, &lb, sizeof(int), hipMemcpyHostToDevice, s));
        // r.grp doubles as the cm sequence store; levels are contiguous ranges of it
        int *cm = r.grp;
        int *newl = r.lst[0];
        int *par = r.lst[1];
        while (true) {
            const int m = le - lb;
            OASIS_TRY(fill_i(s, 1, r.ctr, 0));
            hipLaunchKernelGGL(k_bfs_expand, dim3(grid_for(m, kBlock, 8192)), dim3(kBlock), 0, s, m,
                               cm + lb, row_ptr, col_idx, r.pos, r.claim, 1, newl, r.ctr);
            OASIS_TRY_LAUNCH();
            int nm = 0;
            OASIS_TRY_HIP(hipMemcpyAsync(&nm, r.ctr, sizeof(int), hipMemcpyDeviceToHost, s));
            OASIS_TRY_HIP(hipStreamSynchronize(s));
            if (nm == 0) break;
            const int gm = grid_for(nm, kBlock, 8192);
            OASIS_TRY(fill_i(s, m + 1, r.cnt, 0));
            OASIS_TRY(fill_i(s, m + 1, r.fillc, 0));
            hipLaunchKernelGGL(k_cm_parent, dim3(gm), dim3(kBlock), 0, s, nm, newl, row_ptr, col_idx,
                               r.pos, lb, m, par, r.cnt);
            OASIS_TRY_LAUNCH();
            OASIS_TRY(exclusive_scan(s, m, r.cnt, r.off, r.tmp));
            // group buffer: reuse dist (free during the CM pass)
            hipLaunchKernelGGL(k_cm_group, dim3(gm), dim3(kBlock), 0, s, nm, newl, par, lb, r.off,
                               r.fillc, r.dist);
            OASIS_TRY_LAUNCH();
            hipLaunchKernelGGL(k_cm_place, dim3(gm), dim3(kBlock), 0, s, nm, newl, par, lb, r.off,
                               r.cnt, r.dist, row_ptr, le, r.pos, cm);
            OASIS_TRY_LAUNCH();
            lb = le;
            le += nm;
        }
        placed = le;
    }
    hipLaunchKernelGGL(k_rcm_finish, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, r.pos,
                       r.grp, perm, order);
    OASIS_TRY_LAUNCH();
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    return OASIS_OK;
}

extern "C" int oasis_relabel(void *stream, int32_t count, const int32_t *in, const int32_t *perm,
                             int32_t *out) {
    if (count < 0 || (count > 0 && (!in || !perm || !out))) return OASIS_EINVAL;
    if (count == 0) return OASIS_OK;
    hipLaunchKernelGGL(k_relabel, dim3(grid_for(count, kBlock, 8192)), dim3(kBlock), 0,
                       as_stream(stream), count, in, perm, out);
    OASIS_TRY_LAUNCH();
    return OASIS_OK;
}
