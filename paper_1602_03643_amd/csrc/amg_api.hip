// C ABI of the multigrid preconditioner: set-up on the host, upload into a
// caller workspace, the cycle and the preconditioned CG (amg.hip).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "amg.hpp"

using namespace oasis;

// The hierarchy's image in the caller's workspace.
struct AmgImage {
    short *ecol = nullptr;                      // level 0's ELL copy (when it fits)
    unsigned short *pid = nullptr;
    short *ptab = nullptr;
    double *e64 = nullptr;
    float *e32 = nullptr;
    _Float16 *e16 = nullptr;                    // FP16 copy of e32 (OASIS_AMG_HALF_LEVEL0)
    EllCols cols;
    int ell_storage = 0;
    AmgCycle<double> c64;
    AmgCycle<float> c32;
    CGWork<double> cg;
    CGWork<float> cg32;                         // the mixed-precision CG (FP32 handles)
    float *r32 = nullptr;                       // its FP32 recursive residual
    double *r = nullptr;                        // CG residual
    double *ones = nullptr;                     // unit norm weights of the stand-alone solve
    int *tmp = nullptr;
};

struct oasis_amg {
    oasis_amg() = default;
    oasis_amg(const oasis_amg &) = delete;
    oasis_amg &operator=(const oasis_amg &) = delete;
    ~oasis_amg() { stage_free(stage); }
    HostStage stage;   // pinned read-back block of the solve loop
    int last_iters = 0;   // iterations of the last step solve (the first launch's hint)
    oasis_amg_params par{};
    Tuning tun;
    bool f32 = false, singular = false, half0 = false;
    int n = 0, nnz = 0;
    const int *rp = nullptr, *ci = nullptr;     // the input matrix (device, by reference)
    const double *val = nullptr;
    const double *B = nullptr;                  // its near-null vector (device, by reference; may be null)
    std::vector<HostLevel> levels;
    std::vector<double> cinv;
    bool ell_fits = false;                      // level 0 fits the ELL copy (host check)
    bool uploaded = false;
    AmgImage d;
};

namespace {

// Whether the rows fit the 16-slot ELL copy with 16-bit cyclic offsets (the
// rule of csr_to_ell).
bool ell_fits_host(const HostCsr &A) {
    const long long half = A.n / 2;
    for (int i = 0; i < A.n; ++i) {
        if (A.rp[i + 1] - A.rp[i] > kEll) return false;
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            long long d = static_cast<long long>(A.ci[k]) - i;
            if (d >= half) d -= A.n;
            if (d < -half) d += A.n;
            if (d < -32768 || d > 32767) return false;
        }
    }
    return true;
}

template <typename T>
void carve_levels(Carver &c, const oasis_amg &h, AmgCycle<T> &cy) {
    const int L = static_cast<int>(h.levels.size());
    cy = AmgCycle<T>();
    cy.nlev = L;
    for (int l = 0; l < L; ++l) {
        const HostLevel &hl = h.levels[l];
        AmgDevLevel<T> &d = cy.lv[l];
        d.n = hl.A.n;
        if (l > 0) {
            d.rp = c.take<int>(hl.A.n + 1);
            d.ci = c.take<int>(hl.A.nnz());
            d.val = c.take<T>(hl.A.nnz());
        } else if (!h.ell_fits) {
            d.rp = h.rp;
            d.ci = h.ci;
            d.val = c.take<T>(hl.A.nnz());
        }
        if (l + 1 < L) {
            d.wd = c.take<T>(hl.A.n);
            d.y = c.take<T>(hl.A.n);
            d.prp = c.take<int>(hl.A.n + 1);
            d.pci = c.take<int>(hl.P.nnz());
            d.pval = c.take<T>(hl.P.nnz());
            const HostCsr &R = hl.R;
            d.rrp = c.take<int>(R.n + 1);
            d.rci = c.take<int>(R.nnz());
            d.rval = c.take<T>(R.nnz());
            d.t = c.take<T>(hl.A.n);
        }
        if (l > 0) {
            d.b = c.take<T>(hl.A.n);
            d.x = c.take<T>(hl.A.n);
        }
    }
    cy.nc = h.levels.back().A.n;
    cy.cinv = c.take<T>(static_cast<size_t>(cy.nc) * cy.nc);
    // CSR lanes per row from the mean row length (the coarse levels' rows
    // grow long, 70-140 entries, and are few: wider groups there)
    auto lanes = [](const HostCsr &M) {
        const double avg = M.n ? static_cast<double>(M.nnz()) / M.n : 0.0;
        return avg <= 6.0 ? 2 : avg <= 12.0 ? 4 : avg <= 28.0 ? 8 : avg <= 56.0 ? 16 : avg <= 100.0 ? 32 : 64;
    };
    for (int l = 0; l < L; ++l) {
        const HostLevel &hl = h.levels[l];
        cy.lv[l].alanes = lanes(hl.A);
        if (l + 1 < L) {
            cy.lv[l].planes = lanes(hl.P);
            cy.lv[l].rlanes = lanes(hl.R);
        }
    }
}

void carve_amg(Carver &c, const oasis_amg &h, AmgImage &d) {
    const int n = h.n;
    d = AmgImage();
    if (h.ell_fits) {
        d.ecol = c.take<short>(static_cast<size_t>(n) * kEll);
        d.pid = c.take<unsigned short>(n);
        d.ptab = c.take<short>(static_cast<size_t>(kMaxEllPatterns) * kEll);
        d.e64 = c.take<double>(static_cast<size_t>(n) * kEll);
        if (h.f32) d.e32 = c.take<float>(static_cast<size_t>(n) * kEll);
        if (h.f32 && h.half0) d.e16 = c.take<_Float16>(static_cast<size_t>(n) * kEll);
    }
    carve_cg<double>(c, n, d.cg);
    if (h.f32) {
        carve_cg<float>(c, n, d.cg32);
        d.r32 = c.take<float>(n);
    }
    d.r = c.take<double>(n);
    d.ones = c.take<double>(n);
    d.tmp = c.take<int>(8);
    if (h.f32)
        carve_levels<float>(c, h, d.c32);
    else
        carve_levels<double>(c, h, d.c64);
}

__global__ __launch_bounds__(kBlock) void k_amg_to_f16(long long m, const float *__restrict__ a,
                                                       _Float16 *__restrict__ b) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m; i += (long long)gridDim.x * blockDim.x)
        b[i] = static_cast<_Float16>(a[i]);
}

__global__ __launch_bounds__(kBlock) void k_amg_fill(int n, double *x, double v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

template <typename T>
int put(hipStream_t s, T *dst, const std::vector<T> &src) {
    if (!src.empty()) OASIS_TRY_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return OASIS_OK;
}

template <typename T>
std::vector<T> cast(const std::vector<double> &v) {
    return std::vector<T>(v.begin(), v.end());
}

// smoother weights omega / a_ii of a host level
std::vector<double> weights(const HostLevel &hl) {
    std::vector<double> w(hl.A.n, 0.0);
    for (int i = 0; i < hl.A.n; ++i)
        for (int k = hl.A.rp[i]; k < hl.A.rp[i + 1]; ++k)
            if (hl.A.ci[k] == i) w[i] = hl.omega / hl.A.v[k];
    return w;
}

template <typename T>
int upload_levels(hipStream_t s, oasis_amg &h, AmgCycle<T> &cy) {
    const int L = cy.nlev;
    for (int l = 0; l < L; ++l) {
        const HostLevel &hl = h.levels[l];
        AmgDevLevel<T> &d = cy.lv[l];
        if (l > 0) {
            OASIS_TRY(put(s, const_cast<int *>(d.rp), hl.A.rp));
            OASIS_TRY(put(s, const_cast<int *>(d.ci), hl.A.ci));
        }
        if (l > 0 || !h.ell_fits) OASIS_TRY(put(s, const_cast<T *>(d.val), cast<T>(hl.A.v)));
        if (l + 1 < L) {
            OASIS_TRY(put(s, const_cast<T *>(d.wd), cast<T>(weights(hl))));
            OASIS_TRY(put(s, const_cast<int *>(d.prp), hl.P.rp));
            OASIS_TRY(put(s, const_cast<int *>(d.pci), hl.P.ci));
            OASIS_TRY(put(s, const_cast<T *>(d.pval), cast<T>(hl.P.v)));
            const HostCsr &R = hl.R;
            OASIS_TRY(put(s, const_cast<int *>(d.rrp), R.rp));
            OASIS_TRY(put(s, const_cast<int *>(d.rci), R.ci));
            OASIS_TRY(put(s, const_cast<T *>(d.rval), cast<T>(R.v)));
        }
    }
    OASIS_TRY(put(s, const_cast<T *>(cy.cinv), cast<T>(h.cinv)));
    if (h.ell_fits) {
        cy.cols = h.d.cols;
        cy.e = std::is_same<T, float>::value ? reinterpret_cast<const T *>(h.d.e32)
                                             : reinterpret_cast<const T *>(h.d.e64);
        if (std::is_same<T, float>::value) cy.e16 = h.d.e16;
    }
    return OASIS_OK;
}


}  // namespace

namespace oasis {

int amg_handle_solve(hipStream_t s, oasis_amg *h, const double *wgt, const double *b, double *x, double rtol,
                     int maxit, SolveOut &out, bool mixed, double delta) {
    if (!h || !h->uploaded) return OASIS_EINVAL;
    AmgImage &d = h->d;
    if (h->f32 && mixed)
        return amg_pcg_mixed(s, h->n, h->rp, h->ci, h->val, d.e64, d.c32, wgt, b, x, rtol,
                             delta > 0.0 ? delta : kAmgMixedDelta, maxit, 0, d.r, d.r32, d.cg32, out);
    // successive pressure solves of a time loop take similar counts: launch
    // about 60% of the last one's iterations before the first poll
    const int first = h->last_iters > 3 ? h->last_iters * 3 / 5 : 0;
    int rc;
    if (h->f32)
        rc = amg_pcg_solve<float>(s, h->n, h->rp, h->ci, h->val, d.e64, d.c32, wgt, b, x, rtol, maxit, 0, false,
                                  d.r, d.cg, out, first);
    else
        rc = amg_pcg_solve<double>(s, h->n, h->rp, h->ci, h->val, d.e64, d.c64, wgt, b, x, rtol, maxit, 0, false,
                                   d.r, d.cg, out, first);
    if (rc == OASIS_OK) h->last_iters = out.iters;
    return rc;
}

bool amg_handle_matches(const oasis_amg *h, int n, const int *rp, const double *val, const double *B) {
    return h && h->uploaded && h->singular && h->n == n && h->rp == rp && h->val == val && h->B == B;
}

}  // namespace oasis

extern "C" int oasis_amg_setup(void *stream, const oasis_csr *A, const double *B, const oasis_amg_params *par,
                               oasis_amg **out) {
    if (!out) return OASIS_EINVAL;
    *out = nullptr;
    if (!A || !par || A->n <= 0 || A->nnz <= 0 || !A->row_ptr || !A->col_idx || !A->val || A->dtype != OASIS_F64)
        return OASIS_EINVAL;
    if (par->precision != OASIS_F64 && par->precision != OASIS_F32) return OASIS_EINVAL;
    if (par->theta < 0.0 || par->theta >= 1.0 || par->coarse_size < 0 || par->coarse_size > kAmgMaxCoarse ||
        par->max_levels < 0 || par->max_levels > kAmgMaxLevels)
        return OASIS_EINVAL;
    Tuning tun;
    OASIS_TRY(Tuning::from(&par->tuning, &tun));
    // the multigrid CG and its cycle take 768 blocks (three per CU) unless
    // told otherwise: on the 129x129x97 channel the headline step ran
    // 12.47-12.49 ms at 768 against 12.59-12.60 at 1024 and 12.61 at 1280,
    // and 512 took the FP32-cycle pressure phase from 6.32 to 6.45 ms, while
    // the Krylov solvers elsewhere run best at the 512 default
    if (par->tuning.grid_cap == 0) tun.grid_cap = 768;
    hipStream_t s = as_stream(stream);
    oasis_amg *h = new (std::nothrow) oasis_amg();
    if (!h) return OASIS_EINVAL;
    h->par = *par;
    h->tun = tun;
    h->f32 = par->precision == OASIS_F32;
    h->singular = (par->flags & OASIS_KRYLOV_NULLSPACE_CONST) != 0;
    h->half0 = (par->flags & OASIS_AMG_HALF_LEVEL0) != 0;
    h->n = A->n;
    h->nnz = A->nnz;
    h->rp = A->row_ptr;
    h->ci = A->col_idx;
    h->val = static_cast<const double *>(A->val);
    h->B = B;
    HostCsr A0;
    A0.n = A0.m = A->n;
    A0.rp.resize(A->n + 1);
    A0.ci.resize(A->nnz);
    A0.v.resize(A->nnz);
    std::vector<double> B0(A->n, 1.0);
    auto fail = [&](int rc) {
        delete h;
        return rc;
    };
    if (hipMemcpyAsync(A0.rp.data(), A->row_ptr, (A->n + 1) * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(A0.ci.data(), A->col_idx, A->nnz * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(A0.v.data(), A->val, A->nnz * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        (B && hipMemcpyAsync(B0.data(), B, A->n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(OASIS_EHIP);
    if (A0.rp[0] != 0 || A0.rp[A->n] != A->nnz) return fail(OASIS_EINVAL);
    for (int i = 0; i < A->n; ++i) {
        if (A0.rp[i + 1] < A0.rp[i]) return fail(OASIS_EINVAL);
        for (int k = A0.rp[i]; k < A0.rp[i + 1]; ++k)
            if (A0.ci[k] < 0 || A0.ci[k] >= A->n || (k > A0.rp[i] && A0.ci[k] <= A0.ci[k - 1]))
                return fail(OASIS_EINVAL);
        if (!(B0[i] != 0.0) || !std::isfinite(B0[i])) return fail(OASIS_EINVAL);
    }
    AmgHostParams hp;
    if (par->theta > 0.0) hp.theta = par->theta;
    if (par->coarse_size > 0) hp.coarse_size = par->coarse_size;
    if (par->max_levels > 0) hp.max_levels = par->max_levels;
    hp.singular = h->singular;
    h->ell_fits = tun.ell() && ell_fits_host(A0);
    const int rc = amg_build(A0, B0, hp, h->levels, h->cinv);
    if (rc != OASIS_OK) return fail(rc);
    *out = h;
    return OASIS_OK;
}

extern "C" int oasis_amg_workspace_size(const oasis_amg *h, size_t *bytes) {
    if (!h || !bytes) return OASIS_EINVAL;
    Carver c(nullptr, 0);
    AmgImage d;
    carve_amg(c, *h, d);
    *bytes = c.bytes();
    return OASIS_OK;
}

extern "C" int oasis_amg_upload(void *stream, oasis_amg *h, void *ws, size_t ws_bytes) {
    if (!h || !ws || !aligned(ws, 256)) return OASIS_EINVAL;
    hipStream_t s = as_stream(stream);
    h->uploaded = false;
    Carver c(ws, ws_bytes);
    carve_amg(c, *h, h->d);
    if (!c.ok) return OASIS_EWORKSPACE;
    AmgImage &d = h->d;
    d.cg.tun = d.cg32.tun = h->tun;
    if (!h->stage.h) stage_alloc(h->stage);
    d.cg.stage = d.cg32.stage = h->stage;
    hipLaunchKernelGGL(k_amg_fill, dim3(grid_for(h->n, kBlock, 8192)), dim3(kBlock), 0, s, h->n, d.ones, 1.0);
    OASIS_TRY_LAUNCH();
    if (h->ell_fits) {
        bool fits = false;
        OASIS_TRY(csr_to_ell(s, h->n, h->rp, h->ci, h->val, d.ecol, d.e64, d.e32, d.tmp, &fits));
        if (!fits) return OASIS_EINVAL;     // the device copy disagrees with the host check
        if (d.e16) {
            const long long m = static_cast<long long>(h->n) * kEll;
            hipLaunchKernelGGL(k_amg_to_f16, dim3(grid_for(m, kBlock, 8192)), dim3(kBlock), 0, s, m, d.e32, d.e16);
            OASIS_TRY_LAUNCH();
        }
        int npat = 0;
        OASIS_TRY(ell_dictionary(s, h->n, d.ecol, d.pid, d.ptab, &npat, h->tun.dict()));
        d.cols = ell_cols(d.ecol, d.pid, d.ptab, npat);
        d.ell_storage = npat > 0 ? npat : -1;
    }
    if (h->f32)
        OASIS_TRY(upload_levels<float>(s, *h, d.c32));
    else
        OASIS_TRY(upload_levels<double>(s, *h, d.c64));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    h->uploaded = true;
    return OASIS_OK;
}

extern "C" int oasis_amg_levels(const oasis_amg *h, int32_t *n_levels) {
    if (!h || !n_levels) return OASIS_EINVAL;
    *n_levels = static_cast<int32_t>(h->levels.size());
    return OASIS_OK;
}

extern "C" int oasis_amg_level(const oasis_amg *h, int32_t level, oasis_amg_level_info *info) {
    if (!h || !info || level < 0 || level >= static_cast<int>(h->levels.size())) return OASIS_EINVAL;
    const HostLevel &hl = h->levels[level];
    std::memset(info, 0, sizeof(*info));
    info->n = hl.A.n;
    info->nnz = static_cast<int32_t>(hl.A.nnz());
    info->row_ptr = hl.A.rp.data();
    info->col_idx = hl.A.ci.data();
    info->val = hl.A.v.data();
    info->near_null = hl.B.data();
    info->omega = hl.omega;
    if (level + 1 < static_cast<int>(h->levels.size())) {
        info->n_agg = hl.n_agg;
        info->agg = hl.agg.data();
        info->p_nnz = static_cast<int32_t>(hl.P.nnz());
        info->p_row_ptr = hl.P.rp.data();
        info->p_col_idx = hl.P.ci.data();
        info->p_val = hl.P.v.data();
    } else {
        info->coarse_inv = h->cinv.data();
    }
    return OASIS_OK;
}

extern "C" int oasis_amg_vcycle(void *stream, oasis_amg *h, const double *r, double *z) {
    if (!h || !h->uploaded || !r || !z) return OASIS_EINVAL;
    hipStream_t s = as_stream(stream);
    if (h->f32)
        return amg_vcycle<float>(s, h->d.c32, r, false, z, 1, nullptr, nullptr, nullptr, nullptr, h->tun.grid_cap);
    return amg_vcycle<double>(s, h->d.c64, r, false, z, 1, nullptr, nullptr, nullptr, nullptr, h->tun.grid_cap);
}

extern "C" int oasis_amg_pcg(void *stream, oasis_amg *h, const double *b, double *x, const oasis_krylov_opts *opt,
                             oasis_krylov_stats *stats) {
    if (!h || !h->uploaded || !b || !x || !opt || !stats || !(opt->rtol > 0) || opt->maxit < 0) return OASIS_EINVAL;
    hipStream_t s = as_stream(stream);
    // the stopping test on the plain 2-norm of the residual (unit weights)
    SolveOut so;
    const int maxit = opt->maxit > 0 ? opt->maxit : 10000;
    const bool timed = (opt->flags & OASIS_KRYLOV_TIME) != 0;
    AmgImage &d = h->d;
    int rc;
    if (h->f32 && opt->precision == OASIS_F32 && !timed)
        rc = amg_pcg_mixed(s, h->n, h->rp, h->ci, h->val, d.e64, d.c32, d.ones, b, x, opt->rtol,
                           opt->inner_rtol > 0.0 ? opt->inner_rtol : kAmgMixedDelta, maxit, opt->check_every, d.r,
                           d.r32, d.cg32, so);
    else if (h->f32)
        rc = amg_pcg_solve<float>(s, h->n, h->rp, h->ci, h->val, d.e64, d.c32, d.ones, b, x, opt->rtol, maxit,
                                  opt->check_every, timed, d.r, d.cg, so);
    else
        rc = amg_pcg_solve<double>(s, h->n, h->rp, h->ci, h->val, d.e64, d.c64, d.ones, b, x, opt->rtol, maxit,
                                   opt->check_every, timed, d.r, d.cg, so);
    if (rc == OASIS_EHIP) return rc;
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    stats->iters = so.iters;
    stats->outer_iters = so.outer;
    stats->status = so.status;
    stats->restarts = so.replacements;
    stats->rel_res = so.rel_res;
    stats->kernel_ms = so.kernel_ms;
    stats->kernel_count = so.kernel_count;
    stats->ell_patterns = d.ell_storage;
    return rc;
}

extern "C" int oasis_amg_destroy(oasis_amg *h) {
    if (!h) return OASIS_EINVAL;
    delete h;
    return OASIS_OK;
}
