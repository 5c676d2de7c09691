// Internal Krylov solver interfaces (CG on a symmetrically scaled SPD
// matrix, BiCGStab on a column-scaled matrix) shared by the standalone entry
// points and the IPCS step.
#pragma once

#include "internal.hpp"
#include "spmv.hpp"

namespace oasis {

struct CGState {
    double rr[2];      // r.r of the residual entering iteration it, slot it & 1
    double tol2;       // (rtol ||b||)^2 in the weighted norm
    double wbb;        // weighted ||b||^2
    double wrr;        // weighted ||r||^2 seen by the last finalize
    double upd2;       // mixed precision: replace the residual once wrr <= upd2
    int flag;          // 0 running, 1 converged candidate, 2 breakdown, 3 non-finite,
                       // 4 residual replacement due (mixed precision)
    int it_done;       // iteration index at which flag was raised
    double wrr_it;     // weighted r.r entering iteration it_last (the last one that ran)
    int it_last;
    int pad;
};

template <typename T>
struct alignas(2 * sizeof(T)) RP {
    T r, p;
};

// One row of the single-reduction CG state: residual r, its product
// w = Ms r, the direction's product s = Ms p and the direction p.
template <typename T>
struct alignas(4 * sizeof(T)) Q4 {
    T r, w, s, p;
};

template <typename T>
struct CGWork {
    // ELL path (single-reduction CG, one kernel per iteration): iteration it
    // reads rec[it & 1] = (r_it, Ms r_it, s_{it-1}, p_{it-1}) and writes
    // (r_{it+1}, Ms r_{it+1}, s_it, p_it) into rec[(it + 1) & 1].
    Q4<T> *rec[2] = {nullptr, nullptr};
    // CSR path (two kernels per iteration), in the same memory: residual and
    // direction interleaved, so that the product kernel fetches both with
    // one gather: iteration it reads pair[it & 1] = (r_it, p_{it-1}) and
    // writes (r_it, p_it) into pair[(it + 1) & 1], whose r the update kernel
    // then turns into r_{it+1}.
    RP<T> *pair[2] = {nullptr, nullptr};
    T *q = nullptr;
    double *partA = nullptr, *partB = nullptr;
    CGState *st = nullptr;
    // optional ELL copy of the iteration matrix (set by the owner); the
    // product kernel uses it when present and the tuning allows it
    EllCols cols;
    const T *eval = nullptr;
    Tuning tun;
    HostStage stage;   // the owner's read-back block (may be null)
};

struct BiState {
    double rho[2], alpha[2], omega[2];
    double tol2, wbb, wrr;
    int active;        // 1 while iterating
    int event;         // see krylov.hip
    int no_sexit_it;   // iteration whose s-exit test is disabled
    int it_rec;        // iteration whose incoming recursive residual is wrr_rec
    double wrr_rec;    // weighted ||r||^2 entering iteration it_rec (for the host's plan)
};

struct BiGlobal {
    int pause;
    int phase;         // 1, 2, 3: kernel of iteration pause_it that paused
    int pause_it;
    int pad;
};

// The per-right-hand-side states and the pause record in one block, so
// that the host moves them with one copy each way.
struct BiBlock {
    BiState st[3];
    BiGlobal glob;
};

// A residual interleaved with a companion vector (BiCGStab's u or v).
template <typename T>
struct alignas(2 * sizeof(T)) RW {
    T r, w;
};

template <typename T>
struct BiWork {
    // ru = (r, u) with u = p - omega v, the part of the next direction
    // beyond r (formed by the update kernel, so the first product gathers
    // one pair per entry and right-hand side); rv = (r, v) written by the
    // first product for the second.  Both hold the pairs of all nr
    // right-hand sides of a row together (right-hand side k of row i at
    // i * nr + k), so that a gathered column's pairs share a cache line.
    // Per right-hand side: the direction p, r_hat, t and the s-stage
    // candidate iterate xs.
    RW<T> *ru, *rv;
    T *p[3], *rhat[3], *t[3], *xs[3];
    double *part1, *part2, *part3;
    BiState *st;       // [3], the start of a BiBlock
    BiGlobal *glob;    // in the same block
    // optional ELL copy of the iteration matrix (set by the owner)
    EllCols cols;
    const T *eval = nullptr;
    HostStage stage;   // the owner's read-back block (may be null)
    Tuning tun;
};

struct SolveOut {
    int iters = 0;
    int status = OASIS_OK;
    int replacements = 0;
    int outer = 0;            // refinement steps (mixed precision)
    double rel_res = 0.0;
    double kernel_ms = 0.0;
    int kernel_count = 0;
};


template <typename T>
void carve_cg(Carver &c, int n, CGWork<T> &w);
template <typename T>
void carve_bi(Carver &c, int n, int nrhs, BiWork<T> &w);

// CG on Ms x = b with Ms the scaled matrix (unit diagonal).  The stopping
// test uses sum_i wgt_i r_i^2 <= rtol^2 sum_i wgt_i b_i^2.
template <typename T>
int cg_solve(hipStream_t s, int n, const int *rp, const int *ci, const T *val, const T *wgt,
             const T *b, T *x, double rtol, int maxit, int check_every, bool time_kernel,
             CGWork<T> &w, SolveOut &out);

// BiCGStab for nrhs systems with the column-scaled matrix As (right Jacobi).
// inner: the solve is the inner one of a refinement loop.  It starts from
// x = 0, which it writes itself (r = b, no product), and stops on its
// recursive residual (or, at an s-stage exit, on the norm of s) without
// confirming it by an explicit residual: the caller's FP64 residual
// decides.
template <typename T>
int bicgstab_solve(hipStream_t s, int n, int nrhs, const int *rp, const int *ci, const T *val,
                   const T *wgt, const T *const *b, T *const *x, double rtol, int maxit,
                   int check_every, bool time_kernel, BiWork<T> &w, SolveOut *out, bool inner = false);

// Mixed-precision CG with reliable updates on the scaled system: FP32
// matrix/vectors inside the iteration, FP64 solution accumulator, and an
// FP64 residual b - Ms x that replaces the FP32 one whenever the latter has
// dropped by `delta` since the last replacement (the search direction is
// kept).  vnull (nullable): unit-norm null vector of Ms, projected out of
// the FP32 residual updates.  vscale > 0 states that the norm weights are
// vscale * vnull^2 (Ms = D^-1/2 K D^-1/2 with K 1 = 0: weights d = s^2 and
// vnull = s / ||s||, vscale = ||s||^2); the single-reduction iterations then
// form them from vnull instead of reading wgt32.
int cg_mixed_solve(hipStream_t s, int n, const int *rp, const int *ci, const double *val,
                   const float *val32, const double *wgt, const float *wgt32, const float *vnull,
                   double vscale, const double *b, double *x, double rtol, double delta, int maxit,
                   int check_every, bool time_kernel, CGWork<float> &w, float *xlo, double *rhi,
                   SolveOut &out);

// Longest row of a CSR pattern (synchronises; tmp: one device int).
int csr_max_row(hipStream_t s, int n, const int *rp, int *tmp, int *out);

// ELL copy of a CSR matrix with rows of at most kEll entries (see
// spmv.hpp): ecol [n][kEll] 16-bit cyclic column offsets, and the values
// as FP64 (eval) and/or their FP32 rounding (eval32); either value array
// may be null, not both.  *fits (host) tells whether every offset fitted;
// if not, the copy must not be used.  tmp: one device int.  Synchronises.
int csr_to_ell(hipStream_t s, int n, const int *rp, const int *ci, const double *val, short *ecol,
               double *eval, float *eval32, int *tmp, bool *fits);

// Most distinct offset lists an ELL pattern dictionary holds.
constexpr int kMaxEllPatterns = 4096;

// Pattern dictionary of an ELL copy's offsets (ecol, as written by
// csr_to_ell): pid [n] receives each row's pattern id and ptab
// [kMaxEllPatterns][kEll] the distinct offset lists, numbered in order of
// first occurrence.  *npat = their number, or 0 when there are more than
// min(kMaxEllPatterns, n / 8) (pid and ptab then must not be used) or
// `enable` is false.  Host work on a copy of ecol; synchronises.
int ell_dictionary(hipStream_t s, int n, const short *ecol, unsigned short *pid, short *ptab, int *npat,
                   bool enable);

// The columns of an ELL copy: the dictionary when it was built, else the
// per-entry offsets.
inline EllCols ell_cols(const short *ecol, const unsigned short *pid, const short *ptab, int npat) {
    EllCols c;
    if (npat > 0) {
        c.pid = pid;
        c.ptab = ptab;
    } else {
        c.ecol = ecol;
    }
    return c;
}

// One direction + product launch of the FP64 CG iteration (the ELL kernel
// when cols and eval are given, else CSR): p_new = g.r + beta p_old from
// the gathered (r, p_old) pairs of cur, q = A p_new, nxt = (r, p_new),
// partials (p.q, 0) per block, with beta = partIn[0] / st->rr of the
// previous iteration and the convergence test on partIn[1] (the same
// contract as the CG solver's own iterations).  *grid: its grid.
int cg_product_launch(hipStream_t s, int cap, int n, const int *rp, const int *ci, const double *val,
                      const EllCols &cols, const double *eval, const RP<double> *cur, RP<double> *nxt, double *q,
                      const double *partIn, int nIn, int stride, CGState *st, int it, int beta_zero,
                      double *partOut, int *grid);
int cg_product_launch(hipStream_t s, int cap, int n, const int *rp, const int *ci, const float *val,
                      const EllCols &cols, const float *eval, const RP<float> *cur, RP<float> *nxt, float *q,
                      const double *partIn, int nIn, int stride, CGState *st, int it, int beta_zero,
                      double *partOut, int *grid);

// r[i * rs] = b - A x with FP64 values (columns from cols when given), then
// the CG state's norms: mode 0 starts a solve (tol2 = rtol2 sum wgt b^2),
// mode 1 refreshes wrr only; the flag is cleared.
int cg_residual_state(hipStream_t s, int cap, int n, const int *rp, const int *ci, const double *val,
                      const EllCols &cols, const double *wgt, const double *b, const double *x, double *r, int rs,
                      double *part, CGState *st, double rtol2, int mode, double upd_factor = 0.0);

// Weighted residual of x for the scaled system: r = b - Ms x, returns
// (sum wgt r^2, sum wgt b^2) on the host.  Uses w's buffers.
int cg_residual(hipStream_t s, int n, const int *rp, const int *ci, const double *val,
                const double *wgt, const double *b, const double *x, double *r,
                CGWork<double> &w, double *wrr, double *wbb);

}  // namespace oasis
