// Smoothed-aggregation algebraic multigrid: the host-built hierarchy, its
// device image and the preconditioned CG that the IPCS step and the
// stand-alone entry points share.
#pragma once

#include <vector>

#include "krylov.hpp"

namespace oasis {

constexpr int kAmgMaxLevels = 16;
constexpr int kAmgMaxCoarse = 2048;

// Host CSR (sorted columns).
struct HostCsr {
    int n = 0, m = 0;            // rows, columns
    std::vector<int> rp, ci;
    std::vector<double> v;
    long long nnz() const { return static_cast<long long>(ci.size()); }
};

// One level of the host hierarchy: its matrix, the smoother weight and,
// below the coarsest level, the aggregation and the prolongator to the next.
struct HostLevel {
    HostCsr A;                   // level 0: a host copy of the input matrix
    std::vector<double> B;       // near-null-space vector
    double omega = 0.0;          // smoother weight (4/3) / rho(D^-1 A)
    std::vector<int> agg;        // aggregate of every row (not on the coarsest level)
    int n_agg = 0;
    HostCsr P;                   // n x n_agg
    HostCsr R;                   // P^T
};

struct AmgHostParams {
    double theta = OASIS_AMG_THETA;
    int coarse_size = 1024;
    int max_levels = 12;
    bool singular = false;
};

// Builds the hierarchy of A0 with near-null vector B0 (host work).
// coarse_inv receives the dense inverse (row-major) of the coarsest level,
// regularised along its near-null vector when `singular`.  EUNSUPPORTED if
// the coarsest matrix is not positive definite (after regularisation).
int amg_build(const HostCsr &A0, const std::vector<double> &B0, const AmgHostParams &p,
              std::vector<HostLevel> &levels, std::vector<double> &coarse_inv);

// Device image of one level below the coarsest: matrix (CSR; level 0 uses
// the ELL copy instead), smoother weights w_i = omega / a_ii, prolongator P
// and restriction R = P^T (CSR), and the cycle's vectors.
template <typename T>
struct AmgDevLevel {
    int n = 0;
    const int *rp = nullptr, *ci = nullptr;
    const T *val = nullptr;
    const T *wd = nullptr;
    const int *prp = nullptr, *pci = nullptr;
    const T *pval = nullptr;
    const int *rrp = nullptr, *rci = nullptr;
    const T *rval = nullptr;
    T *b = nullptr, *t = nullptr, *x = nullptr;   // right-hand side, scratch, solution
    T *y = nullptr;                               // w .* b, the pre-smoothed iterate
    int alanes = 4, planes = 4, rlanes = 4;       // CSR lanes per row of A, P and R
};

// The cycle in precision T: level 0's matrix is the ELL copy (cols, e),
// the coarsest level a dense inverse (nc x nc, row-major).
template <typename T>
struct AmgCycle {
    int nlev = 0;
    AmgDevLevel<T> lv[kAmgMaxLevels];
    EllCols cols;
    const T *e = nullptr;
    const _Float16 *e16 = nullptr;   // level 0's values stored as FP16 (FP32 cycles; null: e)
    int nc = 0;
    const T *cinv = nullptr;
};

// One V(1,1) cycle z = M^{-1} r on level 0: r (type TB, the CG residual)
// is read and z written (type TO) at z[i * zs].  y0_ready: level 0's y = w .* r is
// already in c.lv[0].y (else the cycle forms it first).  With part (nullable), the last kernel
// writes per-block partials (r.z, sum wgt r^2) and returns its grid in
// *gpost.  flag (nullable): a device int; while it is nonzero every kernel
// returns at once.  grid_cap bounds the partial-writing kernel's grid.
template <typename T, typename TB = double, typename TO = double>
int amg_vcycle(hipStream_t s, const AmgCycle<T> &c, const TB *r, bool y0_ready, TO *z, int zs,
               const double *wgt, double *part, int *gpost, const int *flag, int grid_cap);

// CG on level 0's matrix (FP64 ELL values e64 with c's columns) preconditioned
// by the cycle c; stopping test sum wgt r^2 <= rtol^2 sum wgt b^2 on the
// true residual.  r: FP64 scratch [n]; w: CG workspace (pairs, q, partials,
// state).  first_chunk: iterations launched before the first poll (0: 2),
// for callers that expect about as many as a previous solve took.
template <typename T>
int amg_pcg_solve(hipStream_t s, int n, const int *rp, const int *ci, const double *val, const double *e64,
                  const AmgCycle<T> &c, const double *wgt, const double *b, double *x, double rtol, int maxit,
                  int check_every, bool time_kernel, double *r, CGWork<double> &w, SolveOut &out,
                  int first_chunk = 0);

// Mixed-precision CG around an FP32 cycle: the direction, the product with
// level 0's FP32 ELL copy e32 (CSR level 0 of the cycle without it) and the
// recursive residual r32 are FP32, the iterate x and the dot products FP64.
// The FP64 residual b - A x (e64 / val, into r64) replaces the recursive
// one each time the latter has fallen by delta since the last replacement,
// and whenever it claims convergence; the direction is kept.  The stopping
// test is on that FP64 residual.  w: FP32 CG workspace.
int amg_pcg_mixed(hipStream_t s, int n, const int *rp, const int *ci, const double *val, const double *e64,
                  const AmgCycle<float> &c, const double *wgt, const double *b, double *x, double rtol,
                  double delta, int maxit, int check_every, double *r64, float *r32, CGWork<float> &w,
                  SolveOut &out);

// The pressure solve of an IPCS step through an uploaded handle: CG on the
// handle's matrix with its cycle, weights wgt for the stopping test; with
// mixed and an FP32 handle, amg_pcg_mixed with replacement factor delta
// (0: kAmgMixedDelta).
int amg_handle_solve(hipStream_t s, oasis_amg *h, const double *wgt, const double *b, double *x, double rtol,
                     int maxit, SolveOut &out, bool mixed = false, double delta = 0.0);

// Replacement factor of amg_pcg_mixed when none is given.
constexpr double kAmgMixedDelta = 1e-3;

// Whether h was built (and uploaded) on this matrix and null vector as a
// singular pressure matrix.
bool amg_handle_matches(const oasis_amg *h, int n, const int *rp, const double *val, const double *B);

}  // namespace oasis
