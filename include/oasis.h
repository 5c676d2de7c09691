/*
 * oasis.h — C ABI of the MI355X (gfx950) P1-P1 IPCS hot-path library.
 *
 * Method (Mortensen & Valen-Sendstad, "Oasis: a high-level/high-performance
 * open source Navier-Stokes solver"): the incremental pressure-correction
 * scheme with Adams-Bashforth projected convecting velocity and
 * Crank-Nicolson convected velocity (Sec. 2, eq:NStentative, eq:pressure,
 * eq:correction, eq:convection_ABCN), discretised with P1 elements for
 * velocity and pressure, and implemented on the algebraic level of Sec. 5
 * (preassembled M, K, dP^k; Alg. 2 for the coefficient matrix; lumped-mass
 * velocity update).
 *
 * Conventions for every entry point
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    All device work is enqueued on it and is asynchronous unless stated.
 *  - Pointers documented "device" must be device-accessible memory owned
 *    by the caller; "host" pointers are ordinary host memory.  The library
 *    never allocates or frees device memory: every scratch buffer is a
 *    caller-provided workspace whose size is returned by a *_workspace_size
 *    query.  Workspaces must be 256-byte aligned.  The time-step and
 *    multigrid handles each hold one 1 KiB pinned, host-mapped block
 *    (hipHostMalloc at create or upload, freed by destroy) through which
 *    their solver loops read small state back; without it they fall back
 *    to ordinary copies.
 *  - Indices are int32; dense vectors are contiguous; multi-component
 *    fields are stored component-major ([dim][n]).
 *  - Every function returns an int status: 0 = OASIS_OK or a negative
 *    error code; no C++ exception crosses the ABI.  oasis_strerror() gives
 *    text, oasis_last_hip_error() the last HIP runtime error of the calling
 *    thread.
 *  - Results are deterministic: all reductions are fixed-order; no
 *    floating-point atomics are used.
 */
#ifndef OASIS_H
#define OASIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define OASIS_OK            0
#define OASIS_EINVAL       -1   /* bad argument: null/misaligned pointer, dim, dtype, size */
#define OASIS_EHIP         -2   /* a HIP runtime call failed (see oasis_last_hip_error) */
#define OASIS_ENOTCONV     -3   /* Krylov: maxit reached; x holds the last iterate, stats filled */
#define OASIS_EBREAKDOWN   -4   /* Krylov: breakdown (after one restart for BiCGStab) */
#define OASIS_ENAN         -5   /* non-finite value met in a reduction */
#define OASIS_EWORKSPACE   -6   /* workspace smaller than the queried size */
#define OASIS_EUNSUPPORTED -7   /* mesh/graph outside a documented limit */

#define OASIS_F64 0
#define OASIS_F32 1

/* forms for oasis_assemble_p1 (row = test function i, column = trial j) */
#define OASIS_FORM_MASS   0   /* M_ij  = int phi_j phi_i                    */
#define OASIS_FORM_STIFF  1   /* K_ij  = int grad phi_j . grad phi_i        */
#define OASIS_FORM_GRAD_X 2   /* dP^0_ij = int d_x phi_j phi_i  (eq:dp_matrix) */
#define OASIS_FORM_GRAD_Y 3   /* dP^1 */
#define OASIS_FORM_GRAD_Z 4   /* dP^2 (3D only) */
#define OASIS_FORM_CONV   5   /* C_ij  = int (u_bar . grad phi_j) phi_i      */

/* ---- data types -------------------------------------------------------- */

/* CSR matrix; row_ptr [n+1], col_idx [nnz] (sorted within rows), val [nnz]
 * of dtype OASIS_F64 (double) or OASIS_F32 (float).  All device pointers. */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    void *val;
    int32_t dtype;
} oasis_csr;

/* Simplex mesh with P1 dofs.  dim is 2 (triangles) or 3 (tetrahedra).
 *  coords   device double [n_vert][dim]   vertex coordinates
 *  cells    device int32  [n_cell][dim+1] vertex indices
 *  vert2dof device int32  [n_vert]        dof of every vertex; several
 *                                         vertices may share a dof
 *                                         (periodic identification)
 *  n_colors, color_ptr (HOST int32 [n_colors+1]), color_cells (device
 *  int32 [n_cell]): cells grouped so that no two cells of one colour share
 *  a dof (from oasis_color_cells / oasis_color_classes).  Needed by the
 *  assembly and IPCS entry points; ignored by the pattern and colouring
 *  entry points. */
typedef struct {
    int32_t dim;
    int32_t n_vert;
    int32_t n_cell;
    int32_t n_dof;
    const double *coords;
    const int32_t *cells;
    const int32_t *vert2dof;
    int32_t n_colors;
    const int32_t *color_ptr;
    const int32_t *color_cells;
} oasis_mesh;

/* ---- graph set-up (shared sparsity pattern, Sec. 5 after Alg. 2) -------- */

/* Workspace for oasis_p1_pattern / oasis_color_cells on this mesh. */
int oasis_graph_workspace_size(const oasis_mesh *mesh, size_t *bytes);

/* P1 sparsity pattern over dofs: (i, j) is stored iff some cell holds
 * both dofs.  Pass col_idx = NULL to get row_ptr (device int32 [n_dof+1])
 * and *nnz_out (host) only; call again with col_idx (device int32
 * [col_capacity]) to fill sorted column indices.  Synchronises `stream`.
 * EWORKSPACE if ws is too small, EINVAL if col_capacity < nnz. */
int oasis_p1_pattern(void *stream, const oasis_mesh *mesh, int32_t *row_ptr,
                     int32_t *col_idx, int64_t col_capacity, int32_t *nnz_out,
                     void *ws, size_t ws_bytes);

/* Greedy first-fit colouring of the cells, visiting cells in decreasing
 * `priority` (device int32 [n_cell], pairwise distinct): every cell takes
 * the least colour not used by an already coloured cell sharing a dof.
 * Writes color (device int32 [n_cell]) and *n_colors_out (host).  At most
 * 128 colours (else EUNSUPPORTED).  Synchronises `stream`. */
int oasis_color_cells(void *stream, const oasis_mesh *mesh, const int32_t *priority,
                      int32_t *color, int32_t *n_colors_out, void *ws, size_t ws_bytes);

/* Group cells by colour: color_ptr (HOST int32 [n_colors+1]) and
 * color_cells (device int32 [n_cell]) listing each colour's cells in
 * increasing cell index.  ws: at least oasis_graph_workspace_size bytes.
 * Synchronises `stream`. */
int oasis_color_classes(void *stream, int32_t n_cell, const int32_t *color, int32_t n_colors,
                        int32_t *color_ptr, int32_t *color_cells, void *ws, size_t ws_bytes);

/* Workspace for oasis_rcm on an n-vertex graph. */
int oasis_rcm_workspace_size(int32_t n, size_t *bytes);

/* Reverse Cuthill-McKee ordering of the symmetric pattern (row_ptr,
 * col_idx; diagonal stored).  Component roots: least (degree, index)
 * unvisited vertex refined by George-Liu pseudo-peripheral search; at each
 * vertex, unvisited neighbours are appended in (degree, index) order; the
 * sequence is reversed.  Writes perm (device int32 [n], perm[old] = new)
 * and order (device int32 [n], order[new] = old).  Synchronises `stream`. */
int oasis_rcm(void *stream, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
              int32_t *perm, int32_t *order, void *ws, size_t ws_bytes);

/* out[i] = perm[in[i]] for i < count (relabel vert2dof or a dof list). */
int oasis_relabel(void *stream, int32_t count, const int32_t *in, const int32_t *perm,
                  int32_t *out);

/* ---- assembly (Sec. 5, Alg. 2) ----------------------------------------- */

/* out.val = (base ? base.val : 0) + alpha * (assembled `form`) on the
 * pattern of `out` (which must contain the P1 pattern of the mesh; base, if
 * given, must share it).  FORM_CONV needs uab[0..dim-1], device double
 * [n_dof] each: the nodal convecting velocity u_bar.  out.dtype must be
 * F64.  Element matrices are evaluated in closed form in FP64; cells are
 * scattered colour by colour, so no two threads touch one row.  The mesh
 * colouring is required. */
int oasis_assemble_p1(void *stream, const oasis_mesh *mesh, int32_t form,
                      const double *const *uab, double alpha, const oasis_csr *base,
                      oasis_csr *out);

/* ---- sparse matrix-vector product (Sec. 5, eq:tent_algebraic terms) ----- */

/* y = alpha * A x + beta * y.  x and y have A's dtype; F32 products are
 * accumulated in FP32, F64 in FP64.  With beta == 0, y is not read. */
int oasis_spmv(void *stream, const oasis_csr *A, const void *x, void *y, double alpha,
               double beta);

/* ---- Krylov solvers (Sec. 6.2: BiCGStab + Jacobi; CG for pressure) ------ */

/* Storage and kernel-shape choices of the Krylov iterations.  An all-zero
 * struct selects the measured defaults.  They change timings and, for
 * `storage` = CSR or the CG form, the summation order; never the stopping
 * test. */
typedef struct {
    int32_t storage;      /* OASIS_STORAGE_AUTO: products on a 16-slot ELL copy of the matrix
                             with 16-bit column offsets, whose rows share a dictionary of offset
                             lists when they have few distinct ones (else per-entry offsets);
                             OASIS_STORAGE_ELL: the ELL copy with per-entry offsets always;
                             OASIS_STORAGE_CSR: CSR products (no ELL copy is used) */
    int32_t grid_cap;     /* most blocks of a kernel that writes per-block partial sums
                             (0 = 512; otherwise 64..2048) */
    int32_t cg_form;      /* OASIS_CG_FORM_AUTO: one single-reduction pass per CG iteration with
                             FP32 values, two kernels with FP64 values; OASIS_CG_FORM_TWO;
                             OASIS_CG_FORM_SINGLE (both need the ELL copy) */
} oasis_tuning;

#define OASIS_STORAGE_AUTO 0
#define OASIS_STORAGE_ELL 1
#define OASIS_STORAGE_CSR 2
#define OASIS_CG_FORM_AUTO 0
#define OASIS_CG_FORM_TWO 1
#define OASIS_CG_FORM_SINGLE 2

typedef struct {
    double rtol;          /* stop when ||b - A x||_2 <= rtol ||b||_2 (true residual) */
    int32_t maxit;        /* total (inner) iteration cap */
    int32_t precision;    /* OASIS_F64, or OASIS_F32: FP32 matrix/vectors inside the
                             iteration, FP64 dot products and FP64 refinement */
    double inner_rtol;    /* F32 mode.  CG: the FP64 residual replaces the FP32 one each
                             time the latter fell by this factor (reliable updates; 0 =
                             0.1).  BiCGStab: inner tolerance of each refinement step
                             (0 = 1e-4; tightened automatically for the last step) */
    int32_t max_outer;    /* F32 mode BiCGStab: cap on refinement steps (0 = 50) */
    int32_t check_every;  /* iterations launched between host convergence polls (0 = auto) */
    int32_t flags;        /* OASIS_KRYLOV_TIME, OASIS_KRYLOV_NULLSPACE_CONST */
    oasis_tuning tuning;
} oasis_krylov_opts;

/* Kernel timing.  oasis_pcg: when the solve stops at maxit, its last
 * product launch is repeated maxit times back to back between two HIP
 * events: in F32 mode the whole single-reduction iteration (its iterate
 * update goes to scratch memory), in F64 mode the direction+product kernel.
 * kernel_ms is their total and kernel_count = maxit (0 when the solve
 * stopped earlier); x is unchanged by the repeats.  oasis_bicgstab: every
 * first-product launch of the FP64 iteration is bracketed by events. */
#define OASIS_KRYLOV_TIME 1
/* The matrix is singular with the constant vector as null space (pure
 * Neumann pressure matrix) and b is consistent.  In F32 mode the FP32
 * iterations then keep their residual orthogonal to the (scaled) null
 * vector, which FP32 rounding of the matrix would otherwise perturb. */
#define OASIS_KRYLOV_NULLSPACE_CONST 2

typedef struct {
    int32_t iters;        /* total (inner) iterations */
    int32_t outer_iters;  /* refinement steps (F32 mode) */
    int32_t status;       /* OASIS_OK / ENOTCONV / EBREAKDOWN / ENAN */
    int32_t restarts;     /* BiCGStab breakdown restarts, residual replacements */
    double rel_res;       /* final true ||b - A x|| / ||b|| */
    double kernel_ms;     /* OASIS_KRYLOV_TIME: total time of the timed launches */
    int32_t kernel_count; /* number of timed launches */
    int32_t ell_patterns; /* column storage the products used: > 0 the number of distinct
                             per-row offset lists of the ELL dictionary, -1 per-entry
                             16-bit ELL offsets, 0 CSR */
} oasis_krylov_stats;

/* Workspace for oasis_pcg / oasis_bicgstab with nrhs right-hand sides. */
int oasis_krylov_workspace_size(int32_t n, int32_t nnz, int32_t nrhs,
                                const oasis_krylov_opts *opt, size_t *bytes);

/* Jacobi-preconditioned CG on an SPD (or SPSD with consistent b) F64 CSR
 * matrix.  b: device double [n]; x: device double [n], in: x0, out:
 * solution (last iterate on ENOTCONV).  stats: host.  Synchronises
 * `stream`.  The iteration is CG on D^{-1/2} A D^{-1/2} (same iterates as
 * z = D^{-1} r preconditioning in exact arithmetic). */
int oasis_pcg(void *stream, const oasis_csr *A, const double *b, double *x,
              const oasis_krylov_opts *opt, void *ws, size_t ws_bytes,
              oasis_krylov_stats *stats);

/* oasis_pcg for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, with its workspace in a file-scope device array of the
 * library of OASIS_PCG_NOALLOC_BYTES bytes (one per device, held until the
 * process ends) instead of a caller workspace.  It calls no hipMalloc,
 * hipFree or other allocating routine; the offset dictionary (built on the
 * host) is not used, and OASIS_KRYLOV_TIME is refused (EINVAL).
 * EUNSUPPORTED when oasis_krylov_workspace_size(n, nnz, 1, opt) exceeds
 * OASIS_PCG_NOALLOC_BYTES.  All calls on one device share the array: calls
 * that overlap on one device (other streams, other threads) race.
 * Synchronises `stream`. */
#define OASIS_PCG_NOALLOC_BYTES (64u << 20)
int oasis_pcg_noalloc(void *stream, const oasis_csr *A, const double *b, double *x,
                      const oasis_krylov_opts *opt, oasis_krylov_stats *stats);

/* BiCGStab (van der Vorst) with right Jacobi preconditioning (the iteration
 * runs on A D^{-1} y = b, x = D^{-1} y, so its residual is the true one) on
 * an F64 CSR matrix, for nrhs in {1,2,3} right-hand sides sharing A (one
 * pass over A per product for all of them).  b, x: device double [nrhs][n]; stats:
 * host [nrhs].  On a breakdown the solve restarts once with r_hat = r.
 * Returns the worst status over the right-hand sides.  Synchronises. */
int oasis_bicgstab(void *stream, const oasis_csr *A, int32_t nrhs, const double *b,
                   double *x, const oasis_krylov_opts *opt, void *ws, size_t ws_bytes,
                   oasis_krylov_stats *stats);

/* ---- algebraic multigrid for the pressure correction -------------------- */
/* The paper's channel runs precondition the pressure-correction solve with
 * algebraic multigrid (Sec. 6.2, channel performance paragraph: a few
 * iterations per solve).  The method here is smoothed aggregation (Vanek,
 * Mandel & Brezina 1996): per level, strong couplings |a_ij| >= theta_l
 * sqrt(|a_ii a_jj|) with theta_l = theta / 2^l; greedy aggregation in index
 * order; the near-null vector B restricted to each aggregate as the
 * tentative prolongator; one damped Jacobi smoothing step on the filtered
 * matrix, weight (4/3) / (Gershgorin bound); Galerkin coarse matrices
 * P^T A P; a dense inverse on the coarsest level (regularised along its
 * near-null vector for a singular matrix).  The preconditioner is one
 * V(1,1) cycle with damped Jacobi smoothing, weight (4/3) / (Gershgorin
 * bound of D^-1 A) per level. */

typedef struct oasis_amg oasis_amg;   /* opaque host handle */

/* Default strength threshold: measured on the 129x129x97 channel, 0.125
 * keeps the structured mesh at 22-24 iterations per solve and cuts the
 * displaced mesh from 97 (0.25) to about 50. */
#define OASIS_AMG_THETA 0.125

typedef struct {
    double theta;         /* strength threshold of level 0, halved per level (0 = OASIS_AMG_THETA) */
    int32_t coarse_size;  /* a level of at most this many rows is the coarsest (0 = 1024;
                             at most 2048) */
    int32_t max_levels;   /* 0 = 12; at most 16 */
    int32_t precision;    /* values and vectors of the cycle: OASIS_F64 or OASIS_F32 (the CG
                             around it, its dot products and stopping test stay FP64) */
    int32_t flags;        /* OASIS_KRYLOV_NULLSPACE_CONST: A is singular with null vector B;
                             OASIS_AMG_HALF_LEVEL0: see below */
    oasis_tuning tuning;  /* storage of level 0 (an ELL copy when its rows fit, unless CSR)
                             and the grid cap of the CG and cycle kernels (0 = 768 here) */
} oasis_amg_params;

/* An FP32 cycle keeps level 0's ELL values as FP16 as well and its two
 * smoothing kernels read those (widened to FP32): the cycle then applies a
 * preconditioner built on A with its entries rounded to FP16 (relative
 * 2^-11), half the level-0 value bytes per cycle.  The CG around it still
 * multiplies by A in FP64 and stops on its FP64 residual.  Ignored for FP64
 * cycles or when level 0 has no ELL copy. */
#define OASIS_AMG_HALF_LEVEL0 4

/* Build the hierarchy of the symmetric positive (semi-)definite F64 CSR
 * matrix A (device; row_ptr, col_idx and val are kept by reference for the
 * handle's lifetime and used by the CG residuals).  B: device double [n],
 * the near-null-space vector (NULL = ones).  The set-up copies A to the host
 * and runs there, once per matrix.  Synchronises `stream`.  EUNSUPPORTED if
 * the coarsest level exceeds 2048 rows or its (regularised) matrix is not
 * positive definite. */
int oasis_amg_setup(void *stream, const oasis_csr *A, const double *B, const oasis_amg_params *par,
                    oasis_amg **out);

/* Device workspace that oasis_amg_upload needs for this hierarchy. */
int oasis_amg_workspace_size(const oasis_amg *h, size_t *bytes);

/* Copy the hierarchy into ws (device, kept by reference) and build level
 * 0's ELL copy; the handle's cycles and solves then run from ws.
 * Synchronises `stream`. */
int oasis_amg_upload(void *stream, oasis_amg *h, void *ws, size_t ws_bytes);

/* Host view of level `level` (0 = the input matrix) for inspection; the
 * pointers are host memory owned by the handle.  The prolongator and
 * aggregation fields are empty on the coarsest level, whose dense inverse
 * (row-major [n][n], as applied) is in coarse_inv. */
typedef struct {
    int32_t n, nnz;
    const int32_t *row_ptr, *col_idx;   /* the level matrix */
    const double *val;
    const double *near_null;            /* [n] */
    double omega;                       /* smoother weight (4/3) / Gershgorin bound */
    int32_t n_agg;                      /* rows of the next level (0 on the coarsest) */
    const int32_t *agg;                 /* [n] aggregate of every row */
    int32_t p_nnz;
    const int32_t *p_row_ptr, *p_col_idx;   /* prolongator [n][n_agg] */
    const double *p_val;
    const double *coarse_inv;           /* coarsest level only */
} oasis_amg_level_info;

int oasis_amg_levels(const oasis_amg *h, int32_t *n_levels);
int oasis_amg_level(const oasis_amg *h, int32_t level, oasis_amg_level_info *info);

/* z = M^{-1} r: one V(1,1) cycle from a zero start (r, z: device double
 * [n]; the cycle runs in the handle's precision).  Asynchronous. */
int oasis_amg_vcycle(void *stream, oasis_amg *h, const double *r, double *z);

/* CG on the handle's matrix preconditioned by one cycle per iteration:
 * b (device double [n]), x (device double [n], in: x0, out: solution).
 * opt: rtol, maxit, check_every and OASIS_KRYLOV_TIME (a solve stopped at
 * maxit then repeats its last cycle maxit times between two HIP events,
 * kernel_ms / kernel_count) are used.  With opt->precision OASIS_F32 on an
 * FP32 handle (and no timing) the CG itself is mixed: FP32 direction,
 * product and recursive residual, FP64 iterate and dot products, and an
 * FP64 residual b - A x that replaces the recursive one each time the
 * latter has fallen by opt->inner_rtol (0 = 1e-3) and decides convergence;
 * otherwise the CG is FP64.  Uses the uploaded workspace: calls on one handle
 * must not overlap.  Synchronises `stream`. */
int oasis_amg_pcg(void *stream, oasis_amg *h, const double *b, double *x, const oasis_krylov_opts *opt,
                  oasis_krylov_stats *stats);

int oasis_amg_destroy(oasis_amg *h);

/* ---- the IPCS time step (Alg. 1 with one inner iteration + Alg. 2) ------ */

typedef struct {
    double dt, nu;
    double f[3];              /* constant body force */
    int32_t n_bc;             /* velocity Dirichlet dofs (same set for all components) */
    const int32_t *bc_dofs;   /* device int32 [n_bc] */
    double rtol_u, rtol_p;    /* Krylov relative tolerances (true residual) */
    int32_t maxit;
    int32_t precision;        /* OASIS_F64 or OASIS_F32 (FP32 inner Krylov + FP64 refinement) */
    double inner_rtol;        /* F32 mode inner tolerance of the BiCGStab refinement (0 = 3e-5) */
    int32_t assembly;         /* per-step convection assembly: OASIS_ASSEMBLE_ROWS (each row
                                 gathers its cells' contributions; fused with the right-hand
                                 side and scaling) or OASIS_ASSEMBLE_COLORS (colour-by-colour
                                 element scatter as in oasis_assemble_p1); ROWS needs rows of
                                 at most 32 entries and falls back to COLORS otherwise */
    int32_t pressure_start;   /* plain start of the pressure-correction solve (the paper does
                                 not fix it): OASIS_PSTART_PREV (phi_prev, default) or
                                 OASIS_PSTART_ZERO (phi_0 = 0: solving for p from p*) */
    double pressure_delta;    /* F32 mode: the pressure CG replaces its FP32 residual by the FP64
                                 one each time the former fell by this factor (0 = 0.03); with a
                                 multigrid handle attached the pressure CG is FP64 */
    oasis_tuning tuning;      /* Krylov storage and kernel shapes of the step's solves */
    int32_t inner_iters;      /* Alg. 1's inner velocity-pressure iterations (0 = 1, at most 16):
                                 the coefficient matrix and the right-hand side's explicit part
                                 are built once; each iteration subtracts the gradient of the
                                 current p* (eq:dp_matrix), solves the tentative velocity (from
                                 U^{n-1}, then from the previous U^I) and the pressure correction
                                 (from the plain start, then from 0) and sets p* += phi; the
                                 velocity update uses the last correction */
    int32_t velocity_update;  /* OASIS_UPDATE_LUMPED: U^n = U^I - dt M_L^-1 dP^k phi (the channel
                                 runs of Sec. 6.2); OASIS_UPDATE_CONSISTENT: M U^n = M U^I -
                                 dt dP^k phi (eq:velocity_update) by Jacobi-PCG in FP64 to rtol_u,
                                 the Dirichlet dofs eliminated symmetrically;
                                 OASIS_UPDATE_GRADIENT: U^n = U^I - dt G^k phi with the weighted
                                 gradient matrix of Sec. 5 (last paragraphs), which the paper
                                 leaves undefined and is taken as the cell-volume-weighted nodal
                                 average of the cellwise gradient, G^k = M_L^-1 dP^k for P1,
                                 precomputed at create (dim more FP64 matrices on the pattern) */
    int32_t n_scalars;        /* passive scalars solved after the velocity update (Alg. 1),
                                 0..OASIS_MAX_SCALARS: eq:scalar_disc with the velocity's u_bar
                                 and Crank-Nicolson, i.e. (M/dt + C/2 + D K/2) c^n =
                                 (M/dt - C/2 - D K/2) c^{n-1} + f M_L, Dirichlet values on the
                                 velocity's Dirichlet dofs, BiCGStab + Jacobi to rtol_u in the
                                 step's precision */
    double diffusivity[4];    /* D_alpha of each scalar */
    double scalar_source[4];  /* constant f_alpha of each scalar */
    int32_t convection;       /* OASIS_CONV_ABCN: eq:convection_ABCN, A = M/dt + C(u_bar)/2 +
                                 nu K/2 assembled every step (Alg. 2); OASIS_CONV_ABE:
                                 eq:convection_ABE, fully explicit: A = M/dt + nu K/2 is constant
                                 and the right-hand side carries -1.5 C(u^{n-1}) U^{n-1} +
                                 0.5 C(u^{n-2}) U^{n-2}, gathered row by row from the cells.
                                 Scalars keep the u_bar form in either case. */
} oasis_ipcs_params;

#define OASIS_MAX_SCALARS 4
#define OASIS_ASSEMBLE_ROWS 0
#define OASIS_ASSEMBLE_COLORS 1
#define OASIS_PSTART_PREV 0
#define OASIS_PSTART_ZERO 1
#define OASIS_UPDATE_LUMPED 0
#define OASIS_UPDATE_CONSISTENT 1
#define OASIS_UPDATE_GRADIENT 2
#define OASIS_CONV_ABCN 0
#define OASIS_CONV_ABE 1

typedef struct oasis_ipcs oasis_ipcs;   /* opaque host handle */

/* Fields of one step; all device double arrays of length n_dof.
 *  U1[k]  U^{k,n-1}   (read)       U2[k]  U^{k,n-2} (read)
 *  Un[k]  U^{k,n}     (written; may not alias U1/U2)
 *  p      p* on entry, p^{n-1/2} (zero mean) on return
 *  phi    phi_prev on entry (the plain start of the pressure solve under
 *         OASIS_PSTART_PREV, and an input of an attached warm start), the
 *         new correction on return
 *  UI[k], b_phi: optional (NULL) outputs of the tentative velocity and the
 *  projected pressure right-hand side (of the last inner iteration).
 *  C1[a]  c_a^{n-1} (read), Cn[a] c_a^n (written), C_bc[a] its Dirichlet
 *  values at t^n (device double [n_bc]), for a < n_scalars. */
typedef struct {
    const double *U1[3];
    const double *U2[3];
    double *Un[3];
    double *p;
    double *phi;
    double *UI[3];
    double *b_phi;
    const double *C1[4];
    double *Cn[4];
    const double *C_bc[4];
} oasis_state;

typedef struct {
    int32_t iters_u[3], iters_p;  /* summed over inner iterations */
    int32_t outer_u, outer_p;
    int32_t status;           /* worst Krylov status of the step */
    int32_t guess_used;       /* 1 if the guess had a lower CG energy than the plain start */
    double res_u[3], res_p;   /* final true relative residuals (last inner iteration) */
    double ms_assemble, ms_velocity, ms_pressure, ms_update, ms_total;  /* HIP-event phase times;
                                 with inner iterations, ms_velocity is the first velocity solve
                                 and ms_pressure runs to the end of the last pressure solve */
    int32_t iters_m[3];       /* consistent update: CG iterations per component */
    int32_t iters_c[4];       /* BiCGStab iterations per scalar */
    double res_c[4];
    double ms_scalars;        /* scalar phase (included in ms_total) */
} oasis_step_stats;

/* Workspace for a handle on this mesh/pattern/params. */
int oasis_ipcs_workspace_size(const oasis_mesh *mesh, int32_t nnz,
                              const oasis_ipcs_params *par, size_t *bytes);

/* Preassemble M, K, dP^k, M_L and the constant part B = M/dt + nu K/2
 * (Sec. 5: matrices that do not change in time are assembled once).
 * row_ptr/col_idx: the P1 pattern of the mesh (device, kept by reference,
 * like the mesh arrays and bc_dofs, for the handle's lifetime).  The
 * handle is host memory; the workspace holds every matrix and vector.
 * Synchronises `stream`. */
int oasis_ipcs_create(void *stream, const oasis_mesh *mesh, const int32_t *row_ptr,
                      const int32_t *col_idx, int32_t nnz, const oasis_ipcs_params *par,
                      void *ws, size_t ws_bytes, oasis_ipcs **out);

/* One time step t^{n-1} -> t^n: u_bar, convection assembly with
 * A = M/dt + C/2 + nu K/2 and the right-hand side of eq:tent_intermediate1
 * (Alg. 2; with OASIS_CONV_ABE the constant A and the explicit convection
 * vector instead), pressure gradient (eq:dp_matrix), Dirichlet rows,
 * BiCGStab for all velocity components, pressure right-hand side
 * -(1/dt) sum_k dP^k U^I projected on 1-perp, Jacobi-PCG (or AMG-PCG) for
 * phi, p update and normalisation, velocity update (lumped, consistent or
 * gradient matrix), scalars.  bc_values: device double [dim][n_bc] at t^n.
 * phi_guess (device, nullable): a candidate initial guess for the
 * pressure solve; it is used only if its CG energy 1/2 x^T K x - b^T x is
 * below that of the plain start (par->pressure_start).  stats: host (nullable).
 * Synchronises `stream`. */
int oasis_ipcs_step(void *stream, oasis_ipcs *h, oasis_state *state,
                    const double *bc_values, const double *phi_guess,
                    oasis_step_stats *stats);

/* Attach (params != NULL) or detach (NULL) a learned warm start for the
 * pressure-correction solve: every later oasis_ipcs_step without an explicit
 * phi_guess runs the network (oasis_mpnn_forward) on the step's projected
 * right-hand side, phi_prev and the dof coordinates, and starts CG from the
 * prediction only if its CG energy is below that of the plain start
 * (par->pressure_start); the solve still stops at the same rtol.  params: device float
 * [OASIS_MPNN_NPARAM]; coords: device double [n_dof][dim]; ws: at least
 * oasis_mpnn_workspace_size(n_dof) bytes.  All three are kept by reference.
 * The step's forward pass keeps no activations in ws (it is inference only). */
int oasis_ipcs_set_warmstart(oasis_ipcs *h, const float *params, const double *coords,
                             void *ws, size_t ws_bytes);

/* Precondition the pressure-correction solve of every later step with an
 * uploaded multigrid handle (NULL: back to Jacobi).  The handle must have
 * been built on this step handle's scaled pressure matrix: A = the values
 * oasis_ipcs_matrix returns for OASIS_FORM_STIFF on the shared pattern, B
 * = its scaled_diag_sqrt, OASIS_KRYLOV_NULLSPACE_CONST (else EINVAL).  The
 * step then runs FP64 CG with one cycle per iteration (in the multigrid
 * handle's precision) to the same true-residual tolerance.  Kept by
 * reference; the two handles' calls must not overlap. */
int oasis_ipcs_set_amg(oasis_ipcs *h, oasis_amg *amg);

/* Device pointers to the handle's preassembled matrices (values on the
 * shared pattern) for inspection: which = OASIS_FORM_MASS, _STIFF (the
 * unscaled K is returned as scaled values plus sqrt of its diagonal, see
 * below) or _GRAD_X.. ; lumped mass via which = -1.  *scaled_diag_sqrt
 * (may be NULL) receives sqrt(diag K) for _STIFF, with K_ij = Ks_ij *
 * s_i * s_j.  State of the last step: OASIS_INSPECT_A (the tentative
 * matrix after Dirichlet rows, column-scaled: A_ij = val_ij * d_j),
 * OASIS_INSPECT_DIAG_A (d = diag A, [n]), OASIS_INSPECT_RHS + k (the
 * tentative right-hand side of component k, [n]).  Pointers stay valid
 * for the handle's lifetime; their contents change with every step. */
int oasis_ipcs_matrix(const oasis_ipcs *h, int32_t which, const double **val,
                      const double **scaled_diag_sqrt);

#define OASIS_INSPECT_A 100
#define OASIS_INSPECT_DIAG_A 101
#define OASIS_INSPECT_RHS 102

int oasis_ipcs_destroy(oasis_ipcs *h);

/* ---- learned warm start (message-passing network; not in the paper) ----- */

#define OASIS_MPNN_IN 6
#define OASIS_MPNN_HID 32
#define OASIS_MPNN_LAYERS 3
/* Parameter block (host or device float32, packed in this order):
 * We[32][6], ce[32], Ws[3][32][32], Wn[3][32][32], c[3][32], wd[32], cd[1] */
#define OASIS_MPNN_NPARAM (32 * 6 + 32 + 3 * 32 * 32 * 2 + 3 * 32 + 32 + 1)

/* Workspace for the network on an n-node graph (activations kept for the
 * backward pass). */
int oasis_mpnn_workspace_size(int32_t n, size_t *bytes);

/* Features and forward pass.  K: the pressure matrix as held by an IPCS
 * handle (scaled values Ks with Ks_ii = 1 and s = sqrt(diag K)); the edge
 * weights are w_ij = -K_ij / K_ii on off-diagonal entries.  b_phi, phi_prev:
 * device double [n]; coords: device double [n][dim] (dof coordinates);
 * params: device float [OASIS_MPNN_NPARAM].  Writes guess = phi_prev +
 * sigma * delta (device double [n], nullable) and delta (device float [n],
 * nullable); activations stay in ws for oasis_mpnn_backward. */
int oasis_mpnn_forward(void *stream, const oasis_csr *Ks, const double *s, int32_t dim,
                       const double *coords, const double *b_phi, const double *phi_prev,
                       const float *params, double *guess, float *delta,
                       void *ws, size_t ws_bytes);

/* Training losses of oasis_mpnn_backward, with target t = (phi -
 * phi_prev)/sigma and e = delta - t:
 *   MSE    mean over nodes of e^2;
 *   KNORM  e^T K e / t^T K t, the energy norm of the guess error relative
 *          to that of phi_prev (the error norm CG reduces; 0 with a zero
 *          gradient when t^T K t = 0). */
#define OASIS_MPNN_LOSS_MSE 0
#define OASIS_MPNN_LOSS_KNORM 1

/* The loss chosen by loss_kind (EINVAL otherwise) and the parameter
 * gradient (device float [OASIS_MPNN_NPARAM], overwritten) of the forward
 * pass whose activations ws holds; phi: the converged correction, device
 * double [n].  *loss_out: host, nullable (synchronises when given). */
int oasis_mpnn_backward(void *stream, const oasis_csr *Ks, const double *s,
                        const double *phi, const double *phi_prev, const float *params,
                        float *grad, int32_t loss_kind, double *loss_out,
                        void *ws, size_t ws_bytes);

/* Adam step on device float32 params with moments m, v (device float
 * [OASIS_MPNN_NPARAM], zero-initialised by the caller); t = 1, 2, ... */
int oasis_mpnn_adam(void *stream, float *params, const float *grad, float *m, float *v,
                    int32_t t, float lr, float beta1, float beta2, float eps);

/* ---- diagnostics ------------------------------------------------------- */
const char *oasis_strerror(int code);
int oasis_last_hip_error(void);
const char *oasis_version(void);

#ifdef __cplusplus
}
#endif
#endif /* OASIS_H */
