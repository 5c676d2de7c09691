"""Smoothed-aggregation algebraic multigrid as a preconditioner of CG (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's channel runs solve the pressure correction with a symmetric
Krylov method preconditioned by algebraic multigrid, which brings the
iteration count to a handful per solve (Sec. 6.2, channel performance
paragraph), against O(10^3) for Jacobi.  The paper delegates the multigrid
to an external library and does not define it; the method here is
smoothed aggregation (SA) as published by Vanek, Mandel and Brezina,
"Algebraic multigrid by smoothed aggregation for second and fourth order
elliptic problems", Computing 56 (1996) 179-196, written out step by step:

1. strength of connection: i != j are strongly coupled when
   |a_ij| >= theta_l * sqrt(|a_ii a_jj|), with the threshold halved from
   each level to the next, theta_l = theta / 2^l, as in their schedule
2. aggregation by the three greedy passes of their Sec. 3:
   (a) visiting nodes in index order, a node none of whose strong
       neighbours is aggregated yet starts an aggregate with all of them;
   (b) every node still free joins an aggregate of pass (a) that it is
       strongly coupled to;
   (c) the nodes still free start aggregates with their free strong
       neighbours, again in index order;
3. tentative prolongator: on each aggregate the near-null-space vector B
   restricted to it, normalised (a one-column QR), and the coarse
   near-null vector B_c = the norms;
4. prolongator smoothing with one damped Jacobi step on the filtered
   matrix A^F:  P = (I - omega D_F^{-1} A^F) P_tent,  omega = (4/3) / rho,
   with rho an estimate of the spectral radius of D_F^{-1} A^F from above;
5. Galerkin coarse operator A_c = P^T A P; recurse until a level has at
   most `coarse_size` rows, which is solved exactly (a dense inverse,
   regularised along B_c when the matrix is singular);
6. the V(1,1) cycle with damped Jacobi pre- and post-smoothing and
   restriction P^T, which is a symmetric positive (semi-)definite
   preconditioner for CG.

Readings taken where the published method leaves a choice:
* Pass (b) joins the aggregate of the strongest strong neighbour (largest
  |a_ij|, lowest column index on a tie) among the nodes aggregated by pass
  (a), so a node that joins in pass (b) never recruits another.
* The filtered matrix A^F keeps the diagonal and the strong entries and
  adds each dropped entry to the diagonal weighted by B: a^F_ii = a_ii +
  sum_(j weak) a_ij B_j / B_i, so that A^F B = A B (for the pure-Neumann
  pressure matrix, A B = 0 and the smoothed prolongator keeps B exactly).
  A row whose lumped diagonal would fall to half of a_ii or below (a node
  with few or no strong couplings, whose weak entries nearly cancel its
  diagonal) keeps a_ii instead.
* rho is estimated by 15 power iterations on D^{-1/2} A D^{-1/2} (the same
  spectrum as D^{-1} A) from the alternating vector (+1, -1, +1, ...): 1.1
  times the last Rayleigh quotient, capped by the Gershgorin bound
  max_i sum_j |a_ij| / |a_ii|.  The Gershgorin bound alone is safe but loose
  where the off-diagonals have both signs (P1 tetrahedra): 2.23 against a
  spectral radius of 2.00 on the structured channel, 2.87 against 2.08 on
  the displaced one, which under-damps both the prolongator and the
  smoother (18 and 40 AMG-PCG iterations on 49x49x37, against 16 and 32
  with the estimate).  The smoother uses the same estimate for A itself:
  x <- x + omega_s D^{-1} (b - A x), omega_s = (4/3) / rho(D^{-1} A).
* The level-0 threshold defaults to theta = 0.125.  The method leaves it
  to the user; 0.125 was chosen by a sweep of the pressure solve on the
  129x129x97 channel (0.09-0.25), where it keeps the structured mesh at
  22-24 iterations and halves those of the displaced mesh against 0.25.
* A singular coarsest matrix (null vector B_c) is inverted as
  (A_c + sigma b b^T)^{-1} with b = B_c / ||B_c|| and sigma the mean of
  diag(A_c); on b-orthogonal right-hand sides this is the pseudo-inverse.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from .krylov import BREAKDOWN, NAN, NOTCONV, OK, KrylovResult


def strength(A, theta):
    """Boolean CSR mask (same pattern as A) of the strong off-diagonal
    entries: |a_ij| >= theta sqrt(|a_ii a_jj|), i != j, a_ij != 0."""
    A = sp.csr_matrix(A)
    d = np.abs(A.diagonal())
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    v = np.abs(A.data)
    strong = (rows != cols) & (v != 0.0) & (v >= theta * np.sqrt(d[rows] * d[cols]))
    return sp.csr_matrix((strong, cols, A.indptr), shape=A.shape)


def aggregate(A, S):
    """Greedy three-pass aggregation on the strong graph S.  Returns
    agg [n] (aggregate of every node, numbered in order of creation) and the
    number of aggregates."""
    n = A.shape[0]
    A = sp.csr_matrix(A)
    nbrs = [S.indices[S.indptr[i]:S.indptr[i + 1]][S.data[S.indptr[i]:S.indptr[i + 1]]] for i in range(n)]
    agg = np.full(n, -1, dtype=np.int64)
    na = 0
    # (a) nodes whose whole strong neighbourhood is free start an aggregate
    for i in range(n):
        if agg[i] >= 0:
            continue
        if all(agg[j] < 0 for j in nbrs[i]):
            agg[i] = na
            for j in nbrs[i]:
                agg[j] = na
            na += 1
    first = agg.copy()
    # (b) free nodes join the pass-(a) aggregate of their strongest strong neighbour
    for i in range(n):
        if agg[i] >= 0:
            continue
        best, bv = -1, -1.0
        lo, hi = A.indptr[i], A.indptr[i + 1]
        for jj in range(lo, hi):
            j = A.indices[jj]
            if j == i or first[j] < 0 or not _is_strong(S, i, j):
                continue
            v = abs(A.data[jj])
            if v > bv:
                best, bv = j, v
        if best >= 0:
            agg[i] = first[best]
    # (c) the rest start aggregates with their free strong neighbours
    for i in range(n):
        if agg[i] >= 0:
            continue
        agg[i] = na
        for j in nbrs[i]:
            if agg[j] < 0:
                agg[j] = na
        na += 1
    return agg, na


def _is_strong(S, i, j):
    lo, hi = S.indptr[i], S.indptr[i + 1]
    k = lo + np.searchsorted(S.indices[lo:hi], j)
    return k < hi and S.indices[k] == j and bool(S.data[k])


def tentative(agg, na, B):
    """P_tent [n, na] with P[i, agg[i]] = B_i / ||B restricted to agg[i]||,
    and the coarse near-null vector B_c [na] = those norms."""
    n = agg.size
    nrm = np.sqrt(np.bincount(agg, weights=B * B, minlength=na))
    P = sp.csr_matrix((B / nrm[agg], (np.arange(n), agg)), shape=(n, na))
    return P, nrm


def filtered(A, S, B):
    """A^F: diagonal and strong entries of A; each dropped off-diagonal
    entry is added to the diagonal weighted by B (A^F B = A B)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    keep = (rows == cols) | S.data.astype(bool)
    drop = ~keep
    lump = np.bincount(rows[drop], weights=A.data[drop] * B[cols[drop]], minlength=n) / B
    d = A.diagonal()
    lump = np.where(d + lump > 0.5 * d, lump, 0.0)
    AF = sp.csr_matrix((np.where(keep, A.data, 0.0), cols, A.indptr), shape=A.shape)
    AF = AF + sp.diags(lump)
    AF.eliminate_zeros()
    return AF.tocsr()


def gershgorin(A):
    """max_i sum_j |a_ij| / |a_ii|: an upper bound of rho(D^{-1} A)."""
    A = sp.csr_matrix(A)
    rs = np.asarray(abs(A).sum(axis=1)).ravel()
    return float(np.max(rs / np.abs(A.diagonal())))


def rho_estimate(A, iters=15, safety=1.1):
    """Estimate of rho(D^{-1} A) from above (see the module notes): power
    iterations on D^{-1/2} A D^{-1/2} from (+1, -1, ...), safety times the
    last Rayleigh quotient, capped by the Gershgorin bound."""
    A = sp.csr_matrix(A)
    s = 1.0 / np.sqrt(np.abs(A.diagonal()))
    v = np.where(np.arange(A.shape[0]) % 2 == 0, 1.0, -1.0)
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = s * (A @ (s * v))
        lam = float(v @ w)
        v = w / np.linalg.norm(w)
    return min(gershgorin(A), safety * lam)


def smoothed_prolongator(A, S, B, agg, na):
    Pt, Bc = tentative(agg, na, B)
    AF = filtered(A, S, B)
    omega = (4.0 / 3.0) / rho_estimate(AF)
    P = Pt - omega * (sp.diags(1.0 / AF.diagonal()) @ (AF @ Pt))
    return sp.csr_matrix(P), Bc, Pt


@dataclasses.dataclass
class Level:
    A: sp.csr_matrix
    P: sp.csr_matrix | None = None       # to the next level
    agg: np.ndarray | None = None
    B: np.ndarray | None = None
    omega: float = 0.0                   # smoother weight (4/3) / rho(D^{-1} A)


@dataclasses.dataclass
class Hierarchy:
    levels: list
    coarse_inv: np.ndarray               # dense inverse of the coarsest level
    singular: bool

    def operator_complexity(self):
        return sum(lv.A.nnz for lv in self.levels) / self.levels[0].A.nnz


def hierarchy(A, B=None, theta=0.125, coarse_size=1024, max_levels=12, singular=False):
    """Smoothed-aggregation hierarchy of the SPD (or, with `singular`,
    SPSD with null vector B) matrix A.  B: near-null-space vector (ones when
    None).  The strength threshold of level l is theta / 2^l."""
    A = sp.csr_matrix(A, dtype=np.float64, copy=True)
    A.sort_indices()
    B = np.ones(A.shape[0]) if B is None else np.asarray(B, dtype=np.float64)
    levels = []
    while True:
        lv = Level(A=A, B=B, omega=(4.0 / 3.0) / rho_estimate(A))
        levels.append(lv)
        if A.shape[0] <= coarse_size or len(levels) == max_levels:
            break
        S = strength(A, theta * 0.5 ** (len(levels) - 1))
        agg, na = aggregate(A, S)
        if na >= A.shape[0]:
            break                         # no coarsening possible
        P, Bc, _ = smoothed_prolongator(A, S, B, agg, na)
        lv.P, lv.agg = P, agg
        A = sp.csr_matrix(P.T @ A @ P)
        A.sort_indices()
        B = Bc
    Ac = levels[-1].A.toarray()
    if singular:
        b = levels[-1].B / np.linalg.norm(levels[-1].B)
        sigma = float(np.mean(np.diag(Ac)))
        Ac = Ac + sigma * np.outer(b, b)
    return Hierarchy(levels, np.linalg.inv(Ac), singular)


def vcycle(H, b, level=0):
    """One V(1,1) cycle from a zero start: M^{-1} b."""
    lv = H.levels[level]
    if level == len(H.levels) - 1:
        return H.coarse_inv @ b
    A, d, w = lv.A, lv.A.diagonal(), lv.omega
    x = w * b / d                                   # pre-smoothing from x = 0
    r = b - A @ x
    xc = vcycle(H, lv.P.T @ r, level + 1)
    x = x + lv.P @ xc                               # coarse-grid correction
    x = x + w * (b - A @ x) / d                     # post-smoothing
    return x


def amg_pcg(A, b, x0, H, rtol=1e-8, maxit=1000):
    """Preconditioned CG (Hestenes-Stiefel) with one V-cycle per iteration,
    stopped on the true residual as the Jacobi-PCG of krylov.py."""
    x = np.array(x0, dtype=np.float64, copy=True)
    bnorm = float(np.linalg.norm(b))
    tol = rtol * bnorm
    r = b - A @ x
    if not np.all(np.isfinite(r)):
        return KrylovResult(x, 0, float("nan"), NAN, [])
    if np.linalg.norm(r) <= tol:
        return KrylovResult(x, 0, float(np.linalg.norm(r) / bnorm) if bnorm else 0.0, OK, [])
    z = vcycle(H, r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    while it < maxit:
        q = A @ p
        pq = float(p @ q)
        if pq == 0.0 or not np.isfinite(pq):
            return KrylovResult(x, it, float("nan"), BREAKDOWN if pq == 0.0 else NAN, [])
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        if np.linalg.norm(r) <= tol:
            r = b - A @ x                           # confirm on the true residual
            if np.linalg.norm(r) <= tol:
                return KrylovResult(x, it, float(np.linalg.norm(r) / bnorm), OK, [])
        z = vcycle(H, r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return KrylovResult(x, it, float(np.linalg.norm(b - A @ x) / bnorm), NOTCONV, [])
