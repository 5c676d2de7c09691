// Host construction of the smoothed-aggregation hierarchy (Vanek, Mandel,
// Brezina, Computing 56 (1996) 179-196), once per matrix.  The pressure
// matrix of the time step is constant over a run (Sec. 5: preassembled
// once), so the hierarchy is built once on the host and every cycle then
// runs on the device (amg.hip).
//
// Per level l, with theta_l = theta / 2^l (theta = OASIS_AMG_THETA unless
// the caller sets it):
//   strong couplings  |a_ij| >= theta_l sqrt(|a_ii a_jj|), i != j;
//   aggregation       three greedy passes in index order: (a) a node whose
//                     strong neighbours are all free starts an aggregate
//                     with them; (b) a free node joins the pass-(a)
//                     aggregate of its strongest strong neighbour; (c) the
//                     rest start aggregates with their free strong
//                     neighbours;
//   tentative P       B restricted to each aggregate, normalised; the
//                     coarse near-null vector is the norms;
//   smoothing         P = (I - w D_F^-1 A_F) P_t on the filtered matrix
//                     A_F (strong entries; weak ones added to the diagonal
//                     weighted by B unless that would halve it),
//                     w = (4/3) / rho(D_F^-1 A_F), rho estimated from above
//                     (rho_estimate; the smoother's weight likewise);
//   coarse matrix     A_c = P^T A P.
// The coarsest level (at most coarse_size rows) gets a dense inverse,
// regularised along its near-null vector when the matrix is singular.
#include <algorithm>
#include <cmath>

#include "amg.hpp"

namespace oasis {

namespace {

std::vector<double> diagonal(const HostCsr &A) {
    std::vector<double> d(A.n, 0.0);
    for (int i = 0; i < A.n; ++i)
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
            if (A.ci[k] == i) d[i] = A.v[k];
    return d;
}

std::vector<char> strength(const HostCsr &A, const std::vector<double> &d, double theta) {
    std::vector<char> s(A.ci.size(), 0);
    for (int i = 0; i < A.n; ++i)
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int j = A.ci[k];
            const double v = std::fabs(A.v[k]);
            s[k] = j != i && v != 0.0 && v >= theta * std::sqrt(std::fabs(d[i]) * std::fabs(d[j]));
        }
    return s;
}

int aggregate(const HostCsr &A, const std::vector<char> &S, std::vector<int> &agg) {
    const int n = A.n;
    agg.assign(n, -1);
    int na = 0;
    for (int i = 0; i < n; ++i) {            // (a)
        if (agg[i] >= 0) continue;
        bool free = true;
        for (int k = A.rp[i]; k < A.rp[i + 1] && free; ++k)
            if (S[k] && agg[A.ci[k]] >= 0) free = false;
        if (!free) continue;
        agg[i] = na;
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
            if (S[k]) agg[A.ci[k]] = na;
        ++na;
    }
    const std::vector<int> first(agg);
    for (int i = 0; i < n; ++i) {            // (b)
        if (agg[i] >= 0) continue;
        int best = -1;
        double bv = -1.0;
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int j = A.ci[k];
            if (j == i || first[j] < 0 || !S[k]) continue;
            const double v = std::fabs(A.v[k]);
            if (v > bv) {
                best = j;
                bv = v;
            }
        }
        if (best >= 0) agg[i] = first[best];
    }
    for (int i = 0; i < n; ++i) {            // (c)
        if (agg[i] >= 0) continue;
        agg[i] = na;
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
            if (S[k] && agg[A.ci[k]] < 0) agg[A.ci[k]] = na;
        ++na;
    }
    return na;
}

// Sparse accumulator for one output row: values by column plus the list of
// touched columns.
struct Spa {
    std::vector<double> val;
    std::vector<int> mark, cols;
    explicit Spa(int m) : val(m, 0.0), mark(m, -1) {}
    void add(int row, int c, double v) {
        if (mark[c] != row) {
            mark[c] = row;
            val[c] = v;
            cols.push_back(c);
        } else {
            val[c] += v;
        }
    }
    // append the row in increasing column order, without exact zeros, and
    // reset
    void flush(HostCsr &out) {
        std::sort(cols.begin(), cols.end());
        for (int c : cols) {
            if (val[c] == 0.0) continue;
            out.ci.push_back(c);
            out.v.push_back(val[c]);
        }
        out.rp.push_back(static_cast<int>(out.ci.size()));
        cols.clear();
    }
};

HostCsr matmul(const HostCsr &A, const HostCsr &B) {
    HostCsr C;
    C.n = A.n;
    C.m = B.m;
    C.rp.reserve(A.n + 1);
    C.rp.push_back(0);
    Spa spa(B.m);
    for (int i = 0; i < A.n; ++i) {
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int j = A.ci[k];
            const double a = A.v[k];
            for (int q = B.rp[j]; q < B.rp[j + 1]; ++q) spa.add(i, B.ci[q], a * B.v[q]);
        }
        spa.flush(C);
    }
    return C;
}

HostCsr transpose(const HostCsr &A) {
    HostCsr T;
    T.n = A.m;
    T.m = A.n;
    T.rp.assign(A.m + 1, 0);
    for (int c : A.ci) T.rp[c + 1]++;
    for (int i = 0; i < A.m; ++i) T.rp[i + 1] += T.rp[i];
    T.ci.resize(A.ci.size());
    T.v.resize(A.v.size());
    std::vector<int> pos(T.rp.begin(), T.rp.end() - 1);
    for (int i = 0; i < A.n; ++i)          // rows in increasing order: sorted columns
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int p = pos[A.ci[k]]++;
            T.ci[p] = i;
            T.v[p] = A.v[k];
        }
    return T;
}

double gershgorin(const HostCsr &A, const std::vector<double> &d) {
    double g = 0.0;
    for (int i = 0; i < A.n; ++i) {
        double rs = 0.0;
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) rs += std::fabs(A.v[k]);
        g = std::max(g, rs / std::fabs(d[i]));
    }
    return g;
}

// Estimate of rho(D^-1 A) from above: 15 power iterations on
// D^-1/2 A D^-1/2 (the same spectrum) from (+1, -1, +1, ...), 1.1 times the
// last Rayleigh quotient, capped by the Gershgorin bound.  The Gershgorin
// bound alone is loose where rows hold off-diagonals of both signs (P1
// tetrahedra, more so on distorted meshes) and then under-damps the
// prolongator and the smoother.
double rho_estimate(const HostCsr &A, const std::vector<double> &d) {
    const int n = A.n;
    std::vector<double> s(n), v(n), w(n);
    for (int i = 0; i < n; ++i) s[i] = 1.0 / std::sqrt(std::fabs(d[i]));
    const double v0 = 1.0 / std::sqrt(static_cast<double>(n));
    for (int i = 0; i < n; ++i) v[i] = (i % 2 == 0) ? v0 : -v0;
    double lam = 0.0;
    for (int it = 0; it < 15; ++it) {
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) acc += A.v[k] * (s[A.ci[k]] * v[A.ci[k]]);
            w[i] = s[i] * acc;
        }
        double vw = 0.0, ww = 0.0;
        for (int i = 0; i < n; ++i) {
            vw += v[i] * w[i];
            ww += w[i] * w[i];
        }
        lam = vw;
        const double inv = 1.0 / std::sqrt(ww);
        for (int i = 0; i < n; ++i) v[i] = w[i] * inv;
    }
    return std::min(gershgorin(A, d), 1.1 * lam);
}

// Filtered matrix: the diagonal and the strong entries; the dropped ones
// are added to the diagonal weighted by B, unless the diagonal would fall
// to half its value or below.
HostCsr filtered(const HostCsr &A, const std::vector<char> &S, const std::vector<double> &B,
                 const std::vector<double> &d) {
    HostCsr F;
    F.n = A.n;
    F.m = A.m;
    F.rp.push_back(0);
    for (int i = 0; i < A.n; ++i) {
        double lump = 0.0;
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int j = A.ci[k];
            if (j != i && !S[k]) lump += A.v[k] * B[j];
        }
        lump /= B[i];
        if (!(d[i] + lump > 0.5 * d[i])) lump = 0.0;
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int j = A.ci[k];
            double v;
            if (j == i)
                v = A.v[k] + lump;
            else if (S[k])
                v = A.v[k];
            else
                continue;
            if (v == 0.0) continue;
            F.ci.push_back(j);
            F.v.push_back(v);
        }
        F.rp.push_back(static_cast<int>(F.ci.size()));
    }
    return F;
}

// Inverse of a dense SPD matrix (row-major, n x n) by Cholesky; false if a
// pivot is not positive.
bool spd_inverse(int n, std::vector<double> &M) {
    std::vector<double> L(static_cast<size_t>(n) * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double s = M[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > 0.0)) return false;
        const double ljj = std::sqrt(s);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = M[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / ljj;
        }
    }
    // W = L^-1 (lower triangular), column by column of the identity
    std::vector<double> W(static_cast<size_t>(n) * n, 0.0);
    for (int c = 0; c < n; ++c)
        for (int i = c; i < n; ++i) {
            double t = i == c ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) t -= L[(size_t)i * n + k] * W[(size_t)k * n + c];
            W[(size_t)i * n + c] = t / L[(size_t)i * n + i];
        }
    // M^-1 = W^T W
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double t = 0.0;
            for (int k = i; k < n; ++k) t += W[(size_t)k * n + i] * W[(size_t)k * n + j];
            M[(size_t)i * n + j] = t;
            M[(size_t)j * n + i] = t;
        }
    return true;
}

}  // namespace

int amg_build(const HostCsr &A0, const std::vector<double> &B0, const AmgHostParams &p,
              std::vector<HostLevel> &levels, std::vector<double> &coarse_inv) {
    levels.clear();
    levels.emplace_back();
    levels[0].A = A0;
    levels[0].B = B0;
    for (int l = 0;; ++l) {
        HostLevel &lv = levels[l];
        const std::vector<double> d = diagonal(lv.A);
        for (int i = 0; i < lv.A.n; ++i)
            if (!(d[i] != 0.0) || !std::isfinite(d[i])) return OASIS_EINVAL;
        lv.omega = (4.0 / 3.0) / rho_estimate(lv.A, d);
        if (lv.A.n <= p.coarse_size || l + 1 == p.max_levels || l + 1 == kAmgMaxLevels) break;
        const double theta = p.theta * std::pow(0.5, l);
        const std::vector<char> S = strength(lv.A, d, theta);
        std::vector<int> agg;
        const int na = aggregate(lv.A, S, agg);
        if (na >= lv.A.n) break;            // no coarsening possible
        // tentative prolongator and the coarse near-null vector
        std::vector<double> nrm(na, 0.0);
        for (int i = 0; i < lv.A.n; ++i) nrm[agg[i]] += lv.B[i] * lv.B[i];
        for (double &v : nrm) v = std::sqrt(v);
        HostCsr Pt;
        Pt.n = lv.A.n;
        Pt.m = na;
        Pt.rp.resize(lv.A.n + 1);
        Pt.ci.resize(lv.A.n);
        Pt.v.resize(lv.A.n);
        for (int i = 0; i < lv.A.n; ++i) {
            Pt.rp[i] = i;
            Pt.ci[i] = agg[i];
            Pt.v[i] = lv.B[i] / nrm[agg[i]];
        }
        Pt.rp[lv.A.n] = lv.A.n;
        // smoothed prolongator
        const HostCsr F = filtered(lv.A, S, lv.B, d);
        const std::vector<double> dF = diagonal(F);
        const double w = (4.0 / 3.0) / rho_estimate(F, dF);
        HostCsr FP = matmul(F, Pt);
        HostCsr P;
        P.n = lv.A.n;
        P.m = na;
        P.rp.push_back(0);
        for (int i = 0; i < lv.A.n; ++i) {
            const double dinv = 1.0 / dF[i];
            bool has_own = false;
            for (int k = FP.rp[i]; k < FP.rp[i + 1]; ++k) {
                const int c = FP.ci[k];
                const double own = c == agg[i] ? Pt.v[i] : 0.0;
                has_own = has_own || c == agg[i];
                const double v = own - w * (dinv * FP.v[k]);
                if (v == 0.0) continue;
                P.ci.push_back(c);
                P.v.push_back(v);
            }
            if (!has_own) {                 // the row's own aggregate, kept in column order
                P.ci.push_back(agg[i]);
                P.v.push_back(Pt.v[i]);
                const int s0 = P.rp.back();
                for (int k = static_cast<int>(P.ci.size()) - 1; k > s0 && P.ci[k] < P.ci[k - 1]; --k) {
                    std::swap(P.ci[k], P.ci[k - 1]);
                    std::swap(P.v[k], P.v[k - 1]);
                }
            }
            P.rp.push_back(static_cast<int>(P.ci.size()));
        }
        // Galerkin coarse matrix
        const HostCsr AP = matmul(lv.A, P);
        const HostCsr R = transpose(P);
        HostLevel next;
        next.A = matmul(R, AP);
        next.B = nrm;
        lv.agg = std::move(agg);
        lv.n_agg = na;
        lv.P = std::move(P);
        lv.R = R;
        levels.push_back(std::move(next));
    }
    // dense inverse of the coarsest level
    const HostLevel &cl = levels.back();
    const int nc = cl.A.n;
    if (nc > kAmgMaxCoarse) return OASIS_EUNSUPPORTED;
    coarse_inv.assign(static_cast<size_t>(nc) * nc, 0.0);
    for (int i = 0; i < nc; ++i)
        for (int k = cl.A.rp[i]; k < cl.A.rp[i + 1]; ++k) coarse_inv[(size_t)i * nc + cl.A.ci[k]] = cl.A.v[k];
    if (p.singular) {
        double bb = 0.0, sig = 0.0;
        for (int i = 0; i < nc; ++i) {
            bb += cl.B[i] * cl.B[i];
            sig += coarse_inv[(size_t)i * nc + i];
        }
        sig /= nc;
        const double nb = std::sqrt(bb);
        for (int i = 0; i < nc; ++i)
            for (int j = 0; j < nc; ++j) coarse_inv[(size_t)i * nc + j] += sig * (cl.B[i] / nb) * (cl.B[j] / nb);
    }
    if (!spd_inverse(nc, coarse_inv)) return OASIS_EUNSUPPORTED;
    return OASIS_OK;
}

}  // namespace oasis
