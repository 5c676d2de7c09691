// P1 element geometry and closed-form element matrices (FP64).
//
// For a simplex with vertices x_0..x_D: J = [x_1-x_0 .. x_D-x_0],
// vol = |det J| / D!, barycentric gradients g_i (i >= 1) are the rows of
// J^{-1}, g_0 = -sum g_i.  Integrals of products of two barycentric
// functions are exact: int l_i l_j = vol (1 + delta_ij) / ((D+1)(D+2)).
// Row index i = test function, column j = trial function:
//   mass        vol (1 + delta_ij) / ((D+1)(D+2))
//   stiffness   vol g_i . g_j
//   gradient k  vol g_j[k] / (D+1)                     (eq:dp_matrix)
//   convection  vol / ((D+1)(D+2)) * g_j . (S + u_i),  S = sum_m u_m
#pragma once

#include "internal.hpp"

namespace oasis {

template <int D>
struct Elem {
    double vol;
    double g[D + 1][D];
};

template <int D>
__device__ __forceinline__ void p1_element(const double (&x)[D + 1][D], Elem<D> &e);

template <>
__device__ __forceinline__ void p1_element<3>(const double (&x)[4][3], Elem<3> &e) {
    double a[3], b[3], c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a[k] = x[1][k] - x[0][k];
        b[k] = x[2][k] - x[0][k];
        c[k] = x[3][k] - x[0][k];
    }
    // rows of J^{-1}: (b x c), (c x a), (a x b) over det = a . (b x c)
    const double bc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
    const double ca[3] = {c[1] * a[2] - c[2] * a[1], c[2] * a[0] - c[0] * a[2], c[0] * a[1] - c[1] * a[0]};
    const double ab[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    const double det = a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2];
    const double inv = 1.0 / det;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        e.g[1][k] = bc[k] * inv;
        e.g[2][k] = ca[k] * inv;
        e.g[3][k] = ab[k] * inv;
        e.g[0][k] = -(e.g[1][k] + e.g[2][k] + e.g[3][k]);
    }
    e.vol = fabs(det) * (1.0 / 6.0);
}

template <>
__device__ __forceinline__ void p1_element<2>(const double (&x)[3][2], Elem<2> &e) {
    const double a0 = x[1][0] - x[0][0], a1 = x[1][1] - x[0][1];
    const double b0 = x[2][0] - x[0][0], b1 = x[2][1] - x[0][1];
    const double det = a0 * b1 - a1 * b0;
    const double inv = 1.0 / det;
    e.g[1][0] = b1 * inv;
    e.g[1][1] = -b0 * inv;
    e.g[2][0] = -a1 * inv;
    e.g[2][1] = a0 * inv;
    e.g[0][0] = -(e.g[1][0] + e.g[2][0]);
    e.g[0][1] = -(e.g[1][1] + e.g[2][1]);
    e.vol = fabs(det) * 0.5;
}

// Local matrix entry (i, j) of a form for one element.  ub: nodal u_bar
// at the element's vertices (CONV only).
template <int D>
__device__ __forceinline__ double p1_entry(int form, const Elem<D> &e, int i, int j,
                                           const double (&ub)[D + 1][D]) {
    constexpr double mfac = 1.0 / ((D + 1) * (D + 2));
    switch (form) {
        case OASIS_FORM_MASS:
            return e.vol * mfac * (i == j ? 2.0 : 1.0);
        case OASIS_FORM_STIFF: {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) s += e.g[i][k] * e.g[j][k];
            return e.vol * s;
        }
        case OASIS_FORM_CONV: {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                double S = 0.0;
#pragma unroll
                for (int m = 0; m < D + 1; ++m) S += ub[m][k];
                s += e.g[j][k] * (S + ub[i][k]);
            }
            return e.vol * mfac * s;
        }
        default: {  // gradient forms
            const int k = form - OASIS_FORM_GRAD_X;
            return e.vol * e.g[j][k] * (1.0 / (D + 1));
        }
    }
}

}  // namespace oasis
