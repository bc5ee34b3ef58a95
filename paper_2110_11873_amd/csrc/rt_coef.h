// rt_coef.h -- step coefficients of the formal solvers (device code shared by
// the sweep and the dense assembly).
#pragma once

#include <hip/hip_runtime.h>

#include "rt.h"

namespace rt {

// --------------------------------------------------------------------------
// Step coefficients of one interval with optical step d (FP64).
//
// DELO-linear (exact integral of a linearly interpolated source along the
// ray, Sect. 4.1): c_u = int_0^d (s/d) e^{-s} ds = (1 - (1 + d) e^{-d}) / d,
// c_k = (1 - e^{-d}) - c_u.  Below d = 0.1 the closed forms cancel; their
// Taylor series sum_{n>=2} (-1)^n (n-1) d^(n-1)/n! and
// sum_{n>=2} (-1)^n d^(n-1)/n! are evaluated by Horner's rule instead.
// Trapezoidal (Crank-Nicolson): c_u = c_k = (d/2) / (1 + d/2).  Implicit Euler
// (backward difference): c_u = 0, c_k = d / (1 + d).
// --------------------------------------------------------------------------
namespace {

constexpr int kSeriesTerms = 14;  // n = 2 .. 15: below 1e-20 relative at d = 0.1

struct SeriesCoef {
    double u[kSeriesTerms];
    double k[kSeriesTerms];
};

constexpr SeriesCoef make_series() {
    SeriesCoef s{};
    double fact = 1.0;  // n!
    for (int n = 1; n <= kSeriesTerms + 1; ++n) {
        fact *= n;
        if (n >= 2) {
            const double sgn = (n % 2 == 0) ? 1.0 : -1.0;
            s.u[n - 2] = sgn * (n - 1) / fact;
            s.k[n - 2] = sgn / fact;
        }
    }
    return s;
}

// compile-time tables: immutable, so the compiler folds each coefficient into
// the instruction that uses it instead of keeping the table in registers
constexpr SeriesCoef c_series = make_series();

}  // namespace

__device__ inline void step_coef(int fs, double d, double &cu, double &ck) {
    if (fs == RT_FS_TRAPEZOIDAL) {
        const double h = 0.5 * d;
        cu = ck = h / (1.0 + h);
        return;
    }
    if (fs == RT_FS_IMPLICIT_EULER) {
        cu = 0.0;
        ck = d / (1.0 + d);
        return;
    }
    if (d < 0.1) {
        double pu = c_series.u[kSeriesTerms - 1];
        double pk = c_series.k[kSeriesTerms - 1];
#pragma unroll
        for (int t = kSeriesTerms - 2; t >= 0; --t) {
            pu = fma(pu, d, c_series.u[t]);
            pk = fma(pk, d, c_series.k[t]);
        }
        cu = pu * d;
        ck = pk * d;
    } else {
        const double e = exp(-d);
        const double w0 = -expm1(-d);
        const double w1 = w0 - d * e;
        cu = w1 / d;
        ck = w0 - cu;
    }
}

// Step coefficients in the form the sweep uses: E = e^{-d} (trapezoid:
// (1 - d/2) / (1 + d/2)) and w = 1 - c_k = E + c_u, with which the step
// becomes I_k - S_k = E (I_u - S_u) + w (S_u - S_k).
__device__ inline void step_ew(int fs, double d, double &E, double &w) {
    if (fs == RT_FS_TRAPEZOIDAL) {
        const double h = 0.5 * d;
        E = (1.0 - h) / (1.0 + h);
        w = 1.0 / (1.0 + h);
        return;
    }
    if (fs == RT_FS_IMPLICIT_EULER) {  // c_u = 0: E = w = 1 - c_k
        E = w = 1.0 / (1.0 + d);
        return;
    }
    double cu, ck;
    step_coef(fs, d, cu, ck);
    E = exp(-d);
    w = E + cu;
}

// --------------------------------------------------------------------------
// DELO-parabolic step (Sect. 4.1; without dichroism DELOPAR is the same
// step).  t is the optical path from the current point back to the upwind
// one (t = d there); the source is the parabola through the upwind, current
// and downwind (t = -dd) points, and the coefficients are the integrals of
// exp(-t) against its Lagrange basis:
//   c_u = (w2 + dd w1) / (d (d + dd)),  c_k = ((d - dd) w1 + d dd w0 - w2) / (d dd),
//   c_d = (w2 - d w1) / (dd (d + dd)),
// with the moments w_n = int_0^d t^n exp(-t) dt: 1 - E, 1 - (1 + d) E,
// 2 - (d^2 + 2d + 2) E, or below d = 1 the incomplete-gamma series of w_2
// and a downward recurrence (exp_moments).
// --------------------------------------------------------------------------
namespace {

constexpr int kGammaTerms = 20;  // d < 1: 2 / 22! ~ 1.8e-21 of the leading 1/3

// c[k] = 2 / (k + 3)!: gamma(3, d) = d^3 e^-d sum_k c[k] d^k (all terms positive)
struct GammaSeries {
    double c[kGammaTerms];
};

constexpr GammaSeries make_gamma_series() {
    GammaSeries s{};
    double fact = 6.0;  // (k + 3)!
    for (int k = 0; k < kGammaTerms; ++k) {
        if (k > 0) fact *= (k + 3);
        s.c[k] = 2.0 / fact;
    }
    return s;
}

constexpr GammaSeries c_gamma3 = make_gamma_series();

}  // namespace

// E = e^-d and the moments w_n = int_0^d t^n e^-t dt = gamma(n + 1, d),
// n = 0, 1, 2.  Below d = 1: gamma(3, d) from its positive series, then the
// stable downward recurrence gamma(s, d) = (gamma(s + 1, d) + d^s e^-d) / s;
// above: the closed forms, free of cancellation there.
__device__ inline void exp_moments(double d, double &E, double &w0, double &w1, double &w2) {
    E = exp(-d);
    if (d < 1.0) {
        double sr = c_gamma3.c[kGammaTerms - 1];
#pragma unroll
        for (int k = kGammaTerms - 2; k >= 0; --k) sr = fma(sr, d, c_gamma3.c[k]);
        const double dE = d * E;
        w2 = d * d * dE * sr;
        w1 = 0.5 * fma(d, dE, w2);
        w0 = w1 + dE;
    } else {
        w0 = 1.0 - E;
        w1 = 1.0 - (1.0 + d) * E;
        w2 = 2.0 - (d * d + 2.0 * d + 2.0) * E;
    }
}

// Quadratic (DELO-parabolic) step coefficients from the moments, with one
// reciprocal of d dd (d + dd).
__device__ inline void parabolic_coef(double d, double dd, double &E, double &cu, double &ck,
                                      double &cd) {
    double w0, w1, w2;
    exp_moments(d, E, w0, w1, w2);
    const double s = d + dd, inv = 1.0 / (d * dd * s);
    cu = (w2 + dd * w1) * dd * inv;
    ck = ((d - dd) * w1 + d * dd * w0 - w2) * s * inv;
    cd = (w2 - d * w1) * d * inv;
}

__device__ inline void ray_step(int fs, double d, double dd, bool has_dn, double &E,
                                double &cu, double &ck, double &cd) {
    cd = 0.0;
    if (fs == RT_FS_DELO_PARABOLIC && has_dn) {
        parabolic_coef(d, dd, E, cu, ck, cd);
        return;
    }
    if (fs == RT_FS_TRAPEZOIDAL) {
        const double h = 0.5 * d;
        E = (1.0 - h) / (1.0 + h);
        cu = ck = h / (1.0 + h);
        return;
    }
    if (fs == RT_FS_IMPLICIT_EULER) {
        E = 1.0 / (1.0 + d);
        cu = 0.0;
        ck = d / (1.0 + d);
        return;
    }
    // DELO-linear with one exponential: below d = 0.1 the series gives c_u
    // and c_k and E = 1 - (c_u + c_k) (a constant source is transmitted
    // exactly, so c_u + c_k = 1 - E); above it 1 - E >= 0.095 carries no
    // cancellation.
    if (d < 0.1) {
        step_coef(RT_FS_DELO_LINEAR, d, cu, ck);
        E = 1.0 - (cu + ck);
    } else {
        E = exp(-d);
        const double w0 = 1.0 - E;
        cu = (w0 - d * E) / d;
        ck = w0 - cu;
    }
}

// Lambda(k, k) of one DELO-parabolic ray through depth k, walking toward
// larger depth indices (step = 1) or smaller (step = -1): the source at k
// enters I_k through c_k of the step into k and, through c_d of the step into
// the point before k (when that point is not the ray's entry), I there,
// which reaches k with the factor E of the step into k.
__device__ inline double parabolic_diag(const double *tau, int ns, int k, double kap, int step) {
    const int i = step > 0 ? k : ns - 1 - k;  // position along the ray
    if (i == 0) return 0.0;
    const int u = k - step, dn = k + step;
    const bool has_dn = i < ns - 1;
    double E, cu, ck, cd;
    ray_step(RT_FS_DELO_PARABOLIC, kap * fabs(tau[k] - tau[u]),
             has_dn ? kap * fabs(tau[dn] - tau[k]) : 1.0, has_dn, E, cu, ck, cd);
    double lam = ck;
    if (i >= 2) {
        double E2, cu2, ck2, cd2;
        ray_step(RT_FS_DELO_PARABOLIC, kap * fabs(tau[u] - tau[u - step]),
                 kap * fabs(tau[k] - tau[u]), true, E2, cu2, ck2, cd2);
        lam += E * cd2;
    }
    return lam;
}

}  // namespace rt
