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

__constant__ SeriesCoef c_series = make_series();

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

}  // namespace rt
