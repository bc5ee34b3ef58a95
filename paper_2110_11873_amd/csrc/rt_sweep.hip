// rt_sweep.hip -- the operator A = Id - J Lambda T on gfx950.
//
// Algorithm 1 of the paper computes S = T sigma, then a formal solution along
// every ray (mu_m, nu_p) with zero incoming radiation, then the quadrature of
// eqs. J00/J02.  This file fuses the three steps into one launch:
//
//  * T step (eqs. sourceI/sourceQ).  S_I = s00 + T1(mu) s20, S_Q = T2(mu) s20
//    with T1, T2 functions of mu^2 only, so the rays mu and -mu see the same
//    source.  The formal solver is linear, so Lambda S_I = Lambda s00 +
//    T1 Lambda s20 and Lambda S_Q = T2 Lambda s20: each lane runs two
//    recurrences per direction (sources s00 and s20) and the T factors are
//    applied when the intensities are weighted into the quadrature.
//  * Lambda step (eqs. RTE_delo1/2).  One lane owns one chunk of one ray
//    pair (|mu|, nu); it sweeps its chunk downward (the mu < 0 ray) and upward
//    (the mu > 0 ray) with the step I_k = E I_u + c_u S_u + c_k S_k,
//    E = 1 - c_u - c_k (true of both DELO-linear and the trapezoidal rule,
//    which reproduce a constant source exactly).  The C chunks of a ray sit in
//    C adjacent lanes; a chunk is swept once with zero inflow, the affine
//    maps I_out = P I_in + e of the chunks are composed by a lane scan
//    (row-local DPP shifts, then row broadcasts), and the inflow's share T_k I_in (T_k
//    the transmission from the chunk's entry to point k, kept from the sweep)
//    is added at every point.  The step coefficients are read once per
//    launch, in a tile order where a wavefront's 64 lanes read 64 consecutive
//    pairs, one ray batch ahead of use.
//  * J step (eqs. J00/J02, S00/S02).  Each lane accumulates
//    q (I_down + I_up) and the T-weighted combination for J20 over all the
//    rays it handles, in registers; the rays of a wave are summed by an xor
//    butterfly, the waves of a block in LDS in a fixed order, and each block
//    stores its sums in a slot of its own.  A second, light pass adds a
//    slab's slots in block order and applies the scattering step.  No
//    atomics and no device-wide fences (which on gfx950 write back and
//    invalidate a whole L2): results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "rt_internal.h"

namespace rt {

// --------------------------------------------------------------------------
// Step coefficients of one interval with optical step d (FP64).
//
// DELO-linear (exact integral of a linearly interpolated source along the
// ray, Sect. 4.1): c_u = int_0^d (s/d) e^{-s} ds = (1 - (1 + d) e^{-d}) / d,
// c_k = (1 - e^{-d}) - c_u.  Below d = 0.1 the closed forms cancel; their
// Taylor series sum_{n>=2} (-1)^n (n-1) d^(n-1)/n! and
// sum_{n>=2} (-1)^n d^(n-1)/n! are evaluated by Horner's rule instead.
// Trapezoidal (Crank-Nicolson): c_u = c_k = (d/2) / (1 + d/2).
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

// --------------------------------------------------------------------------
// Ray constants: q = (w_m / 2) w~_p, w~_p = w_p phi_p (/ sum if normalized),
// with T1 = sqrt2 (3 mu^2 - 1) / 4, T2 = sqrt2 (3 mu^2 - 3) / 4.
// One block per slab.
// --------------------------------------------------------------------------
__global__ void ray_setup_kernel(const AtmDesc *atm, const double *mu_pos, const double *w_pos,
                                 int M, const double *w_nu, const double *phi, int n_nu,
                                 int normalize, RayConst *rayc, double *qray, double2 *dirc,
                                 double4 *Qs) {
    __shared__ double red[256 / kWave];
    __shared__ double red3[3 * (256 / kWave)];
    const int a = blockIdx.x;
    const double *ph = phi + (long long)a * n_nu;
    double norm = 1.0;
    if (normalize) {
        double s = 0.0;
        for (int p = threadIdx.x; p < n_nu; p += blockDim.x) s += w_nu[p] * ph[p];
        for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
        __syncthreads();
        norm = 0.0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) norm += red[i];
    }
    const AtmDesc at = atm[a];
    double sq = 0.0, sq1 = 0.0, sq12 = 0.0;
    for (int r = threadIdx.x; r < M * n_nu; r += blockDim.x) {
        const int m = r / n_nu, p = r % n_nu;
        const double mu2 = mu_pos[m] * mu_pos[m];
        const double t1 = sqrt(2.0) * (3.0 * mu2 - 1.0) / 4.0;
        const double t2 = sqrt(2.0) * (3.0 * mu2 - 3.0) / 4.0;
        const double q = 0.5 * w_pos[m] * (w_nu[p] * ph[p] / norm);
        RayConst rc;
        rc.q = q;
        rc.qt1 = q * t1;
        rc.qt12 = q * (t1 * t1 + t2 * t2);
        rc.pad = 0.0;
        rayc[at.ray_off + r] = rc;
        qray[at.ray_off + r] = q;
        if (a == 0 && p == 0) dirc[m] = make_double2(t1, t1 * t1 + t2 * t2);
        sq += rc.q;
        sq1 += rc.qt1;
        sq12 += rc.qt12;
    }
    // both directions of every (|mu|, nu) pair carry the weight q
    for (int off = kWave / 2; off > 0; off >>= 1) {
        sq += __shfl_xor(sq, off);
        sq1 += __shfl_xor(sq1, off);
        sq12 += __shfl_xor(sq12, off);
    }
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red3[3 * (threadIdx.x / kWave)] = sq;
        red3[3 * (threadIdx.x / kWave) + 1] = sq1;
        red3[3 * (threadIdx.x / kWave) + 2] = sq12;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
            t0 += red3[3 * w];
            t1 += red3[3 * w + 1];
            t2 += red3[3 * w + 2];
        }
        Qs[a] = make_double4(2.0 * t0, 2.0 * t1, 2.0 * t2, 0.0);
    }
}

// --------------------------------------------------------------------------
// Tile-ordered coefficients: pair (c_u, c_k) of step i of the chunk held by
// lane `lane` in wave-batch b of direction m lives at
//   coef_off + ((m * nwb + b) * Leff + i) * 64 + lane.
// Lane = g * C + c holds chunk c (intervals c*Leff .. c*Leff+Leff-1) of the
// ray (m, p = b*G + g).  Padding (frequencies beyond the last, intervals
// beyond ns - 2) is zero, which makes the step the identity.  The rays'
// quadrature weights are laid out the same way (q_off + (m*nwb + b)*G + g),
// zero for padding rays, so the sweep never masks a loaded value.
// --------------------------------------------------------------------------
__global__ void coef_build_kernel(int W, const AtmDesc *atm, const BlockDesc *blk,
                                  const double *tau, const double *opac, const double *mu_pos,
                                  int fs, const double *qray, double2 *coef64, float2 *coef32,
                                  double *qtile) {
    const BlockDesc bd = blk[blockIdx.x];
    const AtmDesc at = atm[bd.atm];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int c = lane % at.C, g = lane / at.C;
    for (int b = bd.wb_first + wave; b < bd.wb_first + bd.wb_count; b += W) {
        const int p = b * at.G + g;
        if (c == 0)  // quadrature weight of the ray, zero for padding rays
            qtile[at.q_off + ((long long)bd.m * at.nwb + b) * at.G + g] =
                (p < at.n_nu) ? qray[at.ray_off + (long long)bd.m * at.n_nu + p] : 0.0;
        for (int i = 0; i < at.Leff; ++i) {
            const int j = c * at.Leff + i;
            double cu = 0.0, ck = 0.0;
            if (p < at.n_nu && j < at.ns - 1) {
                const double kap = opac[(long long)bd.atm * at.n_nu + p] / mu_pos[bd.m];
                const double d = kap * (tau[at.doff + j + 1] - tau[at.doff + j]);
                step_coef(fs, d, cu, ck);
            }
            const long long e =
                at.coef_off + (((long long)bd.m * at.nwb + b) * at.Leff + i) * kWave + lane;
            coef64[e] = make_double2(cu, ck);
            coef32[e] = make_float2((float)cu, (float)ck);
        }
    }
}

// --------------------------------------------------------------------------
// Jacobi diagonal D = diag(A).  A point source at depth k reaches the
// intensity at k only through the c_k coefficient of the interval entering
// k on each ray (the upwind part of the sweep is zero), so
//   D(k,0) = 1 - xi     sum_rays q        (c_k^down(k) + c_k^up(k)),
//   D(k,2) = 1 - xi W2  sum_rays q (T1^2 + T2^2) (c_k^down(k) + c_k^up(k)),
// the second because s20 enters S_I through T1 and S_Q through T2 and J20
// weights I by T1 and Q by T2.  One thread per depth point.
// --------------------------------------------------------------------------
__global__ void diag_kernel(int npts, const int *pt_atm, const AtmDesc *atm, const double *tau,
                            const double *opac, const double *mu_pos, const RayConst *rayc, int M,
                            int n_nu, int fs, double *diag, double *dinv) {
    const int kk = blockIdx.x * blockDim.x + threadIdx.x;
    if (kk >= npts) return;
    const int a = pt_atm[kk];
    const AtmDesc at = atm[a];
    const int k = kk - at.doff;
    const double dprev = (k >= 1) ? tau[kk] - tau[kk - 1] : 0.0;
    const double dnext = (k <= at.ns - 2) ? tau[kk + 1] - tau[kk] : 0.0;
    double s0 = 0.0, s2 = 0.0;
    for (int m = 0; m < M; ++m) {
        for (int p = 0; p < n_nu; ++p) {
            const double kap = opac[(long long)a * n_nu + p] / mu_pos[m];
            double cu, ck, s = 0.0;
            if (k >= 1) {
                step_coef(fs, kap * dprev, cu, ck);
                s += ck;
            }
            if (k <= at.ns - 2) {
                step_coef(fs, kap * dnext, cu, ck);
                s += ck;
            }
            const RayConst rc = rayc[at.ray_off + m * n_nu + p];
            s0 += rc.q * s;
            s2 += rc.qt12 * s;
        }
    }
    const double d0 = 1.0 - at.xi * s0;
    const double d2 = 1.0 - at.xi * at.W2 * s2;
    diag[2 * (long long)kk] = d0;
    diag[2 * (long long)kk + 1] = d2;
    dinv[2 * (long long)kk] = 1.0 / d0;
    dinv[2 * (long long)kk + 1] = 1.0 / d2;
}

// --------------------------------------------------------------------------
// The fused sweep.  T: arithmetic type of the recurrences and accumulators
// (double, or float inside the mixed-precision inner solve).  L: register
// capacity of a chunk (Leff <= L).  W: waves per block.  Each block writes
// the 2 ns quadrature sums of its rays to its own slot of `partial`; the
// finalize pass (or a Krylov kernel) adds the slots of a slab in block order
// and applies sigma_out = z - xi [J00, W2 J20].
// --------------------------------------------------------------------------
template <typename T>
struct Pair;
template <>
struct Pair<double> {
    using type = double2;
};
template <>
struct Pair<float> {
    using type = float2;
};

// --------------------------------------------------------------------------
// Cross-lane moves for the chunk scans.  DPP (data-parallel primitives) move
// a register between lanes inside the VALU without going through LDS:
// row_shr:d / row_shl:d shift within rows of 16 lanes, row_bcast:15 / :31
// broadcast the last lane of a row (of two rows) to the next row(s),
// wave_shr:1 / wave_shl:1 shift the whole wave by one lane.  Lanes with no
// source receive 0.
// --------------------------------------------------------------------------
namespace {

constexpr int kRowShr = 0x110, kRowShl = 0x100, kWaveShr1 = 0x138, kWaveShl1 = 0x130,
              kRowBcast15 = 0x142, kRowBcast31 = 0x143;

template <int CTRL, int ROWS>
__device__ inline float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ inline double dpp(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(x & 0xffffffffLL), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Compose the chunk maps x -> P x + e of a ray's C chunks (C adjacent lanes,
// C a power of two).  Forward: lane c ends with the map of chunks 0..c;
// backward: lane c ends with the map of chunks c..C-1.  (U, V) are the two
// sources sharing the transmission P.
template <typename T>
__device__ inline void affine_level(T &P, T &U, T &V, T pP, T pU, T pV, bool take) {
    if (take) {
        U = P * pU + U;
        V = P * pV + V;
        P = P * pP;
    }
}

template <int D, typename T>
__device__ inline void fwd_row_level(T &P, T &U, T &V, int lr, int R) {
    if (D < R) {
        const T pP = dpp<kRowShr + D, 0xF>(P), pU = dpp<kRowShr + D, 0xF>(U),
                pV = dpp<kRowShr + D, 0xF>(V);
        affine_level(P, U, V, pP, pU, pV, lr >= D);
    }
}
template <int D, typename T>
__device__ inline void bwd_row_level(T &P, T &U, T &V, int lr, int R) {
    if (D < R) {
        const T nP = dpp<kRowShl + D, 0xF>(P), nU = dpp<kRowShl + D, 0xF>(U),
                nV = dpp<kRowShl + D, 0xF>(V);
        affine_level(P, U, V, nP, nU, nV, lr + D < R);
    }
}

template <typename T>
__device__ inline void scan_forward(T &P, T &U, T &V, int lane, int C) {
    const int R = C < 16 ? C : 16;  // segment length inside a row
    const int lr = lane & (R - 1);
    fwd_row_level<1>(P, U, V, lr, R);
    fwd_row_level<2>(P, U, V, lr, R);
    fwd_row_level<4>(P, U, V, lr, R);
    fwd_row_level<8>(P, U, V, lr, R);
    if (C >= 32) {  // rows 1 and 3 take the last lane of rows 0 and 2
        const T pP = dpp<kRowBcast15, 0xA>(P), pU = dpp<kRowBcast15, 0xA>(U),
                pV = dpp<kRowBcast15, 0xA>(V);
        affine_level(P, U, V, pP, pU, pV, (lane & 16) != 0);
    }
    if (C == 64) {  // rows 2 and 3 take lane 31
        const T pP = dpp<kRowBcast31, 0xC>(P), pU = dpp<kRowBcast31, 0xC>(U),
                pV = dpp<kRowBcast31, 0xC>(V);
        affine_level(P, U, V, pP, pU, pV, (lane & 32) != 0);
    }
}

template <typename T>
__device__ inline void scan_backward(T &P, T &U, T &V, int lane, int C) {
    const int R = C < 16 ? C : 16;
    const int lr = lane & (R - 1);
    bwd_row_level<1>(P, U, V, lr, R);
    bwd_row_level<2>(P, U, V, lr, R);
    bwd_row_level<4>(P, U, V, lr, R);
    bwd_row_level<8>(P, U, V, lr, R);
    if (C >= 32) {  // rows 0 and 2 take the first lane of rows 1 and 3
        const int src = (lane | 15) + 1;
        const T nP = __shfl(P, src & 63), nU = __shfl(U, src & 63), nV = __shfl(V, src & 63);
        affine_level(P, U, V, nP, nU, nV, (lane & 16) == 0);
    }
    if (C == 64) {  // rows 0 and 1 take lane 32
        const T nP = __shfl(P, 32), nU = __shfl(U, 32), nV = __shfl(V, 32);
        affine_level(P, U, V, nP, nU, nV, (lane & 32) == 0);
    }
}

}  // namespace

template <typename T, int L, int W, int PF>
__global__ __launch_bounds__(kWave *W) void sweep_kernel(SweepArgs a) {
    using P2 = typename Pair<T>::type;
    extern __shared__ unsigned char smem_raw[];
    T *sacc = reinterpret_cast<T *>(smem_raw);  // LDS rows of quadrature sums

    const BlockDesc bd = a.blk[blockIdx.x];
    if (a.mask && a.mask[bd.atm] == 0) return;  // uniform over the block
    const AtmDesc at = a.atm[bd.atm];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int C = at.C, Leff = at.Leff, ns = at.ns;
    const int c = lane % C, g = lane / C;
    const int s0 = c * Leff;  // first depth point of this lane's chunk
    const long long vbase = 2LL * at.doff;

    // The sweep carries the deviation D = I - S of the intensity from the
    // local source: with E + c_u = 1 - c_k the step becomes
    //   D_k = E D_u + (1 - c_k) (S_u - S_k),
    // which only accumulates differences of the source, so its rounding stays
    // small against J even where I ~ S (thermalized layers, the FP32 sweep of
    // the mixed-precision solve).  The source part sum q S is added exactly,
    // in FP64, by the finalize pass.
    //
    // Sources s00, s20 at the chunk's points, every load issued before any
    // use (addresses clamped into the slab, values past it zeroed); dl[i] =
    // S(point i) - S(point i + 1); top/bottom: sources at the slab's first and
    // last point, for the boundary deviations.
    T dl0[L], dl2[L];
    T top0 = (T)0, top2 = (T)0, bot0 = (T)0, bot2 = (T)0;
    if (a.sig_in) {
        double2 v[L + 1], vt, vb;
#pragma unroll
        for (int i = 0; i <= L; ++i) {
            const int k = min(s0 + i, ns - 1);
            v[i] = *reinterpret_cast<const double2 *>(a.sig_in + vbase + 2LL * k);
        }
        vt = *reinterpret_cast<const double2 *>(a.sig_in + vbase);
        vb = *reinterpret_cast<const double2 *>(a.sig_in + vbase + 2LL * (ns - 1));
        if (a.scale) {
            double2 sc[L + 1], st, sb;
#pragma unroll
            for (int i = 0; i <= L; ++i) {
                const int k = min(s0 + i, ns - 1);
                sc[i] = *reinterpret_cast<const double2 *>(a.scale + vbase + 2LL * k);
            }
            st = *reinterpret_cast<const double2 *>(a.scale + vbase);
            sb = *reinterpret_cast<const double2 *>(a.scale + vbase + 2LL * (ns - 1));
#pragma unroll
            for (int i = 0; i <= L; ++i) {
                v[i].x *= sc[i].x;
                v[i].y *= sc[i].y;
            }
            vt.x *= st.x;
            vt.y *= st.y;
            vb.x *= sb.x;
            vb.y *= sb.y;
        }
        T s0v[L + 1], s2v[L + 1];
#pragma unroll
        for (int i = 0; i <= L; ++i) {
            const bool in = (i <= Leff) && (s0 + i < ns);
            s0v[i] = in ? (T)v[i].x : (T)0;
            s2v[i] = in ? (T)v[i].y : (T)0;
        }
#pragma unroll
        for (int i = 0; i < L; ++i) {
            dl0[i] = s0v[i] - s0v[i + 1];
            dl2[i] = s2v[i] - s2v[i + 1];
        }
        top0 = (T)vt.x;
        top2 = (T)vt.y;
        bot0 = (T)vb.x;
        bot2 = (T)vb.y;
    } else {
#pragma unroll
        for (int i = 0; i < L; ++i) dl0[i] = dl2[i] = (T)0;
    }

    // AU = sum_rays q (D from s00), AV = sum_rays q (D from s20), by point;
    // every ray of the block has the same direction, so the T factors are
    // applied once at the end
    T AU[L + 1], AV[L + 1];
#pragma unroll
    for (int i = 0; i <= L; ++i) AU[i] = AV[i] = (T)0;

    // deviations entering the slab: I = 0 at the top; I = Ibot (right-hand
    // side) or 0 (operator) at the bottom, whose entry point is the last
    // chunk's end point -- a point of the slab or past it (source zero)
    const T inflow = (a.mode == 1) ? (T)at.Ibot : (T)0;
    const T topD0 = -top0, topD2 = -top2;
    const bool bottom_on_grid = C * Leff == ns - 1;
    const T botD0 = inflow - (bottom_on_grid ? bot0 : (T)0);
    const T botD2 = -(bottom_on_grid ? bot2 : (T)0);
    const P2 *coef = reinterpret_cast<const P2 *>(a.coef) + at.coef_off +
                     (long long)bd.m * at.nwb * Leff * kWave + lane;
    const double *qdir = a.q + at.q_off + (long long)bd.m * at.nwb * at.G + g;
    const int bend = bd.wb_first + bd.wb_count;

    // ray batches are loaded PF batches ahead of use (PF = 0: on use)
    constexpr int NBUF = PF > 0 ? PF : 1;
    P2 cbuf[NBUF][L];
    double qbuf[NBUF];
    auto load_batch = [&](int b, P2 (&cn)[L], double &qn) {
        const P2 *tile = coef + (long long)b * Leff * kWave;
#pragma unroll
        for (int i = 0; i < L; ++i) cn[i] = tile[(long long)min(i, Leff - 1) * kWave];
        qn = qdir[(long long)b * at.G];
    };
    const int b0 = bd.wb_first + wave;
#pragma unroll
    for (int s = 0; s < PF; ++s)
        if (b0 + s * W < bend) load_batch(b0 + s * W, cbuf[s], qbuf[s]);
    for (int b = b0; b < bend; b += W) {
        if (PF == 0) load_batch(b, cbuf[0], qbuf[0]);
        T cu[L], ck[L];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            cu[i] = cbuf[0][i].x;
            ck[i] = cbuf[0][i].y;
        }
        const T q = (T)qbuf[0];
        if (PF > 0) {
            // rotate the ring and load the batch PF steps ahead into its tail
#pragma unroll
            for (int s = 0; s + 1 < NBUF; ++s) {
#pragma unroll
                for (int i = 0; i < L; ++i) cbuf[s][i] = cbuf[s + 1][i];
                qbuf[s] = qbuf[s + 1];
            }
            if (b + PF * W < bend) load_batch(b + PF * W, cbuf[NBUF - 1], qbuf[NBUF - 1]);
        }

        // one pass over the chunk with zero inflow in both directions: the
        // local deviations go into the quadrature at once, and the running
        // transmissions Td[i] = E_0..E_i, Tu[i] = E_i..E_{Leff-1} are kept
        // for the inflow term added after the scan
        T Td[L], Tu[L];
        T dU = (T)0, dV = (T)0, t = (T)1;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            if (i < Leff) {
                const T w = (T)1 - ck[i];
                const T E = w - cu[i];
                dU = fma(E, dU, w * dl0[i]);
                dV = fma(E, dV, w * dl2[i]);
                t *= E;
                Td[i] = t;
                AU[i + 1] = fma(q, dU, AU[i + 1]);
                AV[i + 1] = fma(q, dV, AV[i + 1]);
            }
        }
        T uU = (T)0, uV = (T)0;
        t = (T)1;
#pragma unroll
        for (int i = L - 1; i >= 0; --i) {
            if (i < Leff) {
                const T w = (T)1 - ck[i];
                const T E = w - cu[i];
                uU = fma(E, uU, -w * dl0[i]);
                uV = fma(E, uV, -w * dl2[i]);
                t *= E;
                Tu[i] = t;
                AU[i] = fma(q, uU, AU[i]);
                AV[i] = fma(q, uV, AV[i]);
            }
        }

        // lane scans of the chunk maps I_out = P I_in + e: downward chunks
        // compose left to right, upward ones right to left
        T Pd = t, Pu = t;
        scan_forward(Pd, dU, dV, lane, C);
        scan_backward(Pu, uU, uV, lane, C);
        // inflows at the chunk's entry points: from the chunk above (down),
        // from the chunk below or the bottom boundary (up)
        const T pPd = dpp<kWaveShr1, 0xF>(Pd), nPu = dpp<kWaveShl1, 0xF>(Pu);
        T cdU = dpp<kWaveShr1, 0xF>(dU) + pPd * topD0, cdV = dpp<kWaveShr1, 0xF>(dV) + pPd * topD2;
        T cuU = dpp<kWaveShl1, 0xF>(uU) + nPu * botD0, cuV = dpp<kWaveShl1, 0xF>(uV) + nPu * botD2;
        if (c == 0) {
            cdU = topD0;
            cdV = topD2;
        }
        if (c == C - 1) {
            cuU = botD0;
            cuV = botD2;
        }

        // inflow terms: D_true = D_local + T * D_in at every point of the chunk
        const T qdU = q * cdU, qdV = q * cdV, quU = q * cuU, quV = q * cuV;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            if (i < Leff) {
                AU[i + 1] = fma(Td[i], qdU, AU[i + 1]);
                AV[i + 1] = fma(Td[i], qdV, AV[i + 1]);
                AU[i] = fma(Tu[i], quU, AU[i]);
                AV[i] = fma(Tu[i], quV, AV[i]);
            }
        }
        if (c == 0) {  // the top point's downward deviation is the top inflow's
            AU[0] += qdU;
            AV[0] += qdV;
        }
        if (c == C - 1 && bottom_on_grid) {
            // the bottom point is this chunk's entry point: its upward
            // deviation is the bottom inflow's
#pragma unroll
            for (int i = 0; i <= L; ++i) {
                if (i == Leff) {
                    AU[i] += quU;
                    AV[i] += quV;
                }
            }
        }
    }

    // sum over the G rays of the wave that share chunk c (lanes c, c+C, ...)
    for (int off = C; off < kWave; off <<= 1) {
#pragma unroll
        for (int i = 0; i <= L; ++i) {
            AU[i] += __shfl_xor(AU[i], off);
            AV[i] += __shfl_xor(AV[i], off);
        }
    }
    // the downward value at a chunk's end point belongs to the next chunk's first point
    T bU = (T)0, bV = (T)0;
#pragma unroll
    for (int i = 0; i <= L; ++i) {
        if (i == Leff) {
            bU = AU[i];
            bV = AV[i];
        }
    }
    {
        const T pU = dpp<kWaveShr1, 0xF>(bU), pV = dpp<kWaveShr1, 0xF>(bV);
        if (c > 0) {
            AU[0] += pU;
            AV[0] += pV;
        }
    }
    // J00 = AU + T1 AV, J20 = T1 AU + (T1^2 + T2^2) AV for this direction
    const double2 tf = a.dirc[bd.m];
    const T t1 = (T)tf.x, t12 = (T)tf.y;

    // block totals of the 2 ns quadrature sums
    const int nthr = kWave * W;
    double *mine = a.partial + at.part_off + (long long)(blockIdx.x - at.blk_first) * 2 * ns;
    if (a.rows) {
        // one LDS row per wave, then a fixed-order sum over the rows
        T *row = sacc + (long long)wave * 2 * ns;
        if (g == 0) {
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const int k = s0 + i;
                if (i < Leff && k < ns) {
                    row[2 * k] = AU[i] + t1 * AV[i];
                    row[2 * k + 1] = t1 * AU[i] + t12 * AV[i];
                }
            }
            if (c == C - 1 && s0 + Leff == ns - 1) {
                row[2 * (ns - 1)] = bU + t1 * bV;
                row[2 * (ns - 1) + 1] = t1 * bU + t12 * bV;
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 2 * ns; e += nthr) {
            T s = sacc[e];
            for (int w = 1; w < W; ++w) s += sacc[(long long)w * 2 * ns + e];
            mine[e] = (double)s;
        }
    } else {
        // one shared row, filled wave after wave (fixed order)
        for (int e = threadIdx.x; e < 2 * ns; e += nthr) sacc[e] = (T)0;
        __syncthreads();
        for (int w = 0; w < W; ++w) {
            if (wave == w && g == 0) {
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    const int k = s0 + i;
                    if (i < Leff && k < ns) {
                        sacc[2 * k] += AU[i] + t1 * AV[i];
                        sacc[2 * k + 1] += t1 * AU[i] + t12 * AV[i];
                    }
                }
                if (c == C - 1 && s0 + Leff == ns - 1) {
                    sacc[2 * (ns - 1)] += bU + t1 * bV;
                    sacc[2 * (ns - 1) + 1] += t1 * bU + t12 * bV;
                }
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < 2 * ns; e += nthr) mine[e] = (double)sacc[e];
    }
}

// --------------------------------------------------------------------------
// Finalize: J = sum over the slab's blocks (in block order) of the partial
// quadrature sums of the deviations, plus the source part
//   sum_rays q S = [Q0 s00 + Q1 s20,  Q1 s00 + Q2 s20],
// Q0, Q1, Q2 the sums over all rays of q, q T1, q (T1^2 + T2^2); then
//   mode 0: sigma_out = z - xi [J00, W2 J20], z = scale .* sigma_in;
//   mode 1: sigma_out = xi [J00, W2 J20] + [eps B, 0].
// One thread per depth point.
// --------------------------------------------------------------------------
__global__ void finalize_kernel(SweepArgs a, const int *pt_atm, int npts) {
    const int kk = blockIdx.x * blockDim.x + threadIdx.x;
    if (kk >= npts) return;
    const int atm = pt_atm[kk];
    if (a.mask && a.mask[atm] == 0) return;
    const AtmDesc at = a.atm[atm];
    const int k = kk - at.doff;
    const long long stride = 2LL * at.ns;
    const double *pJ = a.partial + at.part_off + 2 * k;
    double J0 = 0.0, J2 = 0.0;
    for (int j0 = 0; j0 < at.nblk; j0 += 8) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = min(j0 + u, at.nblk - 1);
            v[u] = *reinterpret_cast<const double2 *>(pJ + j * stride);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (j0 + u < at.nblk) {
                J0 += v[u].x;
                J2 += v[u].y;
            }
        }
    }
    const long long e = 2LL * kk;
    double o0, o2;
    if (a.mode == 0) {
        double z0 = a.sig_in[e], z2 = a.sig_in[e + 1];
        if (a.scale) {
            z0 *= a.scale[e];
            z2 *= a.scale[e + 1];
        }
        // source part of the quadrature: sum over all rays of q S
        const double4 Q = a.Qs[atm];
        J0 += z0 * Q.x + z2 * Q.y;
        J2 += z0 * Q.y + z2 * Q.z;
        o0 = z0 - at.xi * J0;
        o2 = z2 - at.xi * at.W2 * J2;
    } else {
        o0 = at.xi * J0 + at.eps * a.B[kk];
        o2 = at.xi * at.W2 * J2;
    }
    a.sig_out[e] = o0;
    a.sig_out[e + 1] = o2;
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
int sweep_waves(int L, bool fp32) {
    // register footprints measured for gfx950: FP64 L=16 and FP32 L=32 need
    // more than 256 VGPRs + AGPRs, i.e. one wave per SIMD
    if (fp32) return L >= 32 ? 4 : 8;
    return L >= 16 ? 4 : 8;
}

template <typename T, int L, int W>
static hipError_t launch_sweep_tw(SweepArgs a, int nblocks, int ns_max, hipStream_t s) {
    const size_t row = 2 * (size_t)ns_max * sizeof(T);
    a.rows = (W * row <= (size_t)kSweepLdsBudget) ? 1 : 0;
    const size_t lds = a.rows ? W * row : row;
    // ray batches in flight ahead of use: a.prefetch (0 = by register budget)
    int pf = a.prefetch;
    // measured on gfx950 (512-slab batch): one batch ahead helps the FP64
    // sweep (its occupancy is register-bound at two waves per SIMD either
    // way); the FP32 sweep does better keeping four waves per SIMD
    if (pf == 0) pf = (sizeof(T) == 8 && L <= 8) ? 2 : 1;
    pf -= 1;
    if (pf >= 2 && sizeof(T) * L <= 64)
        hipLaunchKernelGGL((sweep_kernel<T, L, W, 2>), dim3(nblocks), dim3(kWave * W), lds, s, a);
    else if (pf >= 1)
        hipLaunchKernelGGL((sweep_kernel<T, L, W, 1>), dim3(nblocks), dim3(kWave * W), lds, s, a);
    else
        hipLaunchKernelGGL((sweep_kernel<T, L, W, 0>), dim3(nblocks), dim3(kWave * W), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_finalize(const SweepArgs &a, const int *pt_atm, int npts, hipStream_t s) {
    if (npts <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3((npts + 255) / 256), dim3(256), 0, s, a, pt_atm, npts);
    return hipGetLastError();
}

template <typename T, int L>
static hipError_t launch_sweep_t(const SweepArgs &a, int nblocks, int ns_max, hipStream_t s) {
    if (sweep_waves(L, sizeof(T) == 4) == 8) return launch_sweep_tw<T, L, 8>(a, nblocks, ns_max, s);
    return launch_sweep_tw<T, L, 4>(a, nblocks, ns_max, s);
}

bool sweep_chunk_supported(int L, bool fp32) {
    (void)fp32;
    return L == 4 || L == 8 || L == 16 || L == 32;
}

hipError_t launch_sweep(int L, bool fp32, const SweepArgs &a, int nblocks, int ns_max,
                        hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    if (fp32) {
        switch (L) {
            case 4: return launch_sweep_t<float, 4>(a, nblocks, ns_max, s);
            case 8: return launch_sweep_t<float, 8>(a, nblocks, ns_max, s);
            case 16: return launch_sweep_t<float, 16>(a, nblocks, ns_max, s);
            case 32: return launch_sweep_t<float, 32>(a, nblocks, ns_max, s);
        }
    } else {
        switch (L) {
            case 4: return launch_sweep_t<double, 4>(a, nblocks, ns_max, s);
            case 8: return launch_sweep_t<double, 8>(a, nblocks, ns_max, s);
            case 16: return launch_sweep_t<double, 16>(a, nblocks, ns_max, s);
            case 32: return launch_sweep_t<double, 32>(a, nblocks, ns_max, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_coef_build(int nblocks, int W, const AtmDesc *atm, const BlockDesc *blk,
                             const double *tau, const double *opac, const double *mu_pos, int fs,
                             const double *qray, double2 *coef64, float2 *coef32, double *qtile,
                             hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(coef_build_kernel, dim3(nblocks), dim3(kWave * W), 0, s, W, atm, blk, tau,
                       opac, mu_pos, fs, qray, coef64, coef32, qtile);
    return hipGetLastError();
}

hipError_t launch_ray_setup(int n_atm, const AtmDesc *atm, const double *mu_pos,
                            const double *w_pos, int M, const double *w_nu, const double *phi,
                            int n_nu, int normalize, RayConst *rayc, double *q, double2 *dirc,
                            double4 *Qs, hipStream_t s) {
    hipLaunchKernelGGL(ray_setup_kernel, dim3(n_atm), dim3(256), 0, s, atm, mu_pos, w_pos, M,
                       w_nu, phi, n_nu, normalize, rayc, q, dirc, Qs);
    return hipGetLastError();
}

hipError_t launch_diag(int npts, const int *pt_atm, const AtmDesc *atm, const double *tau,
                       const double *opac, const double *mu_pos, const RayConst *rayc, int M,
                       int n_nu, int fs, double *diag, double *dinv, hipStream_t s) {
    hipLaunchKernelGGL(diag_kernel, dim3((npts + 255) / 256), dim3(256), 0, s, npts, pt_atm, atm,
                       tau, opac, mu_pos, rayc, M, n_nu, fs, diag, dinv);
    return hipGetLastError();
}

}  // namespace rt
