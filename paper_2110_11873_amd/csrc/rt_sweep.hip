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

#include <type_traits>

#include "rt_coef.h"
#include "rt_internal.h"

namespace rt {

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
// Tile-ordered coefficients.  The lane `lane` of wave-batch b of direction m
// holds chunk c = lane_chunk(lane, C) of ray p = b*G + g, g = lane_slot(lane,
// C); the chunk starts at interval s0 = c (Leff - 1) + min(c, nlong) and has
// Leff intervals if c < nlong, else Leff - 1.  The coefficients of its step i
// live at
//   coef_off + (m * nwb + b) * bstride + i * 64 + lane          (i < Leff - 1)
//   coef_off + (m * nwb + b) * bstride + (Leff - 1) * 64 + g * nlong + c
//                                                       (i = Leff - 1, c < nlong)
// so a wavefront reads each step as 64 consecutive entries, and the last step
// only for the chunks that have one.  An entry is the pair (E, w) or w alone
// (the sweep then derives E = 1 - w d).  Padding (frequencies beyond the
// last, intervals beyond ns - 2) is E = w = 1: the step leaves I unchanged,
// and the source beyond the slab is zero.  The rays' quadrature weights and
// (kappa, 1 / kappa) are laid out by slot (q_off + (m*nwb + b)*G + slot),
// zero for padding rays, so the sweep never masks a loaded value.
// --------------------------------------------------------------------------
__global__ void coef_build_kernel(int W, const AtmDesc *atm, const BlockDesc *blk,
                                  const double *tau, const double *opac, const double *mu_pos,
                                  int fs, const double *qray, double2 *coef64, float2 *coef32,
                                  double *w64, float *w32, double *qtile, double2 *ktile) {
    const BlockDesc bd = blk[blockIdx.x];
    const AtmDesc at = atm[bd.atm];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int c = lane_chunk(lane, at.C), g = lane_slot(lane, at.C);
    const int s0 = c * (at.Leff - 1) + min(c, at.nlong);
    const bool longc = c < at.nlong;
    const bool any = coef64 || coef32 || w64 || w32;
    for (int b = bd.wb_first + wave; b < bd.wb_first + bd.wb_count; b += W) {
        const int p = b * at.G + g;
        const double kap =
            (p < at.n_nu) ? opac[(long long)bd.atm * at.n_nu + p] / mu_pos[bd.m] : 0.0;
        if (c == 0) {  // per ray: weight, kappa and 1 / kappa (zero for padding rays)
            const long long r = at.q_off + ((long long)bd.m * at.nwb + b) * at.G + g;
            qtile[r] = (p < at.n_nu) ? qray[at.ray_off + (long long)bd.m * at.n_nu + p] : 0.0;
            if (ktile) ktile[r] = make_double2(kap, (p < at.n_nu) ? 1.0 / kap : 0.0);
        }
        if (!any) continue;
        for (int i = 0; i < at.Leff; ++i) {
            const bool last = i == at.Leff - 1;
            if (last && !longc) continue;
            const int j = s0 + i;
            double E = 1.0, w = 1.0;
            if (p < at.n_nu && j < at.ns - 1) {
                const double d = kap * (tau[at.doff + j + 1] - tau[at.doff + j]);
                step_ew(fs, d, E, w);
            }
            const long long e = at.coef_off + ((long long)bd.m * at.nwb + b) * at.bstride +
                                (last ? (long long)(at.Leff - 1) * kWave + g * at.nlong + c
                                      : (long long)i * kWave + lane);
            if (coef64) coef64[e] = make_double2(E, w);
            if (coef32) coef32[e] = make_float2((float)E, (float)w);
            if (w64) w64[e] = w;
            if (w32) w32[e] = (float)w;
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
            if (fs == RT_FS_DELO_PARABOLIC) {
                s = parabolic_diag(tau + at.doff, at.ns, k, kap, 1) +
                    parabolic_diag(tau + at.doff, at.ns, k, kap, -1);
            } else {
                if (k >= 1) {
                    step_coef(fs, kap * dprev, cu, ck);
                    s += ck;
                }
                if (k <= at.ns - 2) {
                    step_coef(fs, kap * dnext, cu, ck);
                    s += ck;
                }
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

int chunk_len(int ns, int C, int L) {
    const int step = chunk_len_step(L), lo = chunk_len_min(L);
    int le = (ns - 1 + C - 1) / C;
    if (le < lo) le = lo;
    return lo + ((le - lo + step - 1) / step) * step;
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
// One workgroup per (256 depth points, slab): the slab's descriptor is a
// uniform load, so the partial sums are one memory round trip from the start.
// sigma_out at point k of slab atm from its quadrature sums over the
// sweep's blocks (J0, J2): the source part of the quadrature and the
// scattering step (operator), or the right-hand side.
__device__ inline void finalize_point(const SweepArgs &a, int atm, const AtmDesc &at, int k,
                                      double J0, double J2) {
    const int kk = at.doff + k;
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

// Adds the sums of blocks j0, j0 + step, ... (< nblk) at one point, eight
// loads in flight; pJ points at the point's (J0, J2) in block 0's row.
template <typename P>
__device__ inline void add_block_sums(const P *pJ, long long stride, int j0, int step, int nblk,
                                      double &J0, double &J2) {
    using V2 = typename std::conditional<sizeof(P) == 4, float2, double2>::type;
    for (int j = j0; j < nblk; j += 8 * step) {
        V2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int ju = min(j + u * step, nblk - 1);
            v[u] = *reinterpret_cast<const V2 *>(pJ + ju * stride);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (j + u * step < nblk) {
                J0 += (double)v[u].x;
                J2 += (double)v[u].y;
            }
        }
    }
}

__global__ void finalize_kernel(SweepArgs a) {
    const int atm = blockIdx.y;
    if (a.mask && a.mask[atm] == 0) return;
    const AtmDesc at = a.atm[atm];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= at.ns) return;
    const long long stride = 2LL * at.ns;
    double J0 = 0.0, J2 = 0.0;
    if (a.part_f32)
        add_block_sums(reinterpret_cast<const float *>(a.partial) + at.part_off + 2 * k, stride, 0,
                       1, at.nblk, J0, J2);
    else
        add_block_sums(a.partial + at.part_off + 2 * k, stride, 0, 1, at.nblk, J0, J2);
    finalize_point(a, atm, at, k, J0, J2);
}

// The same pass for slabs of many blocks (a single deep slab's plan has
// hundreds): G lanes share a point, lane r adds blocks r, r + G, ..., and a
// fixed tree in LDS combines the G partial sums, so every call adds in the
// same order.  kFinNT / G consecutive points per workgroup.
constexpr int kFinNT = 1024;

__global__ __launch_bounds__(kFinNT) void finalize_split_kernel(SweepArgs a, int G) {
    __shared__ double2 red[kFinNT];
    const int atm = blockIdx.y;
    if (a.mask && a.mask[atm] == 0) return;
    const AtmDesc at = a.atm[atm];
    const int P = kFinNT / G;
    if (blockIdx.x * P >= at.ns) return;  // the whole workgroup
    const int sub = threadIdx.x / P, kl = threadIdx.x % P;
    const int k = blockIdx.x * P + kl;
    const long long stride = 2LL * at.ns;
    double J0 = 0.0, J2 = 0.0;
    if (k < at.ns) {
        if (a.part_f32)
            add_block_sums(reinterpret_cast<const float *>(a.partial) + at.part_off + 2 * k, stride,
                           sub, G, at.nblk, J0, J2);
        else
            add_block_sums(a.partial + at.part_off + 2 * k, stride, sub, G, at.nblk, J0, J2);
    }
    red[threadIdx.x] = make_double2(J0, J2);
    __syncthreads();
    for (int h = G / 2; h >= 1; h >>= 1) {
        if (sub < h) {
            const double2 o = red[threadIdx.x + h * P];
            red[threadIdx.x].x += o.x;
            red[threadIdx.x].y += o.y;
        }
        __syncthreads();
    }
    if (sub == 0 && k < at.ns) finalize_point(a, atm, at, k, red[kl].x, red[kl].y);
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
int sweep_waves(int L, bool fp32) {
    // measured on gfx950 (512-slab batch, single slabs of 200 and 1024
    // points): blocks of 4 waves; 8 waves only pay on single small slabs
    (void)L;
    (void)fp32;
    return 4;
}

void sweep_config(const rt_handle *h, bool fp32, int *W, bool *pf) {
    *W = h->opt.sweep_waves ? h->opt.sweep_waves : sweep_waves(h->L, fp32);
    // options.prefetch: 0 = automatic, 1 = loads on use, 2 or 3 = one batch
    // ahead (compiled for chunks up to 8); automatic: on use, which measured
    // as fast or faster at four waves per SIMD
    *pf = (h->opt.prefetch >= 2) && h->L <= 8;
}

int finalize_lanes(int nblk_max) {
    if (nblk_max <= 32) return 1;  // at most four rounds of loads per point
    int g = 2;
    while (g < 64 && 8 * g < nblk_max) g *= 2;
    return g;
}

hipError_t launch_finalize(const SweepArgs &a, int n_atm, int ns_max, int nblk_max,
                           hipStream_t s) {
    if (n_atm <= 0 || ns_max <= 0) return hipSuccess;
    const int G = finalize_lanes(nblk_max);
    if (G == 1) {
        hipLaunchKernelGGL(finalize_kernel, dim3((ns_max + 255) / 256, n_atm), dim3(256), 0, s, a);
    } else {
        const int P = kFinNT / G;
        hipLaunchKernelGGL(finalize_split_kernel, dim3((ns_max + P - 1) / P, n_atm), dim3(kFinNT), 0,
                           s, a, G);
    }
    return hipGetLastError();
}

bool sweep_chunk_supported(int L, bool fp32) {
    (void)fp32;
    return L == 4 || L == 8 || L == 16 || L == 32;
}

hipError_t launch_sweep(int L, int W, bool pf, bool fp32, int cm, const SweepArgs &a,
                        int nblocks, int ns_max, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    switch (cm) {
        case kCoefPairs:
            return fp32 ? launch_sweep_f32(L, W, pf, a, nblocks, ns_max, s)
                        : launch_sweep_f64(L, W, pf, a, nblocks, ns_max, s);
        case kCoefW:
            return fp32 ? launch_sweep_f32_w(L, W, pf, a, nblocks, ns_max, s)
                        : launch_sweep_f64_w(L, W, pf, a, nblocks, ns_max, s);
        case kCoefRecompute:
            return fp32 ? launch_sweep_f32_rc(L, W, pf, a, nblocks, ns_max, s)
                        : launch_sweep_f64_rc(L, W, pf, a, nblocks, ns_max, s);
    }
    return hipErrorInvalidValue;
}

int coef_mode_of(const rt_handle *h, bool fp32) { return fp32 ? h->cm32 : h->cm64; }

hipError_t launch_coef_build(int nblocks, int W, const AtmDesc *atm, const BlockDesc *blk,
                             const double *tau, const double *opac, const double *mu_pos, int fs,
                             const double *qray, double2 *coef64, float2 *coef32, double *w64,
                             float *w32, double *qtile, double2 *ktile, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(coef_build_kernel, dim3(nblocks), dim3(kWave * W), 0, s, W, atm, blk, tau,
                       opac, mu_pos, fs, qray, coef64, coef32, w64, w32, qtile, ktile);
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
