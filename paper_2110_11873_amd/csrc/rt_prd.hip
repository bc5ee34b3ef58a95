// rt_prd.hip -- the frequency-redistribution variant on gfx950.
//
// The unknown is sigma^K(k, p) per depth and frequency (K = 0, 2), laid out
// ((doff + k) n_nu + p) 2 + K.  One application:
//  * prd_sweep_kernel, one workgroup per (frequency p, slab): every (|mu|, p)
//    ray is solved in both directions in FP64 on the sources
//    S_I = s0(k, p) + T1 s2(k, p), S_Q = T2 s2(k, p).  The intensity obeys a
//    linear recurrence along the ray, so each ray is cut into depth chunks
//    (one lane per (chunk, |mu|)): a first pass gives every chunk its affine
//    map (the product of the attenuation factors and the response to zero
//    entering intensity), a fold over the preceding chunks gives each chunk
//    its entering intensity, and a second pass writes the lane's share of the
//    monochromatic quadrature
//      J0_p(k) = sum_mu (w_mu / 2) I,  J2_p(k) = sum_mu (w_mu / 2) (T1 I + T2 Q)
//    (eqs. J00/J02 before the frequency integral) per |mu| to a stage; the
//    stage is then summed over |mu| in order into J, frequency-major
//    (J[p][k][K]).  The stage lives in LDS when it fits, else in a global
//    buffer private to the workgroup.  When a lane's chunk has at most 8
//    points, prd_sweep_cached_kernel does the same with the chunk in
//    registers, each interval's coefficients computed once for both
//    directions, and the entering intensity's share added through the
//    attenuation products kept from the one pass;
//  * prd_contract_kernel: the redistribution Jt(p, c) = sum_q R(p, q) w_q
//    J(q, c) over the columns c = (k, K) of a slab -- a dense product, on
//    the FP64 matrix cores (v_mfma_f64_16x16x4: one workgroup per 16 x 16
//    tile of Jt, four q per instruction, both operands read along
//    contiguous rows: R w is stored transposed, J frequency-major) -- with
//    the scattering step fused into its output:
//    sigma_out = sigma_in - xi W_K Jt / phi_p (operator) or
//    xi W_K Jt / phi_p + eps B (K = 0) (right-hand side);
//  * prd_contract_bf16x3_kernel: the same on the BF16 matrix cores with a
//    hi/lo split of both operands (the inner operator of the mixed solve).
// With R proportional to phi(p) phi(q) this is the complete-redistribution
// operator at every frequency.  Deterministic: no atomics, fixed orders.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "rt_coef.h"
#include "rt_internal.h"

namespace rt {

namespace {

constexpr int kPrdNT = 256;       // contraction
constexpr int kPrdSweepNT = 512;  // sweep: lanes per (|mu|, chunk)
constexpr size_t kPrdLdsMax = 64 * 1024;
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct PrdArgs {
    const AtmDesc *atm;
    const int *pt_atm;
    const double *tau, *opac, *mu_pos, *w_pos, *B, *phi;
    const double2 *dirc;  // per |mu|: (T1, T1^2 + T2^2)
    const double *RwT;    // [n_atm][n_nu (q)][n_nu (p)]: R(p, q) w_q
    const unsigned short *Rbf;  // its bf16 split: [hi, lo][n_atm][n_nu (p)][nqp (q)]
    long long nbf;        // entries per half of Rbf
    int nqp;
    const double *sig_in; // NULL: right-hand side (zero source, bottom inflow)
    const double *scale;  // optional: the operator acts on scale .* sig_in
    double *sig_out;
    double *stage;        // global stage (when the LDS one does not fit)
    double *J;            // [n_nu][ns_total][2]
    int fs, M, n_nu, ns_total, ns_max, nch;
};

// Lanes per (|mu|, chunk): M |mu| values times nch chunks <= kPrdSweepNT.
int prd_chunks(const rt_handle *h) { return std::max(1, std::min(kPrdSweepNT / h->M, h->ns_max)); }

size_t prd_stage_bytes(const rt_handle *h) { return (size_t)2 * h->M * h->ns_max * sizeof(double); }

size_t prd_carry_bytes(const rt_handle *h) {
    return (size_t)2 * prd_chunks(h) * h->M * 3 * sizeof(double);
}

bool prd_global_stage(const rt_handle *h) {
    return std::max(prd_stage_bytes(h), prd_carry_bytes(h)) > kPrdLdsMax;
}

// Stage slot of (depth j, |mu| m), rotated by j so that the in-order sum over
// m, one lane per depth, spreads over the LDS banks.
__device__ inline int stage_slot(int j, int m, int M) { return j * M + (m + j) % M; }

template <bool kGlobalStage>
__global__ __launch_bounds__(kPrdSweepNT) void prd_sweep_kernel(PrdArgs a) {
    extern __shared__ double lds[];
    const int p = blockIdx.x, slab = blockIdx.y;
    const AtmDesc at = a.atm[slab];
    const int M = a.M, nch = a.nch, ns = at.ns, t = threadIdx.x;
    const bool active = t < M * nch;
    const int mp = active ? t % M : 0, c = active ? t / M : 0;
    const int L = (ns + nch - 1) / nch;
    const int j0 = std::min(c * L, ns), j1 = std::min(j0 + L, ns);
    double *stage = kGlobalStage ? a.stage + 2 * ((long long)p * a.ns_total + at.doff) * M : lds;
    double *carry = lds;  // [2][nch][M][3]; in LDS mode it aliases the stage
    const double kap = a.opac[(long long)slab * a.n_nu + p] / a.mu_pos[mp];
    const double wq = 0.5 * a.w_pos[mp];
    const double t1 = a.dirc[mp].x, t12 = a.dirc[mp].y;
    const double *tau = a.tau + at.doff;
    auto src = [&](int j, double &s0, double &s2) {
        if (a.sig_in) {
            const long long e = 2 * ((long long)(at.doff + j) * a.n_nu + p);
            const double2 v = *reinterpret_cast<const double2 *>(a.sig_in + e);
            s0 = v.x;
            s2 = v.y;
            if (a.scale) {
                const double2 sc = *reinterpret_cast<const double2 *>(a.scale + e);
                s0 *= sc.x;
                s2 *= sc.y;
            }
        } else {
            s0 = s2 = 0.0;
        }
    };
    auto bnd = [&](int dir) { return (!a.sig_in && dir == 1) ? at.Ibot : 0.0; };
    // ray points [r0, r1) of this lane's chunk in direction dir (point k of
    // the ray is depth k going down, depth ns - 1 - k going up)
    auto range = [&](int dir, int &r0, int &r1) {
        r0 = dir == 0 ? j0 : ns - j1;
        r1 = dir == 0 ? j1 : ns - j0;
    };
    auto emit = [&](int dir, int k, double X, double Y) {
        const int j = dir == 0 ? k : ns - 1 - k;
        double2 v = make_double2(wq * fma(t1, Y, X), wq * fma(t12, Y, t1 * X));
        double2 *d = reinterpret_cast<double2 *>(stage + 2 * stage_slot(j, mp, M));
        if (dir == 1) {
            const double2 o = *d;
            v.x += o.x;
            v.y += o.y;
        }
        *d = v;
    };
    // steps kb..r1-1 of direction dir from (X, Y) at point kb - 1; alpha
    // collects the product of the attenuation factors.  Sources and depths
    // of point k + 1 + kAhead are loaded at step k (a register queue), so the
    // loads overlap the coefficient arithmetic of the steps before.
    auto run = [&](int dir, int kb, int r1, double &X, double &Y, double &alpha, auto EMIT) {
        constexpr int kAhead = 2;
        auto pt = [&](int k) { return dir == 0 ? k : ns - 1 - k; };
        double qs0[kAhead + 2], qs2[kAhead + 2], qt[kAhead + 2];  // points kb - 1 .. kb + kAhead
#pragma unroll
        for (int i = 0; i < kAhead + 2; ++i) {
            const int k = kb - 1 + i;
            qs0[i] = qs2[i] = qt[i] = 0.0;
            if (k < ns) {
                src(pt(k), qs0[i], qs2[i]);
                qt[i] = tau[pt(k)];
            }
        }
        for (int k = kb; k < r1; ++k) {
            // the queue holds points k - 1 .. k + kAhead
            const bool has_dn = k + 1 < ns;
            const double d = kap * fabs(qt[1] - qt[0]);
            const double dd = has_dn ? kap * fabs(qt[2] - qt[1]) : 1.0;
            double E, cu, ck, cd;
            ray_step(a.fs, d, dd, has_dn, E, cu, ck, cd);
            X = E * X + cu * qs0[0] + ck * qs0[1] + cd * qs0[2];
            Y = E * Y + cu * qs2[0] + ck * qs2[1] + cd * qs2[2];
            alpha *= E;
            if constexpr (decltype(EMIT)::value) emit(dir, k, X, Y);
#pragma unroll
            for (int i = 0; i < kAhead + 1; ++i) {
                qs0[i] = qs0[i + 1];
                qs2[i] = qs2[i + 1];
                qt[i] = qt[i + 1];
            }
            const int kn = k + 1 + kAhead;
            qs0[kAhead + 1] = qs2[kAhead + 1] = qt[kAhead + 1] = 0.0;
            if (kn < ns && kn <= r1) {
                src(pt(kn), qs0[kAhead + 1], qs2[kAhead + 1]);
                qt[kAhead + 1] = tau[pt(kn)];
            }
        }
    };
    // pass 1: each chunk's affine map X_out = alpha X_in + (bx, by)
    double map[2][3];
    if (active) {
        for (int dir = 0; dir < 2; ++dir) {
            int r0, r1;
            range(dir, r0, r1);
            double X = 0.0, Y = 0.0, alpha = 1.0;
            if (r0 < r1) {
                if (r0 == 0) X = bnd(dir);
                if (std::max(r0, 1) < r1) run(dir, std::max(r0, 1), r1, X, Y, alpha, std::false_type{});
                if (r0 == 0) alpha = 0.0;  // the boundary fixes this chunk's exit
            }
            map[dir][0] = alpha;
            map[dir][1] = X;
            map[dir][2] = Y;
        }
    }
    if (active)
        for (int dir = 0; dir < 2; ++dir)
            for (int e = 0; e < 3; ++e) carry[((dir * nch + c) * M + mp) * 3 + e] = map[dir][e];
    __syncthreads();
    // fold the preceding chunks (in ray order) into the entering intensity
    double Xin[2] = {0.0, 0.0}, Yin[2] = {0.0, 0.0};
    if (active) {
        for (int dir = 0; dir < 2; ++dir) {
            const int n = dir == 0 ? c : nch - 1 - c;
            for (int i = 0; i < n; ++i) {
                const int cc = dir == 0 ? i : nch - 1 - i;
                const double *m = carry + ((dir * nch + cc) * M + mp) * 3;
                Xin[dir] = m[0] * Xin[dir] + m[1];
                Yin[dir] = m[0] * Yin[dir] + m[2];
            }
        }
    }
    __syncthreads();  // LDS mode: the maps are read before the stage is written
    // pass 2: the chunk again from its entering intensity, to the stage
    if (active) {
        for (int dir = 0; dir < 2; ++dir) {
            int r0, r1;
            range(dir, r0, r1);
            if (r0 >= r1) continue;
            double X = Xin[dir], Y = Yin[dir], alpha = 1.0;
            if (r0 == 0) {
                X = bnd(dir);
                Y = 0.0;
                emit(dir, 0, X, Y);
            }
            if (std::max(r0, 1) < r1) run(dir, std::max(r0, 1), r1, X, Y, alpha, std::true_type{});
        }
    }
    __syncthreads();
    // J[p][k][K] = sum over |mu| in order
    double *Jo = a.J + 2 * ((long long)p * a.ns_total + at.doff);
    for (int e = t; e < 2 * ns; e += kPrdSweepNT) {
        const int j = e >> 1, K = e & 1;
        double s = 0.0;
        for (int m = 0; m < M; ++m) s += stage[2 * stage_slot(j, m, M) + K];
        Jo[e] = s;
    }
}

// The same sweep for one formal solver FS, each chunk held in registers.  The
// frequency's sources and the slab's depths are staged in LDS; a lane loads
// its chunk's points (and the one before and after it) into registers, and
// for the two-point formal solvers computes each interval's coefficients once
// for both directions (they depend on the interval's optical step only).
// Both directions then run from zero entering intensity (or from the
// boundary, for the chunk that holds the ray's entry point), keeping per
// point the sum of the two local intensities and each direction's running
// attenuation product alpha; the chunk maps go to LDS and are folded as in
// the general sweep, and each point's share, local part plus alpha times the
// entering intensity of either direction, is written to the stage once.  A
// lane holds at most LMAX points; the host launches this kernel only when
// every chunk fits.  LDS (doubles): stage [ns_max][M][2], maps
// [2][nch][M][3], sources [ns_max][2], depths [ns_max].
template <int FS, int NT, int LMAX>
__global__ __launch_bounds__(NT) void prd_sweep_cached_kernel(PrdArgs a) {
    extern __shared__ double lds[];
    const int p = blockIdx.x, slab = blockIdx.y;
    const AtmDesc at = a.atm[slab];
    const int M = a.M, nch = a.nch, ns = at.ns, t = threadIdx.x;
    double *stage = lds;
    double *carry = stage + 2LL * M * a.ns_max;
    double *ssrc = carry + 6LL * nch * M;
    double *stau = ssrc + 2LL * a.ns_max;
    for (int j = t; j < ns; j += NT) {
        double2 v = make_double2(0.0, 0.0);
        if (a.sig_in) {
            const long long e = 2 * ((long long)(at.doff + j) * a.n_nu + p);
            v = *reinterpret_cast<const double2 *>(a.sig_in + e);
            if (a.scale) {
                const double2 sc = *reinterpret_cast<const double2 *>(a.scale + e);
                v.x *= sc.x;
                v.y *= sc.y;
            }
        }
        ssrc[2 * j] = v.x;
        ssrc[2 * j + 1] = v.y;
        stau[j] = a.tau[at.doff + j];
    }
    __syncthreads();

    const bool active = t < M * nch;
    const int mp = active ? t % M : 0, c = active ? t / M : 0;
    const int L = (ns + nch - 1) / nch;
    const int j0 = min(c * L, ns), j1 = min(j0 + L, ns), len = j1 - j0;
    const double kap = a.opac[(long long)slab * a.n_nu + p] / a.mu_pos[mp];
    const double wq = 0.5 * a.w_pos[mp];
    const double t1 = a.dirc[mp].x, t12 = a.dirc[mp].y;

    // point index i <-> depth j0 - 1 + i, i = 0 .. LMAX + 1; the chunk's own
    // points are i = 1 .. len; zero source and depth off the slab
    double s0[LMAX + 2], s2[LMAX + 2], dq[LMAX + 1];
    {
        double tt[LMAX + 2];
#pragma unroll
        for (int i = 0; i < LMAX + 2; ++i) {
            const int j = j0 - 1 + i;
            const bool on = j >= 0 && j < ns && i <= len + 1;
            const int jc = min(max(j, 0), ns - 1);
            s0[i] = on ? ssrc[2 * jc] : 0.0;
            s2[i] = on ? ssrc[2 * jc + 1] : 0.0;
            tt[i] = stau[jc];
        }
        // optical step of interval q, between points q and q + 1 (0 off the slab)
#pragma unroll
        for (int q = 0; q < LMAX + 1; ++q) {
            const int j = j0 - 1 + q;
            dq[q] = (j >= 0 && j + 1 < ns) ? kap * fabs(tt[q + 1] - tt[q]) : 0.0;
        }
    }
    // XL, YL: sum of the two directions' local intensities at point i;
    // ad, au: attenuation from the chunk's entry to point i, downward and upward
    double XL[LMAX + 1], YL[LMAX + 1], ad[LMAX + 1], au[LMAX + 1];
#pragma unroll
    for (int i = 0; i <= LMAX; ++i) XL[i] = YL[i] = ad[i] = au[i] = 0.0;
    const bool top_entry = j0 == 0, bot_entry = j1 == ns;
    double mapd[3] = {1.0, 0.0, 0.0}, mapu[3] = {1.0, 0.0, 0.0};
    if (active && len > 0) {
        // step coefficients of every interval (two-point solvers: shared by
        // both directions)
        double Eq[LMAX + 1], uq[LMAX + 1], kq[LMAX + 1];
        if constexpr (FS != RT_FS_DELO_PARABOLIC) {
#pragma unroll
            for (int q = 0; q < LMAX + 1; ++q) {
                double cd;
                ray_step(FS, dq[q], 1.0, false, Eq[q], uq[q], kq[q], cd);
            }
        }
        // downward: point i from i - 1 through interval i - 1
        {
            double X = 0.0, Y = 0.0, al = 1.0;
#pragma unroll
            for (int i = 1; i <= LMAX; ++i) {
                if (i > len) break;
                const int j = j0 - 1 + i;
                if (j == 0) {  // the ray's entry point: no incoming radiation at the top
                    X = Y = 0.0;
                    ad[i] = 0.0;
                    continue;
                }
                double E, cu, ck, cd = 0.0;
                if constexpr (FS == RT_FS_DELO_PARABOLIC) {
                    const bool has_dn = j + 1 < ns;
                    ray_step(FS, dq[i - 1], has_dn ? dq[i] : 1.0, has_dn, E, cu, ck, cd);
                } else {
                    E = Eq[i - 1];
                    cu = uq[i - 1];
                    ck = kq[i - 1];
                }
                X = E * X + cu * s0[i - 1] + ck * s0[i] + cd * s0[i + 1];
                Y = E * Y + cu * s2[i - 1] + ck * s2[i] + cd * s2[i + 1];
                al *= E;
                XL[i] = X;
                YL[i] = Y;
                ad[i] = al;
            }
            mapd[0] = top_entry ? 0.0 : al;  // the boundary fixes this chunk's exit
            mapd[1] = X;
            mapd[2] = Y;
        }
        // upward: point i from i + 1 through interval i
        {
            double X = 0.0, Y = 0.0, al = 1.0;
#pragma unroll
            for (int i = LMAX; i >= 1; --i) {
                if (i > len) continue;
                const int j = j0 - 1 + i;
                if (j == ns - 1) {  // the ray's entry point: the bottom inflow
                    X = (!a.sig_in) ? at.Ibot : 0.0;
                    Y = 0.0;
                    XL[i] += X;
                    au[i] = 0.0;
                    continue;
                }
                double E, cu, ck, cd = 0.0;
                if constexpr (FS == RT_FS_DELO_PARABOLIC) {
                    const bool has_dn = j >= 1;
                    ray_step(FS, dq[i], has_dn ? dq[i - 1] : 1.0, has_dn, E, cu, ck, cd);
                } else {
                    E = Eq[i];
                    cu = uq[i];
                    ck = kq[i];
                }
                X = E * X + cu * s0[i + 1] + ck * s0[i] + cd * s0[i - 1];
                Y = E * Y + cu * s2[i + 1] + ck * s2[i] + cd * s2[i - 1];
                al *= E;
                XL[i] += X;
                YL[i] += Y;
                au[i] = al;
            }
            mapu[0] = bot_entry ? 0.0 : al;
            mapu[1] = X;
            mapu[2] = Y;
        }
    }
    if (active) {
        double *md = carry + ((0 * nch + c) * M + mp) * 3;
        double *mu = carry + ((1 * nch + c) * M + mp) * 3;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            md[e] = mapd[e];
            mu[e] = mapu[e];
        }
    }
    __syncthreads();
    if (active && len > 0) {
        // entering intensities: the preceding chunks (in ray order) folded
        double Xd = 0.0, Yd = 0.0, Xu = 0.0, Yu = 0.0;
#pragma unroll 4
        for (int i = 0; i < c; ++i) {
            const double *m = carry + ((0 * nch + i) * M + mp) * 3;
            Xd = m[0] * Xd + m[1];
            Yd = m[0] * Yd + m[2];
        }
#pragma unroll 4
        for (int i = nch - 1; i > c; --i) {
            const double *m = carry + ((1 * nch + i) * M + mp) * 3;
            Xu = m[0] * Xu + m[1];
            Yu = m[0] * Yu + m[2];
        }
#pragma unroll
        for (int i = 1; i <= LMAX; ++i) {
            if (i > len) break;
            const double X = XL[i] + ad[i] * Xd + au[i] * Xu;
            const double Y = YL[i] + ad[i] * Yd + au[i] * Yu;
            *reinterpret_cast<double2 *>(stage + 2 * stage_slot(j0 - 1 + i, mp, M)) =
                make_double2(wq * fma(t1, Y, X), wq * fma(t12, Y, t1 * X));
        }
    }
    __syncthreads();
    // J[p][k][K] = sum over |mu| in order
    double *Jo = a.J + 2 * ((long long)p * a.ns_total + at.doff);
    for (int e = t; e < 2 * ns; e += NT) {
        const int j = e >> 1, K = e & 1;
        double s = 0.0;
        for (int m = 0; m < M; ++m) s += stage[2 * stage_slot(j, m, M) + K];
        Jo[e] = s;
    }
}

// One workgroup per 16 x 16 tile of Jt (rows p, columns c = 2k + K) of one
// slab; its four wavefronts take the q-steps q0 = 4 (w + 4 t), and their
// accumulators are added in wavefront order through LDS.  Lane l feeds
// A[l % 16][l / 16] = Rw(p0 + l % 16, q0 + l / 16) and
// B[l / 16][l % 16] = J(q0 + l / 16, c0 + l % 16), each 16 lanes reading 16
// consecutive doubles; result register r of lane l is
// Jt(p0 + 4 r + l / 16, c0 + l % 16).  Eight q-steps of loads are issued
// before their products.
__global__ __launch_bounds__(kPrdNT) void prd_contract_kernel(PrdArgs a) {
    constexpr int U = 8, NW = kPrdNT / kWave;
    __shared__ v4d red[NW - 1][kWave];
    const int slab = blockIdx.z;
    const AtmDesc at = a.atm[slab];
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int p0 = blockIdx.y * 16, c0 = blockIdx.x * 16;
    const int ncol = 2 * at.ns, nnu = a.n_nu;
    if (c0 >= ncol) return;  // the whole workgroup
    const double *RwT = a.RwT + (long long)slab * nnu * nnu;
    const int pa = p0 + lane % 16, kq = lane / 16;      // A operand
    const int cb = c0 + lane % 16;                      // B operand column
    const double *Jb = a.J + 2LL * at.doff;
    const long long js = 2LL * a.ns_total;              // J row stride (one q)
    const bool arow = pa < nnu, bcol = cb < ncol;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int q0 = 4 * wv; q0 < nnu; q0 += 4 * NW * U) {
        double av[U], bv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + 4 * NW * u + kq;
            av[u] = (arow && q < nnu) ? RwT[(long long)q * nnu + pa] : 0.0;
            bv[u] = (bcol && q < nnu) ? Jb[q * js + cb] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    if (wv > 0) red[wv - 1][lane] = acc;
    __syncthreads();
    if (wv > 0) return;
#pragma unroll
    for (int w = 0; w < NW - 1; ++w) acc += red[w][lane];
    const int c = c0 + lane % 16;
    if (c >= ncol) return;
    const int k = c / 2, K = c % 2;
    const double wk = K == 0 ? at.xi : at.xi * at.W2;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int p = p0 + 4 * rr + lane / 16;
        if (p >= nnu) continue;
        const long long e = 2 * ((long long)(at.doff + k) * nnu + p) + K;
        const double t = wk * acc[rr] / a.phi[(long long)slab * nnu + p];
        if (a.sig_in)
            a.sig_out[e] = (a.scale ? a.scale[e] * a.sig_in[e] : a.sig_in[e]) - t;
        else
            a.sig_out[e] = t + (K == 0 ? at.eps * a.B[at.doff + k] : 0.0);
    }
}

// The same contraction on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16):
// R w (split on the host) and J (split here from FP64 through FP32) are each
// hi + lo in bf16, about 16 significant bits, and J~ = Rh Jh + (Rh Jl + Rl Jh)
// with the two groups in separate FP32 accumulators, added in FP64 (the
// dropped Rl Jl is below 2^-16 of the product).  One workgroup per 16 x 16
// tile, its four wavefronts on interleaved groups of 32 q, added in
// wavefront order.  Lane l feeds A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16], i = 0..7 (q contiguous per lane: the order of
// q inside an instruction only has to agree between A and B); result
// register r of lane l is D[4 (l / 16) + r][l % 16].
__global__ __launch_bounds__(kPrdNT) void prd_contract_bf16x3_kernel(PrdArgs a) {
    constexpr int NW = kPrdNT / kWave;
    __shared__ f32x4 red[2][NW - 1][kWave];
    const int slab = blockIdx.z;
    const AtmDesc at = a.atm[slab];
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int p0 = blockIdx.y * 16, c0 = blockIdx.x * 16;
    const int ncol = 2 * at.ns, nnu = a.n_nu;
    if (c0 >= ncol) return;  // the whole workgroup
    const unsigned short *Rh = a.Rbf + (long long)slab * nnu * a.nqp;
    const unsigned short *Rl = Rh + a.nbf;
    const int pa = p0 + lane % 16, g = lane / 16;
    const int cb = c0 + lane % 16;
    const double *Jb = a.J + 2LL * at.doff;
    const long long js = 2LL * a.ns_total;
    const bool arow = pa < nnu, bcol = cb < ncol;
    f32x4 big = {0.f, 0.f, 0.f, 0.f}, small = {0.f, 0.f, 0.f, 0.f};
    for (int q0 = 32 * wv; q0 < nnu; q0 += 32 * NW) {
        const int qa = q0 + 8 * g;  // rows are padded to a multiple of 32: qa + 8 <= nqp
        u16x8 uh = {0, 0, 0, 0, 0, 0, 0, 0}, ul = uh;
        if (arow) {
            uh = *reinterpret_cast<const u16x8 *>(Rh + (long long)pa * a.nqp + qa);
            ul = *reinterpret_cast<const u16x8 *>(Rl + (long long)pa * a.nqp + qa);
        }
        double jv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            jv[i] = (bcol && qa + i < nnu) ? Jb[(qa + i) * js + cb] : 0.0;
        bf16x8 bh, bl;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float f = (float)jv[i];
            const __bf16 hi = (__bf16)f;
            bh[i] = hi;
            bl[i] = (__bf16)(f - (float)hi);
        }
        const bf16x8 ah = __builtin_bit_cast(bf16x8, uh), al = __builtin_bit_cast(bf16x8, ul);
        big = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, big, 0, 0, 0);
        small = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, small, 0, 0, 0);
        small = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, small, 0, 0, 0);
    }
    if (wv > 0) {
        red[0][wv - 1][lane] = big;
        red[1][wv - 1][lane] = small;
    }
    __syncthreads();
    if (wv > 0) return;
    double acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = (double)big[r] + (double)small[r];
#pragma unroll
    for (int w = 0; w < NW - 1; ++w)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            acc[r] += (double)red[0][w][lane][r] + (double)red[1][w][lane][r];
    const int c = c0 + lane % 16;
    if (c >= ncol) return;
    const int k = c / 2, K = c % 2;
    const double wk = K == 0 ? at.xi : at.xi * at.W2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = p0 + 4 * g + r;
        if (p >= nnu) continue;
        const long long e = 2 * ((long long)(at.doff + k) * nnu + p) + K;
        const double t = wk * acc[r] / a.phi[(long long)slab * nnu + p];
        if (a.sig_in)
            a.sig_out[e] = (a.scale ? a.scale[e] * a.sig_in[e] : a.sig_in[e]) - t;
        else
            a.sig_out[e] = t + (K == 0 ? at.eps * a.B[at.doff + k] : 0.0);
    }
}

// Jacobi diagonal: sigma^K(k, p) reaches itself through the rays' Lambda(k, k),
// the monochromatic quadrature and R(p, p) w_p.  One thread per (kk, p).
__global__ void prd_diag_kernel(PrdArgs a, double *diag, double *dinv) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)a.ns_total * a.n_nu) return;
    const int kk = (int)(e / a.n_nu), p = (int)(e % a.n_nu);
    const int slab = a.pt_atm[kk];
    const AtmDesc at = a.atm[slab];
    const int k = kk - at.doff, ns = at.ns;
    const double *tau = a.tau + at.doff;
    double s0 = 0.0, s2 = 0.0;
    for (int mp = 0; mp < a.M; ++mp) {
        const double kap = a.opac[(long long)slab * a.n_nu + p] / a.mu_pos[mp];
        double lam = 0.0;
        if (a.fs == RT_FS_DELO_PARABOLIC) {
            lam = parabolic_diag(tau, ns, k, kap, 1) + parabolic_diag(tau, ns, k, kap, -1);
        } else {
            double cu, ck;
            if (k >= 1) {
                step_coef(a.fs, kap * (tau[k] - tau[k - 1]), cu, ck);
                lam += ck;
            }
            if (k <= ns - 2) {
                step_coef(a.fs, kap * (tau[k + 1] - tau[k]), cu, ck);
                lam += ck;
            }
        }
        const double wq = 0.5 * a.w_pos[mp];
        s0 += wq * lam;
        s2 += wq * a.dirc[mp].y * lam;
    }
    const double g = a.RwT[((long long)slab * a.n_nu + p) * a.n_nu + p] / a.phi[(long long)slab * a.n_nu + p];
    const double d0 = 1.0 - at.xi * g * s0, d2 = 1.0 - at.xi * at.W2 * g * s2;
    diag[2 * e] = d0;
    diag[2 * e + 1] = d2;
    dinv[2 * e] = 1.0 / d0;
    dinv[2 * e + 1] = 1.0 / d2;
}

PrdArgs prd_args(const rt_handle *h, const double *in, double *out) {
    PrdArgs a{};
    a.atm = h->d_atm;
    a.pt_atm = h->d_pt_atm;
    a.tau = h->d_tau;
    a.opac = h->d_opac;
    a.mu_pos = h->d_mu_pos;
    a.w_pos = h->d_w_pos;
    a.B = h->d_B;
    a.phi = h->d_phi;
    a.dirc = h->d_dirc;
    a.RwT = h->d_Rw;
    a.Rbf = h->d_Rw_bf;
    a.nqp = h->prd_nqp;
    a.nbf = (long long)h->n_atm * h->n_nu * h->prd_nqp;
    a.sig_in = in;
    a.sig_out = out;
    a.stage = h->d_prd_Jm;
    a.J = h->d_prd_J;
    a.fs = h->fs;
    a.M = h->M;
    a.n_nu = h->n_nu;
    a.ns_total = h->ns_total;
    a.ns_max = h->ns_max;
    a.nch = h->prd_cached_nt ? h->prd_cached_nch : prd_chunks(h);
    return a;
}

// The cached-coefficient sweep (kPrdSweepNT threads, as the general one):
// its LDS bytes, and its kernel for the handle's formal solver.  A
// 1024-thread variant (chunks half as long, twice as many) measured slower
// on the 256-depth, 32 x 256 grid: 27.3 against 25.3 us per application.
constexpr int kPrdCachedLen = 8;  // most points per chunk and direction
size_t prd_cached_lds(const rt_handle *h, int nch) {
    return ((size_t)2 * h->M * h->ns_max + (size_t)6 * nch * h->M + (size_t)3 * h->ns_max) *
           sizeof(double);
}
const void *prd_cached_kernel(int fs) {
    constexpr int NT = kPrdSweepNT, LM = kPrdCachedLen;
    switch (fs) {
        case RT_FS_TRAPEZOIDAL: return (const void *)prd_sweep_cached_kernel<RT_FS_TRAPEZOIDAL, NT, LM>;
        case RT_FS_IMPLICIT_EULER:
            return (const void *)prd_sweep_cached_kernel<RT_FS_IMPLICIT_EULER, NT, LM>;
        case RT_FS_DELO_PARABOLIC:
            return (const void *)prd_sweep_cached_kernel<RT_FS_DELO_PARABOLIC, NT, LM>;
        default: return (const void *)prd_sweep_cached_kernel<RT_FS_DELO_LINEAR, NT, LM>;
    }
}

// Take the cached sweep when every chunk fits its registers and its LDS fits
// the device (raising the kernel's LDS limit where needed); else the general
// sweep.
void choose_prd_sweep(rt_handle *h) {
    h->prd_cached_nt = h->prd_cached_nch = 0;
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) !=
        hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    const int nch = prd_chunks(h);
    const size_t lds = prd_cached_lds(h, nch);
    if ((h->ns_max + nch - 1) / nch > kPrdCachedLen || lds > (size_t)lds_max) return;
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute(prd_cached_kernel(h->fs), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    h->prd_cached_nt = kPrdSweepNT;
    h->prd_cached_nch = nch;
}

}  // namespace

hipError_t apply_prd_operator(const rt_handle *h, const double *in, double *out, hipStream_t s,
                              bool bf16x3, const double *scale) {
    PrdArgs a = prd_args(h, in, out);
    a.scale = in ? scale : nullptr;
    const dim3 grid(h->n_nu, h->n_atm);
    if (h->prd_cached_nt) {
        PrdArgs arg = a;
        void *args[] = {&arg};
        const hipError_t e = hipLaunchKernel(prd_cached_kernel(h->fs), grid,
                                             dim3(h->prd_cached_nt), args,
                                             prd_cached_lds(h, h->prd_cached_nch), s);
        if (e != hipSuccess) return e;
    } else if (prd_global_stage(h))
        hipLaunchKernelGGL(prd_sweep_kernel<true>, grid, dim3(kPrdSweepNT), prd_carry_bytes(h), s,
                           a);
    else
        hipLaunchKernelGGL(prd_sweep_kernel<false>, grid, dim3(kPrdSweepNT),
                           std::max(prd_stage_bytes(h), prd_carry_bytes(h)), s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 tiles((2 * h->ns_max + 15) / 16, (h->n_nu + 15) / 16, h->n_atm);
    if (bf16x3)
        hipLaunchKernelGGL(prd_contract_bf16x3_kernel, tiles, dim3(kPrdNT), 0, s, a);
    else
        hipLaunchKernelGGL(prd_contract_kernel, tiles, dim3(kPrdNT), 0, s, a);
    return hipGetLastError();
}

hipError_t prd_diag(const rt_handle *h, double *diag, double *dinv, hipStream_t s) {
    const PrdArgs a = prd_args(h, nullptr, nullptr);
    const long long npts = (long long)h->ns_total * h->n_nu;
    hipLaunchKernelGGL(prd_diag_kernel, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s, a,
                       diag, dinv);
    return hipGetLastError();
}

int ensure_prd(rt_handle *h, hipStream_t s) {
    if (!h->d_Rw) return fail(RT_EINVAL, "no redistribution matrix: call rt_set_redistribution first");
    if (h->prd_ready) return RT_OK;
    const long long npts = (long long)h->ns_total * h->n_nu;
    auto get = [&](double **p, long long n) {
        if (*p) return true;
        if (hipMalloc((void **)p, sizeof(double) * std::max<long long>(n, 1)) != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
            return false;
        }
        return true;
    };
    if (h->M > kPrdSweepNT) return fail(RT_EINVAL, "redistribution: at most 1024 angle nodes");
    if ((prd_global_stage(h) && !get(&h->d_prd_Jm, 2LL * h->M * npts)) || !get(&h->d_prd_J, 2 * npts) ||
        !get(&h->d_prd_diag, 2 * npts) || !get(&h->d_prd_dinv, 2 * npts))
        return fail(RT_ENOMEM, "redistribution workspace allocation failed");
    choose_prd_sweep(h);
    if (prd_diag(h, h->d_prd_diag, h->d_prd_dinv, s) != hipSuccess)
        return fail(RT_EDEVICE, "redistribution diagonal launch failed");
    h->prd_ready = true;
    return RT_OK;
}

int solve_prd_gmres(rt_handle *h, const double *b, double *x, rt_solve_info *info,
                    hipStream_t st) {
    const int rc = ensure_prd(h, st);
    if (rc != RT_OK) return rc;
    auto op = [&](const double *in, const double *scale, double *out) {
        return apply_prd_operator(h, in, out, st, false, scale);
    };
    auto rhs = [&](double *bo) { return apply_prd_operator(h, nullptr, bo, st); };
    if (h->opt.precision == RT_PREC_MIXED)
        return solve_seg_refined(
            h, op,
            [&](const double *in, const double *scale, double *out) {
                return apply_prd_operator(h, in, out, st, true, scale);
            },
            2LL * h->n_nu, b, rhs, x, h->d_prd_dinv, info, st);
    return solve_seg_gmres(h, op, 2LL * h->n_nu, b, rhs, x, h->d_prd_dinv, info, st);
}

}  // namespace rt
