// rt_raysweep.hip -- the operator for formal solvers with a three-point
// stencil (DELO-parabolic, Sect. 4.1) on gfx950.
//
// The chunked sweep stores one coefficient pair per interval and shares it
// between the two directions of a ray; a parabolic step also depends on the
// next interval in the direction of travel, so its coefficients differ per
// direction.  This path recomputes them instead: one lane owns one
// (|mu|, nu) ray of a slab and walks it downward, then upward, in FP64, with
// two linear recurrences (sources s00 and s20; the T factors are applied when
// the intensities are weighted into the quadrature, as in the chunked
// sweep).  At every depth the wavefront sums q-weighted intensities with an
// xor butterfly and writes them to a slot of its own; a finalize pass adds
// the slots in slot order and applies the scattering step.  No atomics: the
// result is bitwise reproducible.  When a batch has few rays (a single slab),
// each ray is also cut into depth chunks, one wavefront per chunk of the same
// 64 rays in a workgroup: every chunk's affine map from zero entering
// intensity goes to LDS, each chunk folds the maps before it, and a second
// pass from the true entering intensity fills the chunk's depths of the slots.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rt_coef.h"
#include "rt_internal.h"

namespace rt {

namespace {

constexpr int kRayNT = 256;      // one chunk per ray: four ray groups per workgroup
constexpr int kRayMaxChunks = 8;  // chunked: one workgroup of nch wavefronts per ray group

__device__ inline double wave_sum(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

struct RayArgs {
    const AtmDesc *atm;
    const double *tau, *opac, *mu_pos;
    const RayConst *rayc;
    const double *sig_in;   // NULL: zero source
    const double *scale;    // optional elementwise scaling of sig_in
    double *sig_out;
    double *partial;        // [slots][2 ns] per slab at slots * 2 doff
    const int *mask;
    const double *B;
    int fs, M, n_nu, slots, mode;  // mode as in SweepArgs
    int nch;                        // depth chunks per ray (1: the unchunked kernel)
};

__global__ __launch_bounds__(kRayNT) void ray_sweep_kernel(RayArgs a) {
    const int slab = blockIdx.y;
    if (a.mask && a.mask[slab] == 0) return;
    const AtmDesc at = a.atm[slab];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int chunk = blockIdx.x * (kRayNT / kWave) + wave;
    if (2 * chunk >= a.slots) return;
    const int R = a.M * a.n_nu, ns = at.ns;
    const int r = chunk * kWave + lane;
    const bool live = r < R;
    const int m = live ? r / a.n_nu : 0, p = live ? r % a.n_nu : 0;
    const double kap = a.opac[(long long)slab * a.n_nu + p] / a.mu_pos[m];
    const RayConst rc = live ? a.rayc[at.ray_off + r] : RayConst{0.0, 0.0, 0.0, 0.0};
    const double *tau = a.tau + at.doff;
    const long long v0 = 2LL * at.doff;
    auto src = [&](int k, double &s0, double &s2) {
        if (!a.sig_in) {
            s0 = s2 = 0.0;
            return;
        }
        const double2 v = *reinterpret_cast<const double2 *>(a.sig_in + v0 + 2 * k);
        double2 c = make_double2(1.0, 1.0);
        if (a.scale) c = *reinterpret_cast<const double2 *>(a.scale + v0 + 2 * k);
        s0 = v.x * c.x;
        s2 = v.y * c.y;
    };
    double *part = a.partial + (long long)a.slots * 2 * at.doff;
    for (int dir = 0; dir < 2; ++dir) {
        double *slot = part + (long long)(2 * chunk + dir) * 2 * ns;
        // direction order: k-th point of the ray is depth pt(k)
        auto pt = [&](int k) { return dir == 0 ? k : ns - 1 - k; };
        // entry point: zero intensity, except the bottom inflow in mode 1
        double X = 0.0, Y = 0.0;
        if (a.mode == 1 && dir == 1) X = at.Ibot;
        {
            const double c0 = wave_sum(rc.q * X), c2 = wave_sum(rc.qt1 * X);
            if (lane == 0) *reinterpret_cast<double2 *>(slot + 2 * pt(0)) = make_double2(c0, c2);
        }
        double su0, su2, sk0, sk2;
        src(pt(0), su0, su2);
        src(pt(1), sk0, sk2);
        for (int k = 1; k < ns; ++k) {
            const bool has_dn = k + 1 < ns;
            double sd0 = 0.0, sd2 = 0.0;
            if (has_dn) src(pt(k + 1), sd0, sd2);
            const double d = kap * fabs(tau[pt(k)] - tau[pt(k - 1)]);
            const double dd = has_dn ? kap * fabs(tau[pt(k + 1)] - tau[pt(k)]) : 1.0;
            double E, cu, ck, cd;
            ray_step(a.fs, d, dd, has_dn, E, cu, ck, cd);
            X = E * X + cu * su0 + ck * sk0 + cd * sd0;
            Y = E * Y + cu * su2 + ck * sk2 + cd * sd2;
            const double c0 = wave_sum(rc.q * X + rc.qt1 * Y);
            const double c2 = wave_sum(rc.qt1 * X + rc.qt12 * Y);
            if (lane == 0) *reinterpret_cast<double2 *>(slot + 2 * pt(k)) = make_double2(c0, c2);
            su0 = sk0;
            su2 = sk2;
            sk0 = sd0;
            sk2 = sd2;
        }
    }
}

// Chunked variant: workgroup = one ray group (64 rays) of one slab, wave c =
// depth chunk c of those rays.
__global__ __launch_bounds__(kWave * kRayMaxChunks) void ray_sweep_chunked_kernel(RayArgs a) {
    __shared__ double maps[2 * kRayMaxChunks * kWave * 3];  // [dir][chunk][lane][alpha, bx, by]
    const int slab = blockIdx.y;
    if (a.mask && a.mask[slab] == 0) return;
    const AtmDesc at = a.atm[slab];
    const int c = threadIdx.x / kWave, lane = threadIdx.x % kWave, nch = a.nch;
    const int group = blockIdx.x;
    const int R = a.M * a.n_nu, ns = at.ns;
    const int r = group * kWave + lane;
    const bool live = r < R;
    const int m = live ? r / a.n_nu : 0, p = live ? r % a.n_nu : 0;
    const double kap = a.opac[(long long)slab * a.n_nu + p] / a.mu_pos[m];
    const RayConst rc = live ? a.rayc[at.ray_off + r] : RayConst{0.0, 0.0, 0.0, 0.0};
    const double *tau = a.tau + at.doff;
    const long long v0 = 2LL * at.doff;
    const int L = (ns + nch - 1) / nch;
    const int j0 = std::min(c * L, ns), j1 = std::min(j0 + L, ns);
    auto src = [&](int k, double &s0, double &s2) {
        if (!a.sig_in) {
            s0 = s2 = 0.0;
            return;
        }
        const double2 v = *reinterpret_cast<const double2 *>(a.sig_in + v0 + 2 * k);
        double2 cs = make_double2(1.0, 1.0);
        if (a.scale) cs = *reinterpret_cast<const double2 *>(a.scale + v0 + 2 * k);
        s0 = v.x * cs.x;
        s2 = v.y * cs.y;
    };
    double *part = a.partial + (long long)a.slots * 2 * at.doff;
    auto bnd = [&](int dir) { return (a.mode == 1 && dir == 1) ? at.Ibot : 0.0; };
    auto range = [&](int dir, int &r0, int &r1) {
        r0 = dir == 0 ? j0 : ns - j1;
        r1 = dir == 0 ? j1 : ns - j0;
    };
    auto put = [&](int dir, int k, double X, double Y) {
        // the wavefront's q-weighted sum at depth pt(k), into its slot
        const double c0 = wave_sum(rc.q * X + rc.qt1 * Y);
        const double c2 = wave_sum(rc.qt1 * X + rc.qt12 * Y);
        double *slot = part + (long long)(2 * group + dir) * 2 * ns;
        const int j = dir == 0 ? k : ns - 1 - k;
        if (lane == 0) *reinterpret_cast<double2 *>(slot + 2 * j) = make_double2(c0, c2);
    };
    // steps kb..r1-1 of direction dir from (X, Y) at point kb - 1
    auto run = [&](int dir, int kb, int r1, double &X, double &Y, double &alpha, bool emit) {
        auto pt = [&](int k) { return dir == 0 ? k : ns - 1 - k; };
        double su0, su2, sk0, sk2;
        src(pt(kb - 1), su0, su2);
        src(pt(kb), sk0, sk2);
        for (int k = kb; k < r1; ++k) {
            const bool has_dn = k + 1 < ns;
            double sd0 = 0.0, sd2 = 0.0;
            if (has_dn) src(pt(k + 1), sd0, sd2);
            const double d = kap * fabs(tau[pt(k)] - tau[pt(k - 1)]);
            const double dd = has_dn ? kap * fabs(tau[pt(k + 1)] - tau[pt(k)]) : 1.0;
            double E, cu, ck, cd;
            ray_step(a.fs, d, dd, has_dn, E, cu, ck, cd);
            X = E * X + cu * su0 + ck * sk0 + cd * sd0;
            Y = E * Y + cu * su2 + ck * sk2 + cd * sd2;
            alpha *= E;
            if (emit) put(dir, k, X, Y);  // uniform across the wavefront
            su0 = sk0;
            su2 = sk2;
            sk0 = sd0;
            sk2 = sd2;
        }
    };
    // pass 1: the chunk's affine map per direction (the boundary chunk's is
    // absolute: alpha = 0)
    for (int dir = 0; dir < 2; ++dir) {
        int r0, r1;
        range(dir, r0, r1);
        double X = 0.0, Y = 0.0, alpha = 1.0;
        if (r0 < r1) {
            if (r0 == 0) X = bnd(dir);
            if (std::max(r0, 1) < r1) run(dir, std::max(r0, 1), r1, X, Y, alpha, false);
            if (r0 == 0) alpha = 0.0;
        }
        double *mp = maps + ((dir * kRayMaxChunks + c) * kWave + lane) * 3;
        mp[0] = alpha;
        mp[1] = X;
        mp[2] = Y;
    }
    __syncthreads();
    // pass 2: from the entering intensity, the fold of the chunks before
    for (int dir = 0; dir < 2; ++dir) {
        int r0, r1;
        range(dir, r0, r1);
        if (r0 >= r1) continue;
        double X = 0.0, Y = 0.0, alpha = 1.0;
        const int n = dir == 0 ? c : nch - 1 - c;
        for (int i = 0; i < n; ++i) {
            const int cc = dir == 0 ? i : nch - 1 - i;
            const double *mp = maps + ((dir * kRayMaxChunks + cc) * kWave + lane) * 3;
            X = mp[0] * X + mp[1];
            Y = mp[0] * Y + mp[2];
        }
        if (r0 == 0) {
            X = bnd(dir);
            Y = 0.0;
            put(dir, 0, X, Y);
        }
        if (std::max(r0, 1) < r1) run(dir, std::max(r0, 1), r1, X, Y, alpha, true);
    }
}

// sigma_out from the slots: mode 0: z - xi [J00, W2 J20]; mode 1: xi [J00,
// W2 J20] + [eps B, 0].  One thread per depth point.
__global__ void ray_finalize_kernel(RayArgs a, const int *pt_atm, int npts) {
    const int kk = blockIdx.x * blockDim.x + threadIdx.x;
    if (kk >= npts) return;
    const int slab = pt_atm[kk];
    if (a.mask && a.mask[slab] == 0) return;
    const AtmDesc at = a.atm[slab];
    const int k = kk - at.doff;
    const double *part = a.partial + (long long)a.slots * 2 * at.doff + 2 * k;
    double J0 = 0.0, J2 = 0.0;
    for (int sl = 0; sl < a.slots; ++sl) {
        const double2 v = *reinterpret_cast<const double2 *>(part + (long long)sl * 2 * at.ns);
        J0 += v.x;
        J2 += v.y;
    }
    const long long e = 2LL * kk;
    if (a.mode == 1) {
        a.sig_out[e] = at.xi * J0 + at.eps * a.B[kk];
        a.sig_out[e + 1] = at.xi * at.W2 * J2;
    } else {
        double z0 = a.sig_in[e], z2 = a.sig_in[e + 1];
        if (a.scale) {
            z0 *= a.scale[e];
            z2 *= a.scale[e + 1];
        }
        a.sig_out[e] = z0 - at.xi * J0;
        a.sig_out[e + 1] = z2 - at.xi * at.W2 * J2;
    }
}

}  // namespace

int ray_slots(const rt_handle *h) {
    return 2 * ((h->M * h->n_nu + kWave - 1) / kWave);
}

hipError_t apply_ray_operator(rt_handle *h, const double *in, const double *scale, double *out,
                              const int *mask, int mode, hipStream_t s) {
    RayArgs a{};
    a.atm = h->d_atm;
    a.tau = h->d_tau;
    a.opac = h->d_opac;
    a.mu_pos = h->d_mu_pos;
    a.rayc = h->d_rayc;
    a.sig_in = in;
    a.scale = scale;
    a.sig_out = out;
    a.partial = h->d_rpart;
    a.mask = mask;
    a.B = h->d_B;
    a.fs = h->fs;
    a.M = h->M;
    a.n_nu = h->n_nu;
    a.slots = ray_slots(h);
    a.mode = mode;
    const int groups = a.slots / 2, per_wg = kRayNT / kWave;
    // depth chunks per ray: doubled (up to 8) until about 2048 wavefronts
    int nch = 1;
    while (nch < kRayMaxChunks && (long long)groups * h->n_atm * nch < 2048) nch *= 2;
    a.nch = nch;
    if (nch > 1)
        hipLaunchKernelGGL(ray_sweep_chunked_kernel, dim3(groups, h->n_atm), dim3(kWave * nch), 0,
                           s, a);
    else
        hipLaunchKernelGGL(ray_sweep_kernel, dim3((groups + per_wg - 1) / per_wg, h->n_atm),
                           dim3(kRayNT), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ray_finalize_kernel, dim3((h->ns_total + 255) / 256), dim3(256), 0, s, a,
                       (const int *)h->d_pt_atm, h->ns_total);
    return hipGetLastError();
}

}  // namespace rt
