// rt_field.hip -- the Stokes field as unknown (eq. crd_linear_system2):
// (Id - Lambda T J) I = Lambda T c + t, and sigma = J I + c.
//
// Two passes per application:
//  * field_quad_kernel: one wavefront per depth point sums the field over all
//    rays into J I = xi [J00, W2 J20] (eqs. J00/J02, S00/S02); a depth's rays
//    are contiguous in the field, so the reads are coalesced;
//  * field_sweep_kernel: one lane per (|mu|, nu) ray runs the formal solver
//    downward and upward on the sources T (J I) (two linear recurrences, on
//    s00 and s20, combined with the T factors per point), and writes the I
//    and Q field -- subtracted from the input for the operator.  The step
//    coefficients are recomputed from tau (every formal solver, including
//    the three-point DELO-parabolic step).
// Both are FP64 and deterministic (fixed-order butterflies, no atomics).
#include <hip/hip_runtime.h>

#include "rt_coef.h"
#include "rt_internal.h"

namespace rt {

namespace {

constexpr int kFieldNT = 256;

struct FieldArgs {
    const AtmDesc *atm;
    const int *pt_atm;
    const double *tau, *opac, *mu_pos, *B;
    const RayConst *rayc;
    const double2 *dirc;   // per |mu|: (T1, T1^2 + T2^2)
    const int *mu_idx;     // per |mu|: the caller's index of -mu and +mu
    const double *fin;     // field in
    double *fout;          // field out
    const double *sig;     // sweep sources (NULL: c = [eps B, 0])
    double *sig_out;       // quadrature output
    int fs, M, n_mu, n_nu, ns_total;
    int with_c;            // quadrature: add c;  sweep: rhs mode (sources c, bottom inflow)
    int sub;               // sweep: write fin - field
};

__device__ inline double t2_of(double mu) { return sqrt(2.0) * (3.0 * mu * mu - 3.0) / 4.0; }

__global__ __launch_bounds__(kFieldNT) void field_quad_kernel(FieldArgs a) {
    const int kk = blockIdx.x * (kFieldNT / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    if (kk >= a.ns_total) return;
    const AtmDesc at = a.atm[a.pt_atm[kk]];
    const int k = kk - at.doff, ns = at.ns;
    const long long base = 2LL * a.n_mu * a.n_nu * at.doff;
    const double *FI = a.fin + base + (long long)k * a.n_mu * a.n_nu;
    const double *FQ = a.fin + base + (long long)(ns + k) * a.n_mu * a.n_nu;
    double J0 = 0.0, J2 = 0.0;
    const int nr = a.n_mu * a.n_nu;
    for (int r = lane; r < nr; r += kWave) {
        // r runs over (|mu| index, direction, frequency)
        const int mp = r / (2 * a.n_nu), dir = (r / a.n_nu) % 2, p = r % a.n_nu;
        const long long e = (long long)a.mu_idx[2 * mp + dir] * a.n_nu + p;
        const RayConst rc = a.rayc[at.ray_off + mp * a.n_nu + p];
        const double t2 = t2_of(a.mu_pos[mp]);
        const double I = FI[e], Q = FQ[e];
        J0 = fma(rc.q, I, J0);
        J2 = fma(rc.q, fma(a.dirc[mp].x, I, t2 * Q), J2);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        J0 += __shfl_xor(J0, off);
        J2 += __shfl_xor(J2, off);
    }
    if (lane == 0) {
        a.sig_out[2LL * kk] = at.xi * J0 + (a.with_c ? at.eps * a.B[kk] : 0.0);
        a.sig_out[2LL * kk + 1] = at.xi * at.W2 * J2;
    }
}

__global__ __launch_bounds__(kFieldNT) void field_sweep_kernel(FieldArgs a) {
    const int slab = blockIdx.y;
    const AtmDesc at = a.atm[slab];
    const int r = blockIdx.x * kFieldNT + threadIdx.x;
    if (r >= a.M * a.n_nu) return;
    const int mp = r / a.n_nu, p = r % a.n_nu;
    const int ns = at.ns;
    const double kap = a.opac[(long long)slab * a.n_nu + p] / a.mu_pos[mp];
    const double t1 = a.dirc[mp].x, t2 = t2_of(a.mu_pos[mp]);
    const double *tau = a.tau + at.doff;
    const long long base = 2LL * a.n_mu * a.n_nu * at.doff;
    const long long plane = (long long)ns * a.n_mu * a.n_nu;  // Q follows I
    auto src = [&](int k, double &s0, double &s2) {
        if (a.sig) {
            const double2 v = *reinterpret_cast<const double2 *>(a.sig + 2LL * (at.doff + k));
            s0 = v.x;
            s2 = v.y;
        } else {
            s0 = at.eps * a.B[at.doff + k];
            s2 = 0.0;
        }
    };
    for (int dir = 0; dir < 2; ++dir) {
        const long long col = (long long)a.mu_idx[2 * mp + dir] * a.n_nu + p;
        auto pt = [&](int k) { return dir == 0 ? k : ns - 1 - k; };
        auto put = [&](int k, double X, double Y) {
            const long long e = base + (long long)pt(k) * a.n_mu * a.n_nu + col;
            const double I = fma(t1, Y, X), Q = t2 * Y;
            a.fout[e] = a.sub ? a.fin[e] - I : I;
            a.fout[e + plane] = a.sub ? a.fin[e + plane] - Q : Q;
        };
        double X = (!a.sig && a.with_c && dir == 1) ? at.Ibot : 0.0, Y = 0.0;
        put(0, X, Y);
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
            put(k, X, Y);
            su0 = sk0;
            su2 = sk2;
            sk0 = sd0;
            sk2 = sd2;
        }
    }
}

FieldArgs field_args(const rt_handle *h) {
    FieldArgs a{};
    a.atm = h->d_atm;
    a.pt_atm = h->d_pt_atm;
    a.tau = h->d_tau;
    a.opac = h->d_opac;
    a.mu_pos = h->d_mu_pos;
    a.B = h->d_B;
    a.rayc = h->d_rayc;
    a.dirc = h->d_dirc;
    a.mu_idx = h->d_mu_idx;
    a.fs = h->fs;
    a.M = h->M;
    a.n_mu = h->n_mu;
    a.n_nu = h->n_nu;
    a.ns_total = h->ns_total;
    return a;
}

hipError_t launch_quad(const FieldArgs &a, hipStream_t s) {
    const int per = kFieldNT / kWave;
    hipLaunchKernelGGL(field_quad_kernel, dim3((a.ns_total + per - 1) / per), dim3(kFieldNT), 0, s,
                       a);
    return hipGetLastError();
}

hipError_t launch_field_sweep(const rt_handle *h, const FieldArgs &a, hipStream_t s) {
    const int R = h->M * h->n_nu;
    hipLaunchKernelGGL(field_sweep_kernel, dim3((R + kFieldNT - 1) / kFieldNT, h->n_atm),
                       dim3(kFieldNT), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t field_sigma(rt_handle *h, const double *I, double *sigma, int with_c, hipStream_t s) {
    FieldArgs a = field_args(h);
    a.fin = I;
    a.sig_out = sigma;
    a.with_c = with_c;
    return launch_quad(a, s);
}

hipError_t apply_field_operator(rt_handle *h, const double *in, double *out, hipStream_t s) {
    hipError_t e = field_sigma(h, in, h->d_fsig, 0, s);
    if (e != hipSuccess) return e;
    FieldArgs a = field_args(h);
    a.fin = in;
    a.fout = out;
    a.sig = h->d_fsig;
    a.sub = 1;
    return launch_field_sweep(h, a, s);
}

hipError_t field_rhs(rt_handle *h, double *b, hipStream_t s) {
    FieldArgs a = field_args(h);
    a.fout = b;
    a.sig = nullptr;  // sources c = [eps B, 0]
    a.with_c = 1;     // and the bottom inflow
    return launch_field_sweep(h, a, s);
}

}  // namespace rt
