// rt_prd.hip -- the frequency-redistribution variant on gfx950.
//
// The unknown is sigma^K(k, p) per depth and frequency (K = 0, 2), laid out
// ((doff + k) n_nu + p) 2 + K.  One application:
//  * prd_sweep_kernel: one lane per (|mu|, nu) ray solves both directions in
//    FP64 on the sources S_I = s0(k, p) + T1 s2(k, p), S_Q = T2 s2(k, p) (two
//    linear recurrences, step coefficients recomputed), and writes its
//    |mu|'s share of the monochromatic quadrature
//      J0_p(k) = sum_mu (w_mu / 2) I,  J2_p(k) = sum_mu (w_mu / 2) (T1 I + T2 Q)
//    (eqs. J00/J02 before the frequency integral) to a slot per |mu|;
//  * prd_jsum_kernel adds the |mu| slots in order;
//  * prd_contract_kernel: the redistribution Jt(p, c) = sum_q R(p, q) w_q
//    J(q, c) over the columns c = (k, K) of a slab -- a dense product, on
//    the FP64 matrix cores (v_mfma_f64_16x16x4: one wavefront per 16 x 16
//    tile of Jt, four q per instruction) -- with the scattering step fused
//    into its output: sigma_out = sigma_in - xi W_K Jt / phi_p (operator) or
//    xi W_K Jt / phi_p + eps B (K = 0) (right-hand side).
// With R proportional to phi(p) phi(q) this is the complete-redistribution
// operator at every frequency.  Deterministic: no atomics.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rt_coef.h"
#include "rt_internal.h"

namespace rt {

namespace {

constexpr int kPrdNT = 256;
typedef double v4d __attribute__((ext_vector_type(4)));

struct PrdArgs {
    const AtmDesc *atm;
    const int *pt_atm;
    const double *tau, *opac, *mu_pos, *w_pos, *B, *phi;
    const double2 *dirc;  // per |mu|: (T1, T1^2 + T2^2)
    const double *Rw;     // [n_atm][n_nu][n_nu]: R(p, q) w_q
    const double *sig_in; // NULL: right-hand side (zero source, bottom inflow)
    double *sig_out;
    double *Jm;           // [M][ns_total][n_nu][2]
    double *J;            // [ns_total][n_nu][2]
    int fs, M, n_nu, ns_total;
};

__global__ __launch_bounds__(kPrdNT) void prd_sweep_kernel(PrdArgs a) {
    const int slab = blockIdx.y;
    const AtmDesc at = a.atm[slab];
    const int r = blockIdx.x * kPrdNT + threadIdx.x;
    if (r >= a.M * a.n_nu) return;
    const int mp = r / a.n_nu, p = r % a.n_nu, ns = at.ns;
    const double kap = a.opac[(long long)slab * a.n_nu + p] / a.mu_pos[mp];
    const double wq = 0.5 * a.w_pos[mp];
    const double t1 = a.dirc[mp].x, t12 = a.dirc[mp].y;
    const double *tau = a.tau + at.doff;
    auto src = [&](int k, double &s0, double &s2) {
        if (a.sig_in) {
            const double2 v = *reinterpret_cast<const double2 *>(
                a.sig_in + 2 * ((long long)(at.doff + k) * a.n_nu + p));
            s0 = v.x;
            s2 = v.y;
        } else {
            s0 = s2 = 0.0;
        }
    };
    auto slot = [&](int k) {
        return reinterpret_cast<double2 *>(
            a.Jm + 2 * (((long long)mp * a.ns_total + at.doff + k) * a.n_nu + p));
    };
    for (int dir = 0; dir < 2; ++dir) {
        auto pt = [&](int k) { return dir == 0 ? k : ns - 1 - k; };
        auto put = [&](int k, double X, double Y) {
            double2 c = make_double2(wq * fma(t1, Y, X), wq * fma(t12, Y, t1 * X));
            double2 *d = slot(pt(k));
            if (dir == 1) {
                const double2 o = *d;
                c.x += o.x;
                c.y += o.y;
            }
            *d = c;
        };
        double X = (!a.sig_in && dir == 1) ? at.Ibot : 0.0, Y = 0.0;
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

// J(kk, p) = sum over |mu| (in order) of the slots.  One thread per (kk, p).
__global__ void prd_jsum_kernel(PrdArgs a) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)a.ns_total * a.n_nu) return;
    double2 s = make_double2(0.0, 0.0);
    for (int mp = 0; mp < a.M; ++mp) {
        const double2 v =
            *reinterpret_cast<const double2 *>(a.Jm + 2 * ((long long)mp * a.ns_total * a.n_nu + e));
        s.x += v.x;
        s.y += v.y;
    }
    *reinterpret_cast<double2 *>(a.J + 2 * e) = s;
}

// One wavefront per 16 x 16 tile of Jt (rows p, columns c = 2k + K) of one
// slab.  Lane l feeds A[l % 16][l / 16] = Rw(p0 + l % 16, q0 + l / 16) and
// B[l / 16][l % 16] = J(q0 + l / 16, c0 + l % 16); result register r of lane
// l is Jt(p0 + 4 r + l / 16, c0 + l % 16).
__global__ __launch_bounds__(kPrdNT) void prd_contract_kernel(PrdArgs a) {
    const int slab = blockIdx.z;
    const AtmDesc at = a.atm[slab];
    const int lane = threadIdx.x % kWave;
    const int ctile = blockIdx.x * (kPrdNT / kWave) + threadIdx.x / kWave;
    const int p0 = blockIdx.y * 16, c0 = ctile * 16;
    const int ncol = 2 * at.ns, nnu = a.n_nu;
    if (c0 >= ncol) return;
    const double *Rw = a.Rw + (long long)slab * nnu * nnu;
    const int pa = p0 + lane % 16, kq = lane / 16;      // A operand
    const int cb = c0 + lane % 16;                      // B operand column
    const double *Jcol = a.J + 2LL * (long long)at.doff * nnu + (cb % 2);
    const int kb = cb / 2;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int q0 = 0; q0 < nnu; q0 += 4) {
        const int q = q0 + kq;
        const double av = (pa < nnu && q < nnu) ? Rw[(long long)pa * nnu + q] : 0.0;
        const double bv = (cb < ncol && q < nnu) ? Jcol[2 * ((long long)kb * nnu + q)] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
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
            a.sig_out[e] = a.sig_in[e] - t;
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
    const double g = a.Rw[((long long)slab * a.n_nu + p) * a.n_nu + p] / a.phi[(long long)slab * a.n_nu + p];
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
    a.Rw = h->d_Rw;
    a.sig_in = in;
    a.sig_out = out;
    a.Jm = h->d_prd_Jm;
    a.J = h->d_prd_J;
    a.fs = h->fs;
    a.M = h->M;
    a.n_nu = h->n_nu;
    a.ns_total = h->ns_total;
    return a;
}

}  // namespace

hipError_t apply_prd_operator(const rt_handle *h, const double *in, double *out, hipStream_t s) {
    const PrdArgs a = prd_args(h, in, out);
    const int R = h->M * h->n_nu;
    hipLaunchKernelGGL(prd_sweep_kernel, dim3((R + kPrdNT - 1) / kPrdNT, h->n_atm), dim3(kPrdNT),
                       0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long npts = (long long)h->ns_total * h->n_nu;
    hipLaunchKernelGGL(prd_jsum_kernel, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int ctiles = (2 * h->ns_max + 15) / 16, per = kPrdNT / kWave;
    hipLaunchKernelGGL(prd_contract_kernel,
                       dim3((ctiles + per - 1) / per, (h->n_nu + 15) / 16, h->n_atm), dim3(kPrdNT),
                       0, s, a);
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
    if (!get(&h->d_prd_Jm, 2LL * h->M * npts) || !get(&h->d_prd_J, 2 * npts) ||
        !get(&h->d_prd_diag, 2 * npts) || !get(&h->d_prd_dinv, 2 * npts))
        return fail(RT_ENOMEM, "redistribution workspace allocation failed");
    if (prd_diag(h, h->d_prd_diag, h->d_prd_dinv, s) != hipSuccess)
        return fail(RT_EDEVICE, "redistribution diagonal launch failed");
    h->prd_ready = true;
    return RT_OK;
}

int solve_prd_gmres(rt_handle *h, const double *b, double *x, rt_solve_info *info,
                    hipStream_t st) {
    const int rc = ensure_prd(h, st);
    if (rc != RT_OK) return rc;
    return solve_seg_gmres(
        h, [&](const double *in, double *out) { return apply_prd_operator(h, in, out, st); },
        2LL * h->n_nu, b, [&](double *bo) { return apply_prd_operator(h, nullptr, bo, st); }, x,
        h->d_prd_dinv, info, st);
}

}  // namespace rt
