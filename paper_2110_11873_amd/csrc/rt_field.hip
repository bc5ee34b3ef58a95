// rt_field.hip -- the Stokes field as unknown (eq. crd_linear_system2):
// (Id - Lambda T J) I = Lambda T c + t, and sigma = J I + c.
//
// Two passes per application:
//  * field_quad_kernel: one workgroup per depth point sums the field over all
//    rays into J I = xi [J00, W2 J20] (eqs. J00/J02, S00/S02); a depth's rays
//    are contiguous in the field, so the reads are coalesced;
//  * field_sweep_kernel: the formal solver along every (|mu|, nu) ray,
//    downward and upward, on the sources T (J I) (two linear recurrences, on
//    s00 and s20, combined with the T factors per point), writing the I and Q
//    field -- subtracted from the input for the operator.  The step
//    coefficients are recomputed from tau (every formal solver, including
//    the three-point DELO-parabolic step).  When there are few rays (a
//    single slab) each ray is cut into depth chunks, one lane each: the
//    chunk's affine map from zero entering intensity, a fold over the chunks
//    before it in LDS, and a second pass from the true entering intensity.
// Both are FP64 and deterministic (fixed-order butterflies, no atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "rt_coef.h"
#include "rt_internal.h"

namespace rt {

namespace {

constexpr int kFieldNT = 256;
constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, one L2 each

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
    int nch;               // sweep: depth chunks per ray (a power of two <= kFieldNT)
    int with_c;            // quadrature: add c;  sweep: rhs mode (sources c, bottom inflow)
    int sub;               // sweep: write fin - field
};

__device__ inline double t2_of(double mu) { return sqrt(2.0) * (3.0 * mu * mu - 3.0) / 4.0; }

// One workgroup per depth point: its lanes take the rays in turn, each
// wavefront reduces by butterfly, and the wavefronts' sums are added in
// wavefront order.
__global__ __launch_bounds__(kFieldNT) void field_quad_kernel(FieldArgs a) {
    __shared__ double2 part[kFieldNT / kWave];
    const int kk = blockIdx.x;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const AtmDesc at = a.atm[a.pt_atm[kk]];
    const int k = kk - at.doff, ns = at.ns;
    const long long base = 2LL * a.n_mu * a.n_nu * at.doff;
    const double *FI = a.fin + base + (long long)k * a.n_mu * a.n_nu;
    const double *FQ = a.fin + base + (long long)(ns + k) * a.n_mu * a.n_nu;
    double J0 = 0.0, J2 = 0.0;
    const int nr = a.n_mu * a.n_nu;
    for (int r = threadIdx.x; r < nr; r += kFieldNT) {
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
    if (lane == 0) part[wv] = make_double2(J0, J2);
    __syncthreads();
    if (threadIdx.x == 0) {
        J0 = J2 = 0.0;
        for (int w = 0; w < kFieldNT / kWave; ++w) {
            J0 += part[w].x;
            J2 += part[w].y;
        }
        a.sig_out[2LL * kk] = at.xi * J0 + (a.with_c ? at.eps * a.B[kk] : 0.0);
        a.sig_out[2LL * kk + 1] = at.xi * at.W2 * J2;
    }
}

// Lane t of a workgroup: ray g = t % G of the workgroup's G rays
// (consecutive frequencies, for coalesced field writes) and depth chunk
// c = t / G, with G * nch = kFieldNT.
__global__ __launch_bounds__(kFieldNT) void field_sweep_kernel(FieldArgs a) {
    __shared__ double carry[2 * kFieldNT * 3];  // [dir][chunk][ray][alpha, bx, by]
    // Workgroups are dealt to the eight XCDs in turn; give each XCD a run of
    // consecutive ray groups, so the groups that share the field's cache
    // lines (G rays of one depth row each) meet in one L2
    const int nwg = gridDim.x * gridDim.y, lin = blockIdx.y * gridDim.x + blockIdx.x;
    const int xcd = lin % kXcds, q = nwg / kXcds, rem = nwg % kXcds;
    const int wg = xcd * q + std::min(xcd, rem) + lin / kXcds;
    const int slab = wg / gridDim.x, rg = wg % gridDim.x;
    const AtmDesc at = a.atm[slab];
    const int nch = a.nch, G = kFieldNT / nch, t = threadIdx.x;
    const int g = t % G, c = t / G;
    const int r = rg * G + g;
    const bool active = r < a.M * a.n_nu;
    const int mp = active ? r / a.n_nu : 0, p = active ? r % a.n_nu : 0;
    const int ns = at.ns;
    const int L = (ns + nch - 1) / nch;
    const int j0 = std::min(c * L, ns), j1 = std::min(j0 + L, ns);
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
    auto bnd = [&](int dir) { return (!a.sig && a.with_c && dir == 1) ? at.Ibot : 0.0; };
    auto range = [&](int dir, int &r0, int &r1) {
        r0 = dir == 0 ? j0 : ns - j1;
        r1 = dir == 0 ? j1 : ns - j0;
    };
    auto put = [&](int dir, int k, double X, double Y) {
        const long long col = (long long)a.mu_idx[2 * mp + dir] * a.n_nu + p;
        const int j = dir == 0 ? k : ns - 1 - k;
        const long long e = base + (long long)j * a.n_mu * a.n_nu + col;
        const double I = fma(t1, Y, X), Q = t2 * Y;
        a.fout[e] = a.sub ? a.fin[e] - I : I;
        a.fout[e + plane] = a.sub ? a.fin[e + plane] - Q : Q;
    };
    // steps kb..r1-1 of direction dir from (X, Y) at point kb - 1, with a
    // register queue of the sources and depths two points ahead
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
            const bool has_dn = k + 1 < ns;
            const double d = kap * fabs(qt[1] - qt[0]);
            const double dd = has_dn ? kap * fabs(qt[2] - qt[1]) : 1.0;
            double E, cu, ck, cd;
            ray_step(a.fs, d, dd, has_dn, E, cu, ck, cd);
            X = E * X + cu * qs0[0] + ck * qs0[1] + cd * qs0[2];
            Y = E * Y + cu * qs2[0] + ck * qs2[1] + cd * qs2[2];
            alpha *= E;
            if constexpr (decltype(EMIT)::value) put(dir, k, X, Y);
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
    double Xin[2] = {0.0, 0.0}, Yin[2] = {0.0, 0.0};
    if (nch > 1) {
        // pass 1: each chunk's affine map X_out = alpha X_in + (bx, by)
        if (active) {
            for (int dir = 0; dir < 2; ++dir) {
                int r0, r1;
                range(dir, r0, r1);
                double X = 0.0, Y = 0.0, alpha = 1.0;
                if (r0 < r1) {
                    if (r0 == 0) X = bnd(dir);
                    if (std::max(r0, 1) < r1)
                        run(dir, std::max(r0, 1), r1, X, Y, alpha, std::false_type{});
                    if (r0 == 0) alpha = 0.0;  // the boundary fixes this chunk's exit
                }
                double *m = carry + ((dir * nch + c) * G + g) * 3;
                m[0] = alpha;
                m[1] = X;
                m[2] = Y;
            }
        }
        __syncthreads();
        // fold the preceding chunks (in ray order) into the entering intensity
        if (active) {
            for (int dir = 0; dir < 2; ++dir) {
                const int n = dir == 0 ? c : nch - 1 - c;
                for (int i = 0; i < n; ++i) {
                    const int cc = dir == 0 ? i : nch - 1 - i;
                    const double *m = carry + ((dir * nch + cc) * G + g) * 3;
                    Xin[dir] = m[0] * Xin[dir] + m[1];
                    Yin[dir] = m[0] * Yin[dir] + m[2];
                }
            }
        }
    }
    // pass 2 (the only pass with one chunk): from the entering intensity
    if (active) {
        for (int dir = 0; dir < 2; ++dir) {
            int r0, r1;
            range(dir, r0, r1);
            if (r0 >= r1) continue;
            double X = Xin[dir], Y = Yin[dir], alpha = 1.0;
            if (r0 == 0) {
                X = bnd(dir);
                Y = 0.0;
                put(dir, 0, X, Y);
            }
            if (std::max(r0, 1) < r1) run(dir, std::max(r0, 1), r1, X, Y, alpha, std::true_type{});
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
    // chunks per ray: doubled (up to 64) until about 64k lanes are busy
    const long long rays = (long long)h->M * h->n_nu * h->n_atm;
    int nch = 1;
    while (nch < 64 && rays * nch < 65536) nch *= 2;
    a.nch = nch;
    return a;
}

hipError_t launch_quad(const FieldArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(field_quad_kernel, dim3(a.ns_total), dim3(kFieldNT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_field_sweep(const rt_handle *h, const FieldArgs &a, hipStream_t s) {
    const int R = h->M * h->n_nu, G = kFieldNT / a.nch;
    hipLaunchKernelGGL(field_sweep_kernel, dim3((R + G - 1) / G, h->n_atm), dim3(kFieldNT), 0, s,
                       a);
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
