// rt_krylov.hip -- Jacobi-preconditioned GMRES(m), BiCGSTAB and Richardson
// on gfx950, batched over independent slabs.
//
// Every vector kernel uses one workgroup per slab (a slab has at most
// 2 * RT_MAX_NS unknowns), so a batch of slabs of uneven depth needs no
// grid-wide reduction and every slab keeps its own scalars, counters and
// convergence flag.  The operator is applied by the fused sweep; its launches
// skip converged slabs through a per-slab mask.  The host reads one integer
// (how many slabs are still active) once per GMRES cycle or every
// `check_every` iterations.
//
// Preconditioning is from the right: x = P^-1 u, so the residual the methods
// minimize and test is the unpreconditioned ||b - A x|| / ||b|| of Sect. 4.2.
// The diagonal scaling P^-1 v is folded into the sweep's input load.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include "rt_internal.h"

namespace rt {

namespace {

constexpr int NT = kKrylovThreads;
constexpr int NW = NT / kWave;
constexpr int kTriLds = 32;  // restarts up to this size solve their triangle from LDS

__device__ inline double wave_sum(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Block-wide sums of two values; every thread receives the same results.
__device__ inline void block_sum2(double &a, double &b, double *red) {
    a = wave_sum(a);
    b = wave_sum(b);
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[2 * (threadIdx.x / kWave)] = a;
        red[2 * (threadIdx.x / kWave) + 1] = b;
    }
    __syncthreads();
    a = b = 0.0;
    for (int w = 0; w < NW; ++w) {
        a += red[2 * w];
        b += red[2 * w + 1];
    }
    __syncthreads();
}

__device__ inline double block_sum(double a, double *red) {
    double b = 0.0;
    block_sum2(a, b, red);
    return a;
}

// Reduce 32 per-lane values over the 64 lanes of a wave with 32 shuffles
// (recursive halving: at each step a lane keeps one half of its values and
// receives its partner's copy of that half).  Afterwards lane l holds the
// sum of value index ((l>>5)&1)*16 + ((l>>4)&1)*8 + ((l>>3)&1)*4 +
// ((l>>2)&1)*2 + ((l>>1)&1); lanes l and l^1 hold the same value.
__device__ inline double wave_reduce_scatter32(double (&v)[32]) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const bool up = lane & 32;
        const double send = up ? v[t] : v[t + 16];
        const double keep = up ? v[t + 16] : v[t];
        v[t] = keep + __shfl_xor(send, 32);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const bool up = lane & 16;
        const double send = up ? v[t] : v[t + 8];
        const double keep = up ? v[t + 8] : v[t];
        v[t] = keep + __shfl_xor(send, 16);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bool up = lane & 8;
        const double send = up ? v[t] : v[t + 4];
        const double keep = up ? v[t + 4] : v[t];
        v[t] = keep + __shfl_xor(send, 8);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const bool up = lane & 4;
        const double send = up ? v[t] : v[t + 2];
        const double keep = up ? v[t + 2] : v[t];
        v[t] = keep + __shfl_xor(send, 4);
    }
    {
        const bool up = lane & 2;
        const double send = up ? v[0] : v[1];
        const double keep = up ? v[1] : v[0];
        v[0] = keep + __shfl_xor(send, 2);
    }
    return v[0] + __shfl_xor(v[0], 1);
}

__device__ inline int scatter_index(int lane) {
    return ((lane >> 5) & 1) * 16 + ((lane >> 4) & 1) * 8 + ((lane >> 3) & 1) * 4 +
           ((lane >> 2) & 1) * 2 + ((lane >> 1) & 1);
}

// The same for 16 values with 20 shuffles: lane l ends with the sum of value
// ((l>>5)&1)*8 + ((l>>4)&1)*4 + ((l>>3)&1)*2 + ((l>>2)&1); lanes l, l^1, l^2
// and l^3 hold the same value.
__device__ inline double wave_reduce_scatter16(double (&v)[16]) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const bool up = lane & 32;
        const double send = up ? v[t] : v[t + 8];
        const double keep = up ? v[t + 8] : v[t];
        v[t] = keep + __shfl_xor(send, 32);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bool up = lane & 16;
        const double send = up ? v[t] : v[t + 4];
        const double keep = up ? v[t + 4] : v[t];
        v[t] = keep + __shfl_xor(send, 16);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const bool up = lane & 8;
        const double send = up ? v[t] : v[t + 2];
        const double keep = up ? v[t + 2] : v[t];
        v[t] = keep + __shfl_xor(send, 8);
    }
    {
        const bool up = lane & 4;
        const double send = up ? v[0] : v[1];
        const double keep = up ? v[1] : v[0];
        v[0] = keep + __shfl_xor(send, 4);
    }
    const double s = v[0] + __shfl_xor(v[0], 2);
    return s + __shfl_xor(s, 1);
}

__device__ inline int scatter_index16(int lane) {
    return ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 +
           ((lane >> 2) & 1);
}

// Scatter-reduce K in {16, 32} per-lane values; the lanes that store a sum
// and the value index each of them holds.
template <int K>
__device__ inline double wave_reduce_scatter(double (&v)[K]) {
    if constexpr (K == 32) return wave_reduce_scatter32(v);
    else return wave_reduce_scatter16(v);
}
template <int K>
__device__ inline bool scatter_writer(int lane) {
    return K == 32 ? (lane & 1) == 0 : (lane & 3) == 0;
}
template <int K>
__device__ inline int scatter_slot(int lane) {
    return K == 32 ? scatter_index(lane) : scatter_index16(lane);
}

struct VecArgs {
    const AtmDesc *atm;
    long long N;         // total unknowns (row stride of the basis)
    int m;               // GMRES restart length
    double *V, *H, *cs, *sn, *g;
    const double *w;     // operator output
    const double *b;
    double *x;
    const double *dinv;
    double *r, *rh, *p, *v, *s, *t;  // BiCGSTAB / refinement vectors
    double *q, *u;                   // CGS (u shares the operator output's storage)
    KState *st;
    int *active;
    int *cycle;
    double tol;
    int maxit;
    int max_outer;
    const double *partial;  // the sweep's per-block quadrature sums (float values when part_f32)
    int part_f32;           // 1: written by an FP32 sweep
    const double4 *Qs;      // per slab: sums over all rays of q, q T1, q (T1^2 + T2^2)
    const double *zin;      // fused Arnoldi step: the sweep's input P^-1 v_j when the
                            // preconditioner is not diagonal (NULL: v_j .* dinv)
    const KState *outer;    // inner solve of the mixed refinement: the outer states, whose
                            // tol_next may loosen tol per slab (NULL: tol for every slab)
};

// The relative tolerance slab atm iterates to.
__device__ inline double slab_tol(const VecArgs &a, int atm) {
    return a.outer ? fmax(a.tol, a.outer[atm].tol_next) : a.tol;
}

// ---------------------------------------------------------------- counting
__global__ void count_kernel(const int *flags, int n, int *out) {
    __shared__ int red[NW];
    int c = 0;
    for (int i = threadIdx.x; i < n; i += NT) c += flags[i] != 0;
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < NW; ++w) s += red[w];
        *out = s;
    }
}

__global__ void init_state_kernel(KState *st, int *active, int *cycle, int n_atm,
                                  const int *from_mask) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_atm) return;
    KState k = {};
    k.status = RT_ENOCONV;
    st[i] = k;
    active[i] = from_mask ? (from_mask[i] != 0) : 1;
    cycle[i] = 0;
}

// -------------------------------------------------------------------- GMRES
// (Re)start a cycle: r = b - A x (A x in w; r = b when x is known to be zero),
// test it, and set v_0 = r / ||r||, g = [||r||, 0, ...].  accept_est: also
// accept the previous cycle's Arnoldi residual estimate (inner solves of the
// mixed-precision refinement, whose explicitly recomputed FP32 residual has a
// rounding floor well above the estimate; the outer FP64 residual decides).
__global__ void gm_restart_kernel(VecArgs a, int first, int x_zero, int accept_est) {
    __shared__ double red[2 * NW];
    __shared__ int s_go;
    __shared__ double s_beta;
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    double rr = 0.0, bb = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) {
        const double bl = a.b[base + l];
        const double rl = x_zero ? bl : bl - a.w[base + l];
        a.V[base + l] = rl;
        rr += rl * rl;
        bb += bl * bl;
    }
    block_sum2(rr, bb, red);
    KState &S = a.st[atm];
    if (threadIdx.x == 0) {
        if (first) S.bnorm = sqrt(bb);
        if (!x_zero) S.matvecs += 1;
        const double beta = sqrt(rr);
        S.beta = beta;
        s_beta = beta;
        int go = 0;
        if (S.bnorm == 0.0) {
            S.status = RT_OK;
            S.relres = 0.0;
            go = -1;  // zero right-hand side: x = 0
        } else if (!(beta == beta) || isinf(beta)) {
            S.status = RT_EBREAKDOWN;
            S.relres = beta / S.bnorm;
        } else if (beta / S.bnorm < slab_tol(a, atm) ||
                   (accept_est && !first && S.resid / S.bnorm < slab_tol(a, atm))) {
            S.status = RT_OK;
            S.relres = beta / S.bnorm;
        } else if (S.iters >= a.maxit) {
            S.status = RT_ENOCONV;
            S.relres = beta / S.bnorm;
        } else {
            go = 1;
        }
        s_go = go;
        if (go != 1) {
            a.active[atm] = 0;
            a.cycle[atm] = 0;
        } else {
            S.inner = 0;
            a.cycle[atm] = 1;
            double *g = a.g + (long long)atm * (a.m + 1);
            g[0] = beta;
            for (int i = 1; i <= a.m; ++i) g[i] = 0.0;
        }
    }
    __syncthreads();
    if (s_go == -1) {
        for (int l = threadIdx.x; l < n; l += NT) a.x[base + l] = 0.0;
    } else if (s_go == 1) {
        const double inv = 1.0 / s_beta;
        for (int l = threadIdx.x; l < n; l += NT) a.V[base + l] *= inv;
    }
}

// Column j of the Hessenberg matrix of one slab (thread 0 only): h[0..j]
// are the Gram-Schmidt coefficients, hn = ||w||; the earlier rotations
// (cs, sn)[0..j-1] are applied, the new one is formed, and g and the
// slab's convergence state are updated (Saad & Schultz).  The column is
// stored already rotated (the triangular factor the update solves with).
__device__ inline void hessenberg_finish(const VecArgs &a, int atm, int j, double hjj, double hn) {
    const int m = a.m;
    double *H = a.H + (long long)atm * (m + 1) * m;
    double *g = a.g + (long long)atm * (m + 1);
    const double den = sqrt(hjj * hjj + hn * hn);
    const double c = (den > 0.0) ? hjj / den : 1.0;
    const double s = (den > 0.0) ? hn / den : 0.0;
    a.cs[(long long)atm * m + j] = c;
    a.sn[(long long)atm * m + j] = s;
    H[j * m + j] = den;
    H[(j + 1) * m + j] = 0.0;
    const double gj = g[j];
    g[j + 1] = -s * gj;
    g[j] = c * gj;
    KState &S = a.st[atm];
    S.resid = fabs(s * gj);
    S.iters += 1;
    S.matvecs += 1;
    S.inner = j + 1;
    const bool done = (S.resid / S.bnorm < slab_tol(a, atm)) || !(hn > 0.0) ||
                      (S.iters >= a.maxit) || (j + 1 == m) || !(S.resid == S.resid);
    if (done) a.cycle[atm] = 0;
}

__device__ inline void hessenberg_column_lds(const VecArgs &a, int atm, int j, double *h,
                                             const double *cs, const double *sn, double hn) {
    const int m = a.m;
    double *H = a.H + (long long)atm * (m + 1) * m;
    for (int i = 0; i < j; ++i) {
        const double h0 = h[i], h1 = h[i + 1];
        h[i] = cs[i] * h0 + sn[i] * h1;
        h[i + 1] = -sn[i] * h0 + cs[i] * h1;
    }
    for (int i = 0; i < j; ++i) H[i * m + j] = h[i];
    hessenberg_finish(a, atm, j, h[j], hn);
}

template <int MR_>
__device__ inline void hessenberg_column_regs(const VecArgs &a, int atm, int j, const double *hs,
                                              const double *cs, const double *sn, double hn) {
    const int m = a.m;
    double *H = a.H + (long long)atm * (m + 1) * m;
    double h[MR_];
#pragma unroll
    for (int i = 0; i < MR_; ++i) h[i] = (i <= j) ? hs[i] : 0.0;
#pragma unroll
    for (int i = 0; i + 1 < MR_; ++i) {
        if (i < j) {
            const double c = cs[i], s = sn[i], h0 = h[i], h1 = h[i + 1];
            h[i] = c * h0 + s * h1;
            h[i + 1] = -s * h0 + c * h1;
        }
    }
    double hjj = 0.0;
#pragma unroll
    for (int i = 0; i < MR_; ++i) {
        if (i < j) H[i * m + j] = h[i];
        if (i == j) hjj = h[i];
    }
    hessenberg_finish(a, atm, j, hjj, hn);
}

// One Arnoldi step j: w = A P^-1 v_j is in a.w.  Classical Gram-Schmidt twice
// (h = V^T w; w -= V h; repeated), h_{j+1,j} = ||w||, v_{j+1} = w / ||w||,
// then the Givens rotations of the Hessenberg column and the residual
// estimate |g_{j+1}| (Saad & Schultz).  E: vector elements per thread; the
// basis is read 32 rows at a time so that 32 loads per element are in flight.
template <int E>
__global__ __launch_bounds__(NT) void gm_arnoldi_kernel(VecArgs a, int j) {
    __shared__ double red[32 * NW];
    __shared__ double hsum[RT_MAX_RESTART + 1];
    __shared__ double hp[RT_MAX_RESTART + 1];
    __shared__ double red2[2 * NW];
    __shared__ double scs[RT_MAX_RESTART], ssn[RT_MAX_RESTART];
    const int atm = blockIdx.x;
    if (!a.cycle[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    if (tid < j) {
        scs[tid] = a.cs[(long long)atm * a.m + tid];
        ssn[tid] = a.sn[(long long)atm * a.m + tid];
    }

    double wl[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int l = tid + e * NT;
        wl[e] = (l < n) ? a.w[base + l] : 0.0;
    }
    for (int i = tid; i <= j; i += NT) hsum[i] = 0.0;

    for (int pass = 0; pass < 2; ++pass) {
        for (int i0 = 0; i0 <= j; i0 += 32) {
            const int cnt = min(32, j + 1 - i0);
            double part[32];
#pragma unroll
            for (int t = 0; t < 32; ++t) part[t] = 0.0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int l = tid + e * NT;
                if (l < n) {
                    const double *vp = a.V + (long long)i0 * a.N + base + l;
#pragma unroll
                    for (int t = 0; t < 32; ++t)
                        if (t < cnt) part[t] += vp[(long long)t * a.N] * wl[e];
                }
            }
            const double sum = wave_reduce_scatter32(part);
            if ((lane & 1) == 0) red[scatter_index(lane) * NW + wave] = sum;
            __syncthreads();
            if (tid < cnt) {
                double s = 0.0;
                for (int w = 0; w < NW; ++w) s += red[tid * NW + w];
                hp[i0 + tid] = s;
            }
            __syncthreads();
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int l = tid + e * NT;
            if (l < n) {
                double s = 0.0;
                for (int i0 = 0; i0 <= j; i0 += 32) {
                    const int cnt = min(32, j + 1 - i0);
                    const double *vp = a.V + (long long)i0 * a.N + base + l;
                    double v[32];
#pragma unroll
                    for (int t = 0; t < 32; ++t) v[t] = (t < cnt) ? vp[(long long)t * a.N] : 0.0;
#pragma unroll
                    for (int t = 0; t < 32; ++t)
                        if (t < cnt) s += hp[i0 + t] * v[t];
                }
                wl[e] -= s;
            }
        }
        for (int i = tid; i <= j; i += NT) hsum[i] += hp[i];
        __syncthreads();
    }

    double nn = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) nn += wl[e] * wl[e];
    const double hn = sqrt(block_sum(nn, red2));
    if (hn > 0.0) {
        const double inv = 1.0 / hn;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int l = tid + e * NT;
            if (l < n) a.V[(long long)(j + 1) * a.N + base + l] = wl[e] * inv;
        }
    }
    // the earlier rotations (read into LDS at the start, ordered by the
    // block sums' barriers) are applied by one thread from LDS: global loads
    // and stores in that sequential loop would each wait a memory round trip
    if (tid == 0) hessenberg_column_lds(a, atm, j, hsum, scs, ssn, hn);

}

// The same step for slabs of at most NTF points and restarts m < MR, with the
// operator's last pass fused in and the basis held in registers (MR_ rows:
// steps j < 16 hold half the rows, which halves the basis registers and lets
// two 512-thread workgroups share a CU):
//  * w = A P^-1 v_j is formed here from the sweep's per-block quadrature sums
//    (the finalize pass: J = sum of the slab's block slots in block order plus
//    the source part Q S, w = z - xi [J00, W2 J20], z = P^-1 v_j), so w is
//    never written to memory;
//  * each thread owns one depth point and keeps (s00, s20) of basis rows
//    0..j in registers, so both Gram-Schmidt passes read the basis once.
constexpr int NTF = 512;
constexpr int NWF = NTF / kWave;
constexpr int MR = 32;

__device__ inline double block_sum_f(double a, double *red) {
    a = wave_sum(a);
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = a;
    __syncthreads();
    a = 0.0;
    for (int w = 0; w < NWF; ++w) a += red[w];
    return a;
}

template <int MR_>
__global__ __launch_bounds__(NTF) void gm_arnoldi_fused_kernel(VecArgs a, int j) {
    static_assert(MR_ == 16 || MR_ == 32, "basis rows held in registers");
    __shared__ double red[MR_ * NWF];
    __shared__ double hp[MR_];
    __shared__ double hsum[MR_];
    __shared__ double red2[NWF];
    __shared__ double scs[MR_], ssn[MR_];
    const int atm = blockIdx.x;
    if (!a.cycle[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int k = tid;  // depth point
    const bool on = k < at.ns;
    if (tid < j) {
        scs[tid] = a.cs[(long long)atm * a.m + tid];
        ssn[tid] = a.sn[(long long)atm * a.m + tid];
    }
    const long long e0 = 2LL * (at.doff + k);

    // basis rows 0..j at this point (zero beyond)
    double v0[MR_], v2[MR_];
    if constexpr (MR_ == 32) {
#pragma unroll
        for (int t = 0; t < MR_; ++t) {
            v0[t] = v2[t] = 0.0;
            if (on && t <= j) {
                const double2 x = *reinterpret_cast<const double2 *>(a.V + (long long)t * a.N + e0);
                v0[t] = x.x;
                v2[t] = x.y;
            }
        }
    } else {
        // branch-free: rows past j re-read row j, points past the slab read
        // its first point, and both are replaced by zero (a branch per row
        // would copy the whole register array at every join)
        const long long eb = on ? e0 : 2LL * at.doff;
#pragma unroll
        for (int t = 0; t < MR_; ++t) {
            const double2 x =
                *reinterpret_cast<const double2 *>(a.V + (long long)min(t, j) * a.N + eb);
            const bool use = on && t <= j;
            v0[t] = use ? x.x : 0.0;
            v2[t] = use ? x.y : 0.0;
        }
    }
    if (tid < MR_) hsum[tid] = 0.0;

    // w = A P^-1 v_j from the sweep's block slots, read 8 at a time with all
    // loads of a group in flight (addresses clamped, extra values unused).
    // A slab of many blocks and few points (a single small slab's plan) lets
    // the idle threads share them: G lanes per point, lane s adding slots s,
    // s + G, ..., and the point's thread adding the G sums in order.
    double J0 = 0.0, J2 = 0.0;
    {
        const long long stride = 2LL * at.ns;
        auto add_slots = [&](const auto *pJ, int s0, int step, double &X0, double &X2) {
            using V2 = typename std::conditional<sizeof(*pJ) == 4, float2, double2>::type;
            for (int b0 = s0; b0 < at.nblk; b0 += 8 * step) {
                V2 p[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    p[u] = *reinterpret_cast<const V2 *>(pJ + min(b0 + u * step, at.nblk - 1) * stride);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (b0 + u * step < at.nblk) {
                        X0 += (double)p[u].x;
                        X2 += (double)p[u].y;
                    }
                }
            }
        };
        auto add_point = [&](int kp, int s0, int step, double &X0, double &X2) {
            if (a.part_f32)
                add_slots(reinterpret_cast<const float *>(a.partial) + at.part_off + 2 * kp, s0, step,
                          X0, X2);
            else
                add_slots(a.partial + at.part_off + 2 * kp, s0, step, X0, X2);
        };
        const int G = at.nblk > 16 ? max(1, min(16, NTF / at.ns)) : 1;
        if (G == 1) {
            if (on) add_point(k, 0, 1, J0, J2);
        } else {
            __shared__ double2 sred[NTF];
            double X0 = 0.0, X2 = 0.0;
            if (tid < G * at.ns) add_point(tid % at.ns, tid / at.ns, G, X0, X2);
            sred[tid] = make_double2(X0, X2);
            __syncthreads();
            if (on)
                for (int g = 0; g < G; ++g) {
                    J0 += sred[k + g * at.ns].x;
                    J2 += sred[k + g * at.ns].y;
                }
        }
    }
    double w0 = 0.0, w2 = 0.0;
    if (on) {
        double vj0 = 0.0, vj2 = 0.0;
#pragma unroll
        for (int t = 0; t < MR_; ++t)
            if (t == j) {
                vj0 = v0[t];
                vj2 = v2[t];
            }
        double z0, z2;
        if (a.zin) {
            const double2 z = *reinterpret_cast<const double2 *>(a.zin + e0);
            z0 = z.x;
            z2 = z.y;
        } else {
            const double2 d = *reinterpret_cast<const double2 *>(a.dinv + e0);
            z0 = vj0 * d.x;
            z2 = vj2 * d.y;
        }
        const double4 Q = a.Qs[atm];
        J0 += z0 * Q.x + z2 * Q.y;
        J2 += z0 * Q.y + z2 * Q.z;
        w0 = z0 - at.xi * J0;
        w2 = z2 - at.xi * at.W2 * J2;
    }

    // classical Gram-Schmidt, twice
    for (int pass = 0; pass < 2; ++pass) {
        double part[MR_];
#pragma unroll
        for (int t = 0; t < MR_; ++t) part[t] = v0[t] * w0 + v2[t] * w2;
        const double sum = wave_reduce_scatter<MR_>(part);
        if (scatter_writer<MR_>(lane)) red[scatter_slot<MR_>(lane) * NWF + wave] = sum;
        __syncthreads();
        if (tid < MR_) {
            double s = 0.0;
            for (int w = 0; w < NWF; ++w) s += red[tid * NWF + w];
            hp[tid] = s;
            hsum[tid] += s;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < MR_; ++t) {
            const double h = hp[t];  // zero for t > j
            w0 -= h * v0[t];
            w2 -= h * v2[t];
        }
    }

    const double hn = sqrt(block_sum_f(w0 * w0 + w2 * w2, red2));
    if (hn > 0.0 && on) {
        const double inv = 1.0 / hn;
        *reinterpret_cast<double2 *>(a.V + (long long)(j + 1) * a.N + e0) =
            make_double2(w0 * inv, w2 * inv);
    }
    // the earlier rotations (read into LDS at the start, ordered by the
    // block sums' barriers) are applied by one thread in registers
    if (tid == 0) hessenberg_column_regs<MR_>(a, atm, j, hsum, scs, ssn, hn);

}

// End of a cycle: solve the triangular system H y = g and set x += P^-1 V y.
template <int E>
__global__ __launch_bounds__(NT) void gm_update_kernel(VecArgs a) {
    __shared__ double y[RT_MAX_RESTART];
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    const int jj = a.st[atm].inner;
    const int m = a.m;
    const double *H = a.H + (long long)atm * (m + 1) * m;
    const double *g = a.g + (long long)atm * (m + 1);
    if (jj <= kTriLds) {
        // the triangle and g read into LDS by all threads at once, then the
        // back substitution by one thread from LDS (from global memory each
        // of its ~jj^2/2 reads would wait a full round trip)
        __shared__ double Ht[kTriLds * kTriLds], gt[kTriLds];
        for (int e = threadIdx.x; e < jj * jj; e += NT) {
            const int i = e / jj, l = e % jj;
            if (l >= i) Ht[i * kTriLds + l] = H[i * m + l];
        }
        for (int i = threadIdx.x; i < jj; i += NT) gt[i] = g[i];
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = jj - 1; i >= 0; --i) {
                double s = gt[i];
                for (int l = i + 1; l < jj; ++l) s -= Ht[i * kTriLds + l] * y[l];
                y[i] = s / Ht[i * kTriLds + i];
            }
        }
    } else if (threadIdx.x == 0) {
        for (int i = jj - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < jj; ++l) s -= H[i * m + l] * y[l];
            y[i] = s / H[i * m + i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int l = threadIdx.x + e * NT;
        if (l < n) {
            double s = 0.0;
            for (int i0 = 0; i0 < jj; i0 += 32) {
                const int cnt = min(32, jj - i0);
                const double *vp = a.V + (long long)i0 * a.N + base + l;
                double v[32];
#pragma unroll
                for (int t = 0; t < 32; ++t) v[t] = (t < cnt) ? vp[(long long)t * a.N] : 0.0;
#pragma unroll
                for (int t = 0; t < 32; ++t)
                    if (t < cnt) s += y[i0 + t] * v[t];
            }
            a.x[base + l] += a.dinv[base + l] * s;
        }
    }
    if (threadIdx.x == 0) a.cycle[atm] = 0;
}

// ----------------------------------------------------------------- BiCGSTAB
// r = b - A x, r^ = r, p = v = 0, rho_old = alpha = omega = 1.
__global__ void bi_start_kernel(VecArgs a) {
    __shared__ double red[2 * NW];
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    double rr = 0.0, bb = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) {
        const double bl = a.b[base + l];
        const double rl = bl - a.w[base + l];
        a.r[base + l] = rl;
        a.rh[base + l] = rl;
        a.p[base + l] = 0.0;
        a.v[base + l] = 0.0;
        rr += rl * rl;
        bb += bl * bl;
    }
    block_sum2(rr, bb, red);
    if (threadIdx.x == 0) {
        KState &S = a.st[atm];
        S.bnorm = sqrt(bb);
        S.matvecs += 1;
        S.rho_old = S.alpha = S.omega = 1.0;
        S.iters = 0;
        const double rn = sqrt(rr);
        if (S.bnorm == 0.0) {
            S.status = RT_OK;
            S.relres = 0.0;
            a.active[atm] = 0;
        } else if (rn / S.bnorm < a.tol) {
            S.status = RT_OK;
            S.relres = rn / S.bnorm;
            a.active[atm] = 0;
        }
    }
    if (bb == 0.0)  // every thread holds the same block sum
        for (int l = threadIdx.x; l < n; l += NT) a.x[base + l] = 0.0;
}

// rho = (r^, r); beta = (rho / rho_old)(alpha / omega); p = r + beta (p - omega v).
__global__ void bi_dir_kernel(VecArgs a) {
    __shared__ double red[2 * NW];
    __shared__ int s_ok;
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    KState &S = a.st[atm];
    double rho = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) rho += a.rh[base + l] * a.r[base + l];
    rho = block_sum(rho, red);
    if (threadIdx.x == 0) {
        s_ok = (rho != 0.0) && isfinite(rho) && (S.iters < a.maxit);
        if (!s_ok) {
            S.status = (S.iters >= a.maxit) ? RT_ENOCONV : RT_EBREAKDOWN;
            a.active[atm] = 0;
        } else {
            S.rho = rho;
        }
    }
    __syncthreads();
    if (!s_ok) return;
    const double beta = (rho / S.rho_old) * (S.alpha / S.omega);
    const double om = S.omega;
    for (int l = threadIdx.x; l < n; l += NT)
        a.p[base + l] = a.r[base + l] + beta * (a.p[base + l] - om * a.v[base + l]);
}

// v = A P^-1 p is in a.v.  alpha = rho / (r^, v); s = r - alpha v.
__global__ void bi_half_kernel(VecArgs a) {
    __shared__ double red[2 * NW];
    __shared__ int s_state;
    __shared__ double s_alpha;
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    KState &S = a.st[atm];
    double rv = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) rv += a.rh[base + l] * a.v[base + l];
    rv = block_sum(rv, red);
    if (threadIdx.x == 0) {
        S.matvecs += 1;
        if (rv == 0.0 || !isfinite(rv)) {
            S.status = RT_EBREAKDOWN;
            a.active[atm] = 0;
            s_state = 0;
        } else {
            S.alpha = S.rho / rv;
            s_alpha = S.alpha;
            s_state = 1;
        }
    }
    __syncthreads();
    if (!s_state) return;
    const double alpha = s_alpha;
    double ss = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) {
        const double sl = a.r[base + l] - alpha * a.v[base + l];
        a.s[base + l] = sl;
        ss += sl * sl;
    }
    ss = block_sum(ss, red);
    const double bnorm = S.bnorm;  // written by an earlier kernel
    if (sqrt(ss) / bnorm < a.tol) {  // converged at the half step
        for (int l = threadIdx.x; l < n; l += NT)
            a.x[base + l] += alpha * a.dinv[base + l] * a.p[base + l];
        __syncthreads();
        if (threadIdx.x == 0) {
            S.iters += 1;
            S.status = RT_OK;
            S.half_done = 1;
            a.active[atm] = 0;
        }
    }
}

// t = A P^-1 s is in a.t.  omega = (t, s) / (t, t); x += alpha P^-1 p + omega
// P^-1 s; r = s - omega t.
__global__ void bi_full_kernel(VecArgs a) {
    __shared__ double red[2 * NW];
    __shared__ int s_ok;
    __shared__ double s_omega;
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    KState &S = a.st[atm];
    double ts = 0.0, tt = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) {
        const double tl = a.t[base + l];
        ts += tl * a.s[base + l];
        tt += tl * tl;
    }
    block_sum2(ts, tt, red);
    if (threadIdx.x == 0) {
        S.matvecs += 1;
        s_ok = (tt != 0.0) && isfinite(tt);
        if (!s_ok) {
            S.status = RT_EBREAKDOWN;
            a.active[atm] = 0;
        } else {
            S.omega = ts / tt;
            s_omega = S.omega;
        }
    }
    __syncthreads();
    if (!s_ok) return;
    const double alpha = S.alpha, om = s_omega;  // alpha: written by an earlier kernel
    double rr = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) {
        const double d = a.dinv[base + l];
        a.x[base + l] += alpha * d * a.p[base + l] + om * d * a.s[base + l];
        const double rl = a.s[base + l] - om * a.t[base + l];
        a.r[base + l] = rl;
        rr += rl * rl;
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) {
        S.iters += 1;
        const double rel = sqrt(rr) / S.bnorm;
        if (rel < a.tol) {
            S.status = RT_OK;
            a.active[atm] = 0;
        } else if (om == 0.0 || !isfinite(rel)) {
            S.status = RT_EBREAKDOWN;
            a.active[atm] = 0;
        } else if (S.iters >= a.maxit) {
            S.status = RT_ENOCONV;
            a.active[atm] = 0;
        }
        S.rho_old = S.rho;
    }
}

// ---------------------------------------------------------------------- CGS
// Conjugate gradient squared (Sonneveld; Sect. 2.2), right-preconditioned.
// Vectors: r, r^ (rh), u (the operator output's storage, free after the
// start), p, q, v = A P^-1 p, s = u + q, t = A P^-1 s.
// r = b - A x (A x in a.w), r^ = r.
__global__ void cg_start_kernel(VecArgs a) {
    __shared__ double red[2 * NW];
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    double rr = 0.0, bb = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) {
        const double bl = a.b[base + l];
        const double rl = bl - a.w[base + l];
        a.r[base + l] = rl;
        a.rh[base + l] = rl;
        rr += rl * rl;
        bb += bl * bl;
    }
    block_sum2(rr, bb, red);
    if (threadIdx.x == 0) {
        KState &S = a.st[atm];
        S.bnorm = sqrt(bb);
        S.matvecs += 1;
        S.rho_old = 1.0;
        S.iters = 0;
        const double rn = sqrt(rr);
        if (S.bnorm == 0.0) {
            S.status = RT_OK;
            S.relres = 0.0;
            a.active[atm] = 0;
        } else if (rn / S.bnorm < a.tol) {
            S.status = RT_OK;
            S.relres = rn / S.bnorm;
            a.active[atm] = 0;
        }
    }
    if (bb == 0.0)  // every thread holds the same block sum
        for (int l = threadIdx.x; l < n; l += NT) a.x[base + l] = 0.0;
}

// rho = (r^, r); first step u = p = r, else beta = rho / rho_old,
// u = r + beta q, p = u + beta (q + beta p).
__global__ void cg_dir_kernel(VecArgs a) {
    __shared__ double red[2 * NW];
    __shared__ int s_ok;
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    KState &S = a.st[atm];
    double rho = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) rho += a.rh[base + l] * a.r[base + l];
    rho = block_sum(rho, red);
    if (threadIdx.x == 0) {
        s_ok = (rho != 0.0) && isfinite(rho) && (S.iters < a.maxit);
        if (!s_ok) {
            S.status = (S.iters >= a.maxit) ? RT_ENOCONV : RT_EBREAKDOWN;
            a.active[atm] = 0;
        } else {
            S.rho = rho;
        }
    }
    __syncthreads();
    if (!s_ok) return;
    double *u = a.u;
    if (S.iters == 0) {
        for (int l = threadIdx.x; l < n; l += NT) u[base + l] = a.p[base + l] = a.r[base + l];
    } else {
        const double beta = rho / S.rho_old;
        for (int l = threadIdx.x; l < n; l += NT) {
            const double ql = a.q[base + l];
            const double ul = a.r[base + l] + beta * ql;
            u[base + l] = ul;
            a.p[base + l] = ul + beta * (ql + beta * a.p[base + l]);
        }
    }
}

// v = A P^-1 p is in a.v.  alpha = rho / (r^, v); q = u - alpha v;
// s = u + q; x += alpha P^-1 s.
__global__ void cg_half_kernel(VecArgs a) {
    __shared__ double red[2 * NW];
    __shared__ int s_ok;
    __shared__ double s_alpha;
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    KState &S = a.st[atm];
    double sig = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) sig += a.rh[base + l] * a.v[base + l];
    sig = block_sum(sig, red);
    if (threadIdx.x == 0) {
        S.matvecs += 1;
        s_ok = (sig != 0.0) && isfinite(sig);
        if (!s_ok) {
            S.status = RT_EBREAKDOWN;
            a.active[atm] = 0;
        } else {
            S.alpha = S.rho / sig;
            s_alpha = S.alpha;
        }
    }
    __syncthreads();
    if (!s_ok) return;
    const double alpha = s_alpha;
    const double *u = a.u;
    for (int l = threadIdx.x; l < n; l += NT) {
        const double ul = u[base + l];
        const double ql = ul - alpha * a.v[base + l];
        a.q[base + l] = ql;
        const double sl = ul + ql;
        a.s[base + l] = sl;
        a.x[base + l] += alpha * a.dinv[base + l] * sl;
    }
}

// t = A P^-1 (u + q) is in a.t.  r -= alpha t; test.
__global__ void cg_full_kernel(VecArgs a) {
    __shared__ double red[2 * NW];
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    KState &S = a.st[atm];
    const double alpha = S.alpha;  // written by an earlier kernel
    double rr = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) {
        const double rl = a.r[base + l] - alpha * a.t[base + l];
        a.r[base + l] = rl;
        rr += rl * rl;
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) {
        S.matvecs += 1;
        S.iters += 1;
        const double rel = sqrt(rr) / S.bnorm;
        if (rel < a.tol) {
            S.status = RT_OK;
            a.active[atm] = 0;
        } else if (!isfinite(rel)) {
            S.status = RT_EBREAKDOWN;
            a.active[atm] = 0;
        } else if (S.iters >= a.maxit) {
            S.status = RT_ENOCONV;
            a.active[atm] = 0;
        }
        S.rho_old = S.rho;
    }
}

// --------------------------------------------------------------- Richardson
// One step of x <- x + P^-1 (b - A x) (eq. rich_iteration), A x in a.w.
__global__ void ri_step_kernel(VecArgs a, int first) {
    __shared__ double red[2 * NW];
    __shared__ int s_go;
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    KState &S = a.st[atm];
    double rr = 0.0, bb = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) {
        const double bl = a.b[base + l];
        const double rl = bl - a.w[base + l];
        a.r[base + l] = rl;
        rr += rl * rl;
        bb += bl * bl;
    }
    block_sum2(rr, bb, red);
    if (threadIdx.x == 0) {
        if (first) S.bnorm = sqrt(bb);
        S.matvecs += 1;
        const double rel = (S.bnorm > 0.0) ? sqrt(rr) / S.bnorm : 0.0;
        S.relres = rel;
        int go = 0;
        if (S.bnorm == 0.0) {
            S.status = RT_OK;
            go = -1;
        } else if (rel < a.tol) {
            S.status = RT_OK;
        } else if (!isfinite(rel)) {
            S.status = RT_EBREAKDOWN;
        } else if (S.iters >= a.maxit) {
            S.status = RT_ENOCONV;
        } else {
            go = 1;
            S.iters += 1;
        }
        if (go != 1) a.active[atm] = 0;
        s_go = go;
    }
    __syncthreads();
    if (s_go == 1) {
        for (int l = threadIdx.x; l < n; l += NT) a.x[base + l] += a.dinv[base + l] * a.r[base + l];
    } else if (s_go == -1) {
        for (int l = threadIdx.x; l < n; l += NT) a.x[base + l] = 0.0;
    }
}

// ------------------------------------------------- residual and refinement
// relres = ||b - A x|| / ||b|| (A x in a.w); used after BiCGSTAB.
__global__ void relres_kernel(VecArgs a) {
    __shared__ double red[2 * NW];
    const int atm = blockIdx.x;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    double rr = 0.0, bb = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) {
        const double bl = a.b[base + l];
        const double rl = bl - a.w[base + l];
        rr += rl * rl;
        bb += bl * bl;
    }
    block_sum2(rr, bb, red);
    if (threadIdx.x == 0) {
        KState &S = a.st[atm];
        S.relres = (bb > 0.0) ? sqrt(rr / bb) : 0.0;
        S.matvecs += 1;
    }
}

// Status of a direct solve: converged unless a pivot was zero.
__global__ void direct_status_kernel(KState *st, const int *sing, int n_atm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_atm) return;
    st[i].status = sing[i] ? RT_EBREAKDOWN : RT_OK;
    st[i].iters = 0;
}

// Outer step of the mixed-precision refinement: r = b - A x in FP64 (A x in
// a.w), test it; if the slab goes on, clear the correction d (a.s), and
// record the relative tolerance that brings it below rtol (kIrMargin).
__global__ void ir_residual_kernel(VecArgs a, int first) {
    __shared__ double red[2 * NW];
    __shared__ int s_go;
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    KState &S = a.st[atm];
    double rr = 0.0, bb = 0.0;
    for (int l = threadIdx.x; l < n; l += NT) {
        const double bl = a.b[base + l];
        const double rl = bl - a.w[base + l];
        a.r[base + l] = rl;
        rr += rl * rl;
        bb += bl * bl;
    }
    block_sum2(rr, bb, red);
    if (threadIdx.x == 0) {
        if (first) S.bnorm = sqrt(bb);
        S.matvecs += 1;
        const double rel = (S.bnorm > 0.0) ? sqrt(rr) / S.bnorm : 0.0;
        S.relres = rel;
        int go = 0;
        if (S.bnorm == 0.0) {
            S.status = RT_OK;
            go = -1;
        } else if (rel < a.tol) {
            S.status = RT_OK;
        } else if (!isfinite(rel)) {
            S.status = RT_EBREAKDOWN;
        } else if (S.outer >= a.max_outer || S.iters >= a.maxit) {
            S.status = RT_ENOCONV;
        } else {
            go = 1;
            S.outer += 1;
            S.tol_next = kIrMargin * a.tol / rel;
        }
        if (go != 1) a.active[atm] = 0;
        s_go = go;
    }
    __syncthreads();
    if (s_go == 1) {
        for (int l = threadIdx.x; l < n; l += NT) a.s[base + l] = 0.0;
    } else if (s_go == -1) {
        for (int l = threadIdx.x; l < n; l += NT) a.x[base + l] = 0.0;
    }
}

// x += d for slabs still refining; fold the inner solve's counters in.
__global__ void ir_update_kernel(VecArgs a, const KState *inner) {
    const int atm = blockIdx.x;
    if (!a.active[atm]) return;
    const AtmDesc at = a.atm[atm];
    const int n = 2 * at.ns;
    const long long base = 2LL * at.doff;
    for (int l = threadIdx.x; l < n; l += NT) a.x[base + l] += a.s[base + l];
    if (threadIdx.x == 0) {
        a.st[atm].iters += inner[atm].iters;
        a.st[atm].matvecs += inner[atm].matvecs;
    }
}

__global__ void scale_kernel(const double *v, const double *d, double *z, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = d[i] * v[i];
}

}  // namespace

// ===================================================================== host

hipError_t launch_scale(const double *v, const double *d, double *z, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, d, z,
                       n);
    return hipGetLastError();
}

namespace {

struct Driver {
    rt_handle *h;
    hipStream_t s;
    hipError_t err = hipSuccess;
    // SOR or SSOR: the solvers run on y = P x with the operator A P^-1 and
    // unit scaling in their updates (right preconditioning, the same iterates),
    // and x = P^-1 y at the end.  Jacobi folds D^-1 into the sweep instead.
    bool tri = false;
    // mixed refinement: the outer states while an inner solve runs (per-slab
    // tolerances, VecArgs::outer)
    const KState *outer = nullptr;

    bool ok(hipError_t e) {
        if (e != hipSuccess && err == hipSuccess) err = e;
        return err == hipSuccess;
    }

    // Run `body` (kernel launches on this->s) as a HIP graph: captured on the
    // handle's own stream the first time this key is seen, then replayed.
    // The replay is ordered after the caller's stream and the caller's
    // stream after it, by events.  Captured launches record their arguments,
    // so the key holds every argument that can differ between calls.
    template <typename F>
    void graph(const std::vector<unsigned long long> &key, F body) {
        if (err != hipSuccess) return;
        if (!h->gstream) {
            if (!ok(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking))) return;
            for (hipEvent_t &e : h->gev)
                if (!ok(hipEventCreateWithFlags(&e, hipEventDisableTiming))) return;
        }
        hipGraphExec_t exec = nullptr;
        for (const auto &g : h->graphs)
            if (g.key == key) exec = g.exec;
        if (!exec) {
            const hipStream_t caller = s;
            s = h->gstream;
            if (!ok(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal))) {
                s = caller;
                return;
            }
            body();
            hipGraph_t gr = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &gr);
            s = caller;
            if (!ok(e)) return;
            const hipError_t ei = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (!ok(ei)) return;
            // keep the most recent few (a key holds the caller's x and b)
            if (h->graphs.size() >= 16) {
                ok(hipStreamSynchronize(h->gstream));
                (void)hipGraphExecDestroy(h->graphs.front().exec);
                h->graphs.erase(h->graphs.begin());
            }
            h->graphs.push_back(rt_handle::Graph{key, exec});
        }
        ok(hipEventRecord(h->gev[0], s));
        ok(hipStreamWaitEvent(h->gstream, h->gev[0], 0));
        ok(hipGraphLaunch(exec, h->gstream));
        ok(hipEventRecord(h->gev[1], h->gstream));
        ok(hipStreamWaitEvent(s, h->gev[1], 0));
    }

    static unsigned long long bits(double v) {
        unsigned long long u;
        std::memcpy(&u, &v, sizeof u);
        return u;
    }
    static unsigned long long bits(const void *p) { return (unsigned long long)(uintptr_t)p; }

    // w = A (scale .* in), FP64 or FP32 sweep, for slabs whose mask is set
    void sweep(const double *in, const double *scale, double *out, const int *mask, bool fp32) {
        ok(apply_operator(h, in, scale, out, mask, fp32, 0, s));
    }

    // out = A P^-1 v
    void prec_sweep(const double *v, double *out, const int *mask, bool fp32) {
        if (tri) {
            ok(precond_tri(h, v, h->d_pz, mask, s));
            sweep(h->d_pz, nullptr, out, mask, fp32);
        } else {
            sweep(v, h->d_dinv, out, mask, fp32);
        }
    }

    // the operator on the solver's iterate: A x (Jacobi) or A P^-1 y
    void iter_sweep(const double *x, double *out, const int *mask, bool fp32) {
        if (tri) prec_sweep(x, out, mask, fp32);
        else sweep(x, nullptr, out, mask, fp32);
    }

    // elements per thread for the largest slab: 2, 4, 8 or 16
    int ept() const {
        const int need = (2 * h->ns_max + NT - 1) / NT;
        return need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 16;
    }

    // the fused Arnoldi step covers every slab and the restart length
    bool fused() const {
        return h->ns_max <= NTF && h->ws_restart < MR && h->fs != RT_FS_DELO_PARABOLIC;
    }

    // sweep of A P^-1 v_j, then the Arnoldi step (fused or not)
    void arnoldi_step(const VecArgs &a, int j, bool fp32) {
        const double *vj = h->d_V + (long long)j * h->n_unk;
        if (fused()) {
            if (tri) {
                ok(precond_tri(h, vj, h->d_pz, h->d_cycle, s));
                ok(apply_sweep(h, h->d_pz, nullptr, h->d_cycle, fp32, s));
            } else {
                ok(apply_sweep(h, vj, h->d_dinv, h->d_cycle, fp32, s));
            }
            VecArgs af = a;
            af.part_f32 = fp32 ? 1 : 0;  // the sweep's partial sums are in its precision
            if (j < 16)
                hipLaunchKernelGGL(gm_arnoldi_fused_kernel<16>, dim3(h->n_atm), dim3(NTF), 0, s, af, j);
            else
                hipLaunchKernelGGL(gm_arnoldi_fused_kernel<MR>, dim3(h->n_atm), dim3(NTF), 0, s, af, j);
            ok(hipGetLastError());
        } else {
            prec_sweep(vj, h->d_w, h->d_cycle, fp32);
            arnoldi(a, j);
        }
    }

    void arnoldi(const VecArgs &a, int j) {
        const dim3 g(h->n_atm), b(NT);
        switch (ept()) {
            case 2: hipLaunchKernelGGL(gm_arnoldi_kernel<2>, g, b, 0, s, a, j); break;
            case 4: hipLaunchKernelGGL(gm_arnoldi_kernel<4>, g, b, 0, s, a, j); break;
            case 8: hipLaunchKernelGGL(gm_arnoldi_kernel<8>, g, b, 0, s, a, j); break;
            default: hipLaunchKernelGGL(gm_arnoldi_kernel<16>, g, b, 0, s, a, j); break;
        }
        ok(hipGetLastError());
    }

    void update(const VecArgs &a) {
        const dim3 g(h->n_atm), b(NT);
        switch (ept()) {
            case 2: hipLaunchKernelGGL(gm_update_kernel<2>, g, b, 0, s, a); break;
            case 4: hipLaunchKernelGGL(gm_update_kernel<4>, g, b, 0, s, a); break;
            case 8: hipLaunchKernelGGL(gm_update_kernel<8>, g, b, 0, s, a); break;
            default: hipLaunchKernelGGL(gm_update_kernel<16>, g, b, 0, s, a); break;
        }
        ok(hipGetLastError());
    }

    int count(const int *flags) {
        hipLaunchKernelGGL(count_kernel, dim3(1), dim3(NT), 0, s, flags, h->n_atm, h->d_count);
        ok(hipGetLastError());
        ok(hipMemcpyAsync(h->h_count, h->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
        ok(hipStreamSynchronize(s));
        return err == hipSuccess ? *h->h_count : 0;
    }

    void init_state(KState *st, const int *from_mask) {
        hipLaunchKernelGGL(init_state_kernel, dim3((h->n_atm + 255) / 256), dim3(256), 0, s, st,
                           h->d_active, h->d_cycle, h->n_atm, from_mask);
        ok(hipGetLastError());
    }

    VecArgs args(const double *b, double *x, KState *st, int *active, double tol, int maxit) {
        VecArgs a{};
        a.atm = h->d_atm;
        a.N = h->n_unk;
        a.m = h->ws_restart;
        a.V = h->d_V;
        a.H = h->d_H;
        a.cs = h->d_cs;
        a.sn = h->d_sn;
        a.g = h->d_g;
        a.w = h->d_w;
        a.b = b;
        a.x = x;
        a.dinv = tri ? h->d_ones : h->d_dinv;
        a.zin = tri ? h->d_pz : nullptr;
        a.r = h->d_r;
        a.rh = h->d_rh;
        a.p = h->d_p;
        a.v = h->d_v;
        a.s = h->d_s;
        a.t = h->d_t;
        a.q = h->d_cq;
        a.u = h->d_w;
        a.st = st;
        a.active = active;
        a.cycle = h->d_cycle;
        a.tol = tol;
        a.maxit = maxit;
        a.max_outer = h->opt.max_outer;
        a.partial = h->d_partial;
        a.Qs = h->d_Qs;
        a.outer = outer;
        return a;
    }

    // Restarted GMRES on the slabs flagged in d_active.  st must be
    // initialized; x_zero: x is zero on entry (skip the first A x).
    void gmres(const double *b, double *x, KState *st, double tol, int maxit, bool fp32,
               bool x_zero, bool accept_est = false) {
        const int nb = h->n_atm;
        VecArgs a = args(b, x, st, h->d_active, tol, maxit);
        const int m = h->ws_restart;
        const int check = std::max(1, h->opt.check_every);
        if (!x_zero) iter_sweep(x, h->d_w, h->d_active, fp32);
        hipLaunchKernelGGL(gm_restart_kernel, dim3(nb), dim3(NT), 0, s, a, 1, x_zero ? 1 : 0,
                           accept_est ? 1 : 0);
        ok(hipGetLastError());
        // one cycle: m Arnoldi steps (masked off per slab once its cycle
        // ends), the update of x, and the restart with the explicit residual
        auto tail = [&]() {
            update(a);
            iter_sweep(x, h->d_w, h->d_active, fp32);
            hipLaunchKernelGGL(gm_restart_kernel, dim3(nb), dim3(NT), 0, s, a, 0, 0,
                               accept_est ? 1 : 0);
            ok(hipGetLastError());
        };
        // the last entry is the block plan the cycle was captured with
        std::vector<unsigned long long> key = {
            0, bits(b), bits(x), bits(st), bits(tol), (unsigned long long)maxit, fp32 ? 1ull : 0ull,
            accept_est ? 1ull : 0ull, bits(outer), 0};
        while (err == hipSuccess) {
            const int act = count(h->d_active);
            if (act == 0) break;
            // a cycle that starts with few slabs still iterating sweeps with
            // the tail plan; the choice is made here only, so eager launches
            // and graph replays take the same plan in every cycle
            h->plan_tail = h->n_blocks_tail > 0 && act <= kTailSlabs;
            a.atm = plan_atm(h);
            key.back() = h->plan_tail ? 1 : 0;
            if (h->opt.graphs) {
                graph(key, [&]() {
                    for (int j = 0; j < m; ++j) arnoldi_step(a, j, fp32);
                    tail();
                });
            } else {
                for (int j = 0; j < m; ++j) {
                    arnoldi_step(a, j, fp32);
                    if ((j + 1) % check == 0 && j + 1 < m && count(h->d_cycle) == 0) break;
                }
                tail();
            }
        }
        h->plan_tail = false;
    }

    void bicgstab(const double *b, double *x, KState *st, double tol, int maxit) {
        const int nb = h->n_atm;
        VecArgs a = args(b, x, st, h->d_active, tol, maxit);
        const int check = std::max(1, h->opt.check_every);
        iter_sweep(x, h->d_w, h->d_active, false);
        hipLaunchKernelGGL(bi_start_kernel, dim3(nb), dim3(NT), 0, s, a);
        ok(hipGetLastError());
        auto step = [&]() {
            hipLaunchKernelGGL(bi_dir_kernel, dim3(nb), dim3(NT), 0, s, a);
            prec_sweep(h->d_p, h->d_v, h->d_active, false);
            hipLaunchKernelGGL(bi_half_kernel, dim3(nb), dim3(NT), 0, s, a);
            prec_sweep(h->d_s, h->d_t, h->d_active, false);
            hipLaunchKernelGGL(bi_full_kernel, dim3(nb), dim3(NT), 0, s, a);
            ok(hipGetLastError());
        };
        const std::vector<unsigned long long> key = {1,         bits(b),   bits(x),
                                                     bits(st),  bits(tol), (unsigned long long)maxit,
                                                     (unsigned long long)check};
        while (err == hipSuccess) {
            if (count(h->d_active) == 0) break;
            if (h->opt.graphs) {
                graph(key, [&]() {
                    for (int i = 0; i < check; ++i) step();
                });
            } else {
                for (int i = 0; i < check; ++i) step();
            }
        }
        // explicit final residual of every slab
        iter_sweep(x, h->d_w, nullptr, false);
        hipLaunchKernelGGL(relres_kernel, dim3(nb), dim3(NT), 0, s, a);
        ok(hipGetLastError());
    }

    void cgs(const double *b, double *x, KState *st, double tol, int maxit) {
        const int nb = h->n_atm;
        VecArgs a = args(b, x, st, h->d_active, tol, maxit);
        const int check = std::max(1, h->opt.check_every);
        iter_sweep(x, h->d_w, h->d_active, false);
        hipLaunchKernelGGL(cg_start_kernel, dim3(nb), dim3(NT), 0, s, a);
        ok(hipGetLastError());
        auto step = [&]() {
            hipLaunchKernelGGL(cg_dir_kernel, dim3(nb), dim3(NT), 0, s, a);
            prec_sweep(h->d_p, h->d_v, h->d_active, false);
            hipLaunchKernelGGL(cg_half_kernel, dim3(nb), dim3(NT), 0, s, a);
            prec_sweep(h->d_s, h->d_t, h->d_active, false);
            hipLaunchKernelGGL(cg_full_kernel, dim3(nb), dim3(NT), 0, s, a);
            ok(hipGetLastError());
        };
        const std::vector<unsigned long long> key = {3,         bits(b),   bits(x),
                                                     bits(st),  bits(tol), (unsigned long long)maxit,
                                                     (unsigned long long)check};
        while (err == hipSuccess) {
            if (count(h->d_active) == 0) break;
            if (h->opt.graphs) {
                graph(key, [&]() {
                    for (int i = 0; i < check; ++i) step();
                });
            } else {
                for (int i = 0; i < check; ++i) step();
            }
        }
        // explicit final residual of every slab
        iter_sweep(x, h->d_w, nullptr, false);
        hipLaunchKernelGGL(relres_kernel, dim3(nb), dim3(NT), 0, s, a);
        ok(hipGetLastError());
    }

    void richardson(const double *b, double *x, KState *st, double tol, int maxit) {
        const int nb = h->n_atm;
        VecArgs a = args(b, x, st, h->d_active, tol, maxit);
        const int check = std::max(1, h->opt.check_every);
        auto step = [&](int first) {
            iter_sweep(x, h->d_w, h->d_active, false);
            hipLaunchKernelGGL(ri_step_kernel, dim3(nb), dim3(NT), 0, s, a, first);
            ok(hipGetLastError());
        };
        const std::vector<unsigned long long> key = {2,         bits(b),   bits(x),
                                                     bits(st),  bits(tol), (unsigned long long)maxit,
                                                     (unsigned long long)check};
        // the first check_every updates (the first one sets up the state) eagerly
        for (int i = 0; i < check && err == hipSuccess; ++i) step(i == 0 ? 1 : 0);
        while (err == hipSuccess) {
            if (count(h->d_active) == 0) break;
            if (h->opt.graphs) {
                graph(key, [&]() {
                    for (int i = 0; i < check; ++i) step(0);
                });
            } else {
                for (int i = 0; i < check; ++i) step(0);
            }
        }
    }

    // FP64 iterative refinement around FP32-sweep GMRES solves of A d = r.
    void mixed_gmres(const double *b, double *x, KState *st, KState *st_in) {
        const int nb = h->n_atm;
        // outer flags live in d_cycle's companion: keep them in d_active of the
        // outer loop, and give the inner solve its own copy in the count buffer
        int *outer_active = h->d_active + h->n_atm;  // second half of the flag buffer
        VecArgs a = args(b, x, st, outer_active, h->opt.rtol, h->opt.maxit);
        hipLaunchKernelGGL(init_state_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, st,
                           outer_active, h->d_cycle, nb, (const int *)nullptr);
        ok(hipGetLastError());
        for (int k = 0; err == hipSuccess; ++k) {
            iter_sweep(x, h->d_w, outer_active, false);
            hipLaunchKernelGGL(ir_residual_kernel, dim3(nb), dim3(NT), 0, s, a, k == 0 ? 1 : 0);
            ok(hipGetLastError());
            if (count(outer_active) == 0) break;
            // inner: A32 d = r, d = 0 initially, on the slabs still refining
            init_state(st_in, outer_active);
            outer = st;
            gmres(h->d_r, h->d_s, st_in, h->opt.inner_rtol, h->opt.inner_maxit, true, true, true);
            outer = nullptr;
            hipLaunchKernelGGL(ir_update_kernel, dim3(nb), dim3(NT), 0, s, a, (const KState *)st_in);
            ok(hipGetLastError());
        }
    }
};

}  // namespace

// Allocate the Krylov workspace for the handle's restart length.
int ensure_workspace(rt_handle *h);

// A handful of deep slabs (the single 1024-point atmosphere): the batched
// solver's Arnoldi step runs one workgroup per slab, which leaves the chip
// idle and serializes the slab's basis reads on one CU; the segmented GMRES
// (rt_fieldsolve.hip) spreads every slab's vectors over many workgroups.
static bool few_deep_slabs(const rt_handle *h) { return h->n_atm <= 4 && 2 * h->ns_max >= 2048; }

int run_solver(rt_handle *h, int kind, const double *b, double *x, rt_solve_info *info,
               hipStream_t s) {
    if (kind == 0 && h->opt.precond == RT_PC_JACOBI && h->fs != RT_FS_DELO_PARABOLIC &&
        few_deep_slabs(h)) {
        const double *bb = b ? b : h->d_b;
        auto op64 = [&](const double *in, const double *scale, double *out) {
            return apply_operator(h, in, scale, out, nullptr, false, 0, s);
        };
        auto op32 = [&](const double *in, const double *scale, double *out) {
            return apply_operator(h, in, scale, out, nullptr, true, 0, s);
        };
        auto own = [&](double *bo) {
            return hipMemcpyAsync(bo, h->d_b, sizeof(double) * h->n_unk, hipMemcpyDeviceToDevice, s);
        };
        if (h->opt.precision == RT_PREC_MIXED)
            return solve_seg_refined(h, op64, op32, 2, bb, own, x, h->d_dinv, info, s);
        return solve_seg_gmres(h, op64, 2, bb, own, x, h->d_dinv, info, s);
    }
    int rc = ensure_workspace(h);
    if (rc != RT_OK) return rc;
    if (!b) b = h->d_b;
    Driver d{h, s};
    KState *st = h->d_state;
    KState *st_in = h->d_state + h->n_atm;
    if (kind == 4) {
        // direct: LU of the assembled A, then the explicit FP64 residual
        if ((rc = lu_factor(h, s)) != RT_OK) return rc;
        d.ok(lu_solve(h, b, x, s));
        d.init_state(st, nullptr);
        d.sweep(x, nullptr, h->d_w, nullptr, false);
        const VecArgs a = d.args(b, x, st, h->d_active, 0.0, 0);
        hipLaunchKernelGGL(relres_kernel, dim3(h->n_atm), dim3(NT), 0, s, a);
        hipLaunchKernelGGL(direct_status_kernel, dim3((h->n_atm + 255) / 256), dim3(256), 0, s,
                           st, (const int *)h->d_sing, h->n_atm);
        d.ok(hipGetLastError());
    }
    d.tri = kind != 4 && h->opt.precond != RT_PC_JACOBI;
    if (d.tri) {
        // the assembled A, P^-1 workspace and unit scaling; then y0 = P x0
        if ((rc = ensure_dense(h, s)) != RT_OK) return rc;
        if (!h->d_pz) {
            // both or neither (a later call must not find d_pz without d_ones)
            if (hipMalloc((void **)&h->d_pz, sizeof(double) * h->n_unk) != hipSuccess ||
                hipMalloc((void **)&h->d_ones, sizeof(double) * h->n_unk) != hipSuccess) {
                (void)hipGetLastError();
                for (double **p : {&h->d_pz, &h->d_ones}) {
                    if (*p) (void)hipFree(*p);
                    *p = nullptr;
                }
                return fail(RT_ENOMEM, "preconditioner workspace allocation failed");
            }
            d.ok(fill(h->d_ones, h->n_unk, 1.0, s));
        }
        d.ok(precond_tri_mult(h, x, h->d_pz, s));
        d.ok(hipMemcpyAsync(x, h->d_pz, sizeof(double) * h->n_unk, hipMemcpyDeviceToDevice, s));
    }
    if (kind == 4) {
        // solved above
    } else if (kind == 0 && h->opt.precision == RT_PREC_MIXED) {
        d.mixed_gmres(b, x, st, st_in);
    } else {
        d.init_state(st, nullptr);
        if (kind == 0)
            d.gmres(b, x, st, h->opt.rtol, h->opt.maxit, false, false);
        else if (kind == 1)
            d.bicgstab(b, x, st, h->opt.rtol, h->opt.maxit);
        else if (kind == 3)
            d.cgs(b, x, st, h->opt.rtol, h->opt.maxit);
        else
            d.richardson(b, x, st, h->opt.rtol, h->opt.maxit);
    }
    if (d.tri) {  // x = P^-1 y
        d.ok(precond_tri(h, x, h->d_pz, nullptr, s));
        d.ok(hipMemcpyAsync(x, h->d_pz, sizeof(double) * h->n_unk, hipMemcpyDeviceToDevice, s));
    }
    std::vector<KState> hs(h->n_atm);
    d.ok(hipMemcpyAsync(hs.data(), st, sizeof(KState) * h->n_atm, hipMemcpyDeviceToHost, s));
    d.ok(hipStreamSynchronize(s));
    if (d.err != hipSuccess)
        return fail(RT_EDEVICE, std::string("solver: ") + hipGetErrorString(d.err));
    int worst = RT_OK;
    for (int i = 0; i < h->n_atm; ++i) {
        const KState &k = hs[i];
        if (k.status > worst) worst = k.status;
        if (info) {
            info[i].status = k.status;
            info[i].iterations = k.iters;
            info[i].matvecs = k.matvecs;
            info[i].outer_steps = k.outer;
            info[i].relres = (kind == 0 && h->opt.precision != RT_PREC_MIXED && k.bnorm > 0.0)
                                 ? k.beta / k.bnorm
                                 : k.relres;
        }
    }
    if (worst != RT_OK)
        set_error(worst == RT_ENOCONV ? "solver did not reach rtol within the iteration limit"
                                      : "solver breakdown");
    return worst;
}

}  // namespace rt
