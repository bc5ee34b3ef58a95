// rt_fieldsolve.hip -- GMRES(m) (Sect. 2.1) for the long-vector systems: the
// field-unknown system (Id - Lambda T J) I = Lambda T c + t (eq.
// crd_linear_system2) and the frequency-redistribution variant.
//
// The slabs are independent, so each slab's segment of the field vector is
// its own system with its own basis rows, Hessenberg matrix, Givens
// rotations and test ||b - K I|| / ||b|| < rtol, all kept on the device; the
// slabs advance in lock step and a converged slab stops updating.  Classical
// Gram-Schmidt applied twice with the second pass delayed by one step, so
// that one reduction per step serves both passes (DCGS2: Swirydowicz,
// Langou, Ananthan, Yang and Thomas, 2020), with segmented reductions: each
// workgroup sums a chunk of one slab's segment for all basis rows at once,
// and a second pass adds the chunks in a fixed order (deterministic).  No
// preconditioner:
// the field system is the one Sect. 3.2 calls more favourable to Krylov
// methods.  The redistribution variant uses the same solver with its own
// operator and a Jacobi scaling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <string>
#include <vector>

#include "rt_internal.h"

namespace rt {

namespace {

constexpr int kFsNT = 1024;  // 16 wavefronts per chunk: its basis rows spread over them
constexpr int kFsChunk = 1024;  // vector entries per workgroup
constexpr int kFsPerThread = kFsChunk / kFsNT;
constexpr int kFsPerLane = kFsChunk / kWave;
constexpr int kFsFuseMaxChunks = 256;  // more chunks: the partial sums are added once, apart

// Workspace carved from one device allocation that the handle keeps between
// calls (slot 0: the GMRES, 1: the refinement around it) and grows when a
// call needs more; every piece starts on a 256-byte boundary.
class Carve {
  public:
    Carve(rt_handle *h, int slot) : h_(h), slot_(slot) {}
    template <typename T>
    void want(T **p, size_t count) {
        *p = nullptr;
        reqs_.push_back({(void **)p, (count ? count : 1) * sizeof(T)});
    }
    bool commit() {
        size_t total = 0;
        for (const Req &r : reqs_) total += round(r.bytes);
        void *&base = h_->seg_ws[slot_];
        size_t &have = h_->seg_ws_bytes[slot_];
        if (have < total) {
            if (base) (void)hipFree(base);
            base = nullptr;
            have = 0;
            if (hipMalloc(&base, total) != hipSuccess) {
                (void)hipGetLastError();
                base = nullptr;
                return false;
            }
            have = total;
        }
        char *q = static_cast<char *>(base);
        for (const Req &r : reqs_) {
            *r.p = q;
            q += round(r.bytes);
        }
        return true;
    }

  private:
    struct Req {
        void **p;
        size_t bytes;
    };
    static size_t round(size_t b) { return (b + 255) / 256 * 256; }
    rt_handle *h_;
    int slot_;
    std::vector<Req> reqs_;
};

struct FsArgs {
    const long long *off;  // [n_atm + 1] first entry of each slab's segment
    int n_atm, nchunk, m;
    long long N;           // field length (row stride of V)
    int hs;                // entries per (slab, chunk) of part and per slab of h
    double *V;             // (m + 1) x N basis
    double *part;          // [n_atm][nchunk][hs] partial sums
    double *h;             // [n_atm][hs] sums / coefficients
    double *H;             // [n_atm][m + 1][m] Hessenberg columns, rotated (the triangle)
    double *Hu;            // [n_atm][m + 1][m] the same columns before the rotations
    double *hc;            // [2][n_atm][m + 1] a step's column before its second pass
    double *cs, *sn, *g;   // [n_atm][m], [n_atm][m], [n_atm][m + 1]
    double *bnorm, *beta, *resid;  // [n_atm]
    int *active, *done;    // [n_atm]: still iterating; current cycle finished
    int *jj;               // [n_atm]: Arnoldi steps of the current cycle
    int *iters;            // [n_atm]
    double tol;
    int maxit;
};

__device__ inline bool working(const FsArgs &a, int s) { return a.active[s] && !a.done[s]; }

// out = 1 when some slab's flag is set
__global__ __launch_bounds__(256) void fs_any_kernel(const int *flags, int n, int *out) {
    int any = 0;
    for (int s = threadIdx.x; s < n; s += blockDim.x) any |= flags[s] ? 1 : 0;
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) *out = any;
}

// out = 1 when no slab is still in its cycle (every slab done or inactive)
__global__ __launch_bounds__(256) void fs_ended_kernel(FsArgs a, int *out) {
    int in_cycle = 0;
    for (int s = threadIdx.x; s < a.n_atm; s += blockDim.x) in_cycle |= working(a, s) ? 1 : 0;
    in_cycle = __syncthreads_or(in_cycle);
    if (threadIdx.x == 0) *out = in_cycle ? 0 : 1;
}

// part[s][c][0] = sum over chunk c of slab s of x[e]^2, for the active slabs:
// each wavefront adds its lanes' strided entries, then a butterfly and one
// pass over the 16 wavefronts in LDS (a fixed order).
__global__ __launch_bounds__(kFsNT) void fs_norm2_kernel(FsArgs a, const double *x) {
    __shared__ double red[kFsNT / kWave];
    const int s = blockIdx.y, c = blockIdx.x;
    if (!a.active[s]) return;
    const long long lo = a.off[s] + (long long)c * kFsChunk;
    const long long hi = std::min(a.off[s + 1], lo + kFsChunk);
    double acc = 0.0;
    for (long long e = lo + threadIdx.x; e < hi; e += kFsNT) acc = fma(x[e], x[e], acc);
    for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kFsNT / kWave; ++w) t += red[w];
        a.part[((long long)s * a.nchunk + c) * a.hs] = t;
    }
}

// h[s][i] = sum over the chunks of part[s][c][i]: one wavefront per row i,
// lane l adding chunks l, l + 64, ... in order, then a butterfly (a fixed
// order for a given chunk count: deterministic).
__global__ __launch_bounds__(1024) void fs_reduce_kernel(FsArgs a, int nv, int mode) {
    __shared__ double red[1024];
    const int s = blockIdx.x;
    if (!(mode ? a.active[s] : working(a, s))) return;
    // G groups of nv threads (G a power of two): group g adds chunks g, g + G,
    // ... of entry i, so neighbouring threads read neighbouring entries of a
    // chunk's row; the groups' sums are then added pairwise in a fixed tree
    int G = 1;
    while (2 * G * nv <= (int)blockDim.x) G *= 2;
    const int t = threadIdx.x, i = t % nv, g = t / nv;
    const double *ps = a.part + (long long)s * a.nchunk * a.hs;
    if (g < G) {
        double acc = 0.0;
#pragma unroll 8
        for (int c = g; c < a.nchunk; c += G) acc += ps[(long long)c * a.hs + i];
        red[t] = acc;
    }
    __syncthreads();
    for (int half = G / 2; half > 0; half /= 2) {
        if (g < half) red[t] += red[t + half * nv];
        __syncthreads();
    }
    if (t < nv) a.h[(long long)s * a.hs + t] = red[t];
}

// ---------------------------------------------------------------------------
// One Arnoldi step in two launches after the operator.  Step j holds the
// finished rows q_0..q_{j-1} and u = V_j, the candidate projected once
// against them (q_0 = r / beta is finished at the start of a cycle), and w =
// A u.  One reduction gives, for i < j, s_i = q_i.u (the candidate's second
// pass, delayed) and z_i = q_i.w, and nu = u.u, zeta = u.w; then
//   rho = sqrt(nu - |s|^2),  q_j = (u - sum s_i q_i) / rho,
//   c_i = z_i / rho (i < j),  c_j = (zeta - s.z) / rho^2,
//   u_{j+1} = w / rho - sum_{i <= j} c_i q_i     (the first pass of A q_j),
// column j-1 of the Hessenberg matrix is finished (its first-pass
// coefficients plus s, subdiagonal rho) and rotated, and column j's first
// pass is c - (H s) / rho, H with the finished column j-1 (A q_j = (w -
// A Q s) / rho and A Q = Q H).  The convergence test of column j-1 thus comes
// one step late; the last column of a cycle is finished by a reduction
// without an operator application.
//   fs_dd_dots_kernel:   the partial dot products on each chunk;
//   fs_dd_update_kernel: every workgroup of a slab adds all chunks' partial
//                        sums itself (in one order: the same coefficients,
//                        bit for bit, in every workgroup),
//                        then updates q_j and u_{j+1} on its chunk; the first
//                        workgroup finishes column j-1 and runs the Givens
//                        step.  (From kFsFuseMaxChunks chunks on,
//                        fs_reduce_kernel adds them once into h first.)
// ---------------------------------------------------------------------------

// the Givens part of step j for slab s (below)
__device__ void givens_step(const FsArgs &a, int s, int j, const double *col,
                            const double *rcs, const double *rsn);

// sum over the chunks of one slab's partial sums of entry i, by one wavefront
// (the same order in every workgroup)
__device__ inline double chunk_sum(const FsArgs &a, const double *ps, int i, int lane) {
    double t = 0.0;
    for (int c = lane; c < a.nchunk; c += kWave) t += ps[(long long)c * a.hs + i];
    for (int o = kWave / 2; o > 0; o >>= 1) t += __shfl_xor(t, o);
    return t;
}

// part[2i] = V_i.u, part[2i+1] = V_i.w (i < j); part[2j] = u.u, part[2j+1] =
// u.w, with u = V_j; w = NULL (the end of a cycle): the u products only.
__global__ __launch_bounds__(kFsNT) void fs_dd_dots_kernel(FsArgs a, const double *w, int j) {
    const int s = blockIdx.y, c = blockIdx.x;
    if (!working(a, s)) return;
    const long long lo = a.off[s] + (long long)c * kFsChunk;
    const long long hi = std::min(a.off[s + 1], lo + kFsChunk);
    const int lane = threadIdx.x % kWave;
    const double *u = a.V + (long long)j * a.N;
    // the chunk of u and w, read once for all wavefronts (each wavefront
    // reading it into registers made every workgroup fetch it 16 times)
    __shared__ double su[kFsChunk], sw[kFsChunk];
    for (int t = threadIdx.x; t < kFsChunk; t += kFsNT) {
        const long long e = lo + t;
        su[t] = e < hi ? u[e] : 0.0;
        sw[t] = (w && e < hi) ? w[e] : 0.0;
    }
    __syncthreads();
    double *out = a.part + ((long long)s * a.nchunk + c) * a.hs;
    for (int i = threadIdx.x / kWave; i <= j; i += kFsNT / kWave) {
        const double *Vi = a.V + (long long)i * a.N;  // i == j: u itself
        double as = 0.0, az = 0.0;
#pragma unroll
        for (int k = 0; k < kFsPerLane; ++k) {
            const int t = lane + k * kWave;
            const long long e = lo + t;
            const double vi = e < hi ? Vi[e] : 0.0;
            as = fma(vi, su[t], as);
            az = fma(vi, sw[t], az);
        }
        for (int o = kWave / 2; o > 0; o >>= 1) {
            as += __shfl_xor(as, o);
            az += __shfl_xor(az, o);
        }
        if (lane == 0) {
            out[2 * i] = as;
            out[2 * i + 1] = az;
        }
    }
}

// summed: the sums are in h (fs_reduce_kernel); flush: the end of a cycle
// (j = m): finish column m-1 only.
__global__ __launch_bounds__(kFsNT) void fs_dd_update_kernel(FsArgs a, const double *w, int j,
                                                              int flush, int summed) {
    __shared__ double sv[2 * (RT_MAX_RESTART + 1)];  // s_i, z_i interleaved; nu, zeta
    __shared__ double cf[RT_MAX_RESTART + 1];        // c
    __shared__ double col[RT_MAX_RESTART + 1];       // the finished column j-1
    __shared__ double rcs[RT_MAX_RESTART], rsn[RT_MAX_RESTART];  // earlier rotations
    __shared__ double srho, ssz;
    const int s = blockIdx.y, c = blockIdx.x;
    if (!working(a, s)) return;
    const int m = a.m, lane = threadIdx.x % kWave, nval = 2 * j + 2;
    if (summed) {
        for (int i = threadIdx.x; i < nval; i += kFsNT) sv[i] = a.h[(long long)s * a.hs + i];
    } else {
        const double *ps = a.part + (long long)s * a.nchunk * a.hs;
        for (int i = threadIdx.x / kWave; i < nval; i += kFsNT / kWave) {
            const double t = chunk_sum(a, ps, i, lane);
            if (lane == 0) sv[i] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < kWave) {  // |s|^2 and s.z by the first wavefront
        double ss = 0.0, sz = 0.0;
        for (int i = lane; i < j; i += kWave) {
            ss = fma(sv[2 * i], sv[2 * i], ss);
            sz = fma(sv[2 * i], sv[2 * i + 1], sz);
        }
        for (int o = kWave / 2; o > 0; o >>= 1) {
            ss += __shfl_xor(ss, o);
            sz += __shfl_xor(sz, o);
        }
        if (lane == 0) {
            srho = j > 0 ? sqrt(fmax(sv[2 * j] - ss, 0.0)) : 1.0;  // q_0 is finished
            ssz = sz;
        }
    }
    __syncthreads();
    const double rho = srho;
    if (!flush && rho > 0.0) {
        for (int i = threadIdx.x; i < j; i += kFsNT) cf[i] = sv[2 * i + 1] / rho;
        if (threadIdx.x == 0) cf[j] = (sv[2 * j + 1] - ssz) / (rho * rho);
    }
    if (j > 0 && threadIdx.x <= j) {
        const double *hp = a.hc + ((long long)((j - 1) & 1) * a.n_atm + s) * (m + 1);
        col[threadIdx.x] = threadIdx.x < j ? hp[threadIdx.x] + sv[2 * threadIdx.x] : rho;
    }
    __syncthreads();
    if (c == 0) {
        // the first workgroup: column j-1 kept as it is and rotated (the
        // earlier rotations read into LDS, applied by one thread in
        // registers), and column j before its second pass
        const int jc = j - 1;
        if (j > 0) {
            for (int i = threadIdx.x; i < jc; i += kFsNT) {
                rcs[i] = a.cs[(long long)s * m + i];
                rsn[i] = a.sn[(long long)s * m + i];
            }
            if (threadIdx.x <= j)
                a.Hu[((long long)s * (m + 1) + threadIdx.x) * m + jc] = col[threadIdx.x];
        }
        __syncthreads();
        if (j > 0 && threadIdx.x == 0) givens_step(a, s, jc, col, rcs, rsn);
        if (!flush && rho > 0.0) {
            // row i: c_i - (H s)_i / rho, one wavefront per row
            const double *Hs = a.Hu + (long long)s * (m + 1) * m;
            for (int i = threadIdx.x / kWave; i <= j; i += kFsNT / kWave) {
                double t = 0.0;
                if (j > 0) {
                    for (int l = (i > 0 ? i - 1 : 0) + lane; l < j - 1; l += kWave)
                        t = fma(Hs[(long long)i * m + l], sv[2 * l], t);
                    for (int o = kWave / 2; o > 0; o >>= 1) t += __shfl_xor(t, o);
                    t = fma(col[i], sv[2 * (j - 1)], t);
                }
                if (lane == 0)
                    a.hc[((long long)(j & 1) * a.n_atm + s) * (m + 1) + i] = cf[i] - t / rho;
            }
        }
    }
    if (flush || !(rho > 0.0)) return;
    const long long lo = a.off[s] + (long long)c * kFsChunk;
    const long long hi = std::min(a.off[s + 1], lo + kFsChunk);
    double *Vj = a.V + (long long)j * a.N, *Vn = a.V + (long long)(j + 1) * a.N;
#pragma unroll
    for (int k = 0; k < kFsPerThread; ++k) {
        const long long e = lo + threadIdx.x + (long long)k * kFsNT;
        if (e >= hi) continue;
        double q = Vj[e], nw = w[e] / rho;
#pragma unroll 4
        for (int i = 0; i < j; ++i) {
            const double vi = a.V[(long long)i * a.N + e];
            q = fma(-sv[2 * i], vi, q);
            nw = fma(-cf[i], vi, nw);
        }
        if (j > 0) {
            q /= rho;
            Vj[e] = q;
        }
        Vn[e] = fma(-cf[j], q, nw);
    }
}

// Column j's last part for slab s (one thread): col[0..j+1] is the column as
// computed, (rcs, rsn)[0..j-1] the earlier rotations.  They are applied, the
// new rotation is formed, the rotated column goes to H and g, the residual
// estimate and the convergence test are updated.
__device__ void givens_step(const FsArgs &a, int s, int j, const double *col, const double *rcs,
                            const double *rsn) {
    const int m = a.m;
    double *H = a.H + (long long)s * (m + 1) * m;
    double *g = a.g + (long long)s * (m + 1);
    double x = col[0];
    for (int i = 0; i < j; ++i) {
        const double y = col[i + 1];
        H[(long long)i * m + j] = rcs[i] * x + rsn[i] * y;
        x = -rsn[i] * x + rcs[i] * y;
    }
    const double hn = col[j + 1];
    const double den = sqrt(x * x + hn * hn);
    const double cj = den > 0.0 ? x / den : 1.0, sj = den > 0.0 ? hn / den : 0.0;
    a.cs[(long long)s * m + j] = cj;
    a.sn[(long long)s * m + j] = sj;
    H[(long long)j * m + j] = den;
    H[(long long)(j + 1) * m + j] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sj * gj;
    g[j] = cj * gj;
    a.resid[s] = fabs(g[j + 1]);
    a.jj[s] = j + 1;
    a.iters[s] += 1;
    if (a.resid[s] < a.tol * a.bnorm[s] || hn == 0.0 || j + 1 == m || a.iters[s] >= a.maxit)
        a.done[s] = 1;
}

// v_0 = r / beta (beta in h[s][1]) at the start of a cycle.
__global__ __launch_bounds__(kFsNT) void fs_scale_kernel(FsArgs a) {
    const int s = blockIdx.y;
    if (!a.active[s]) return;
    const double beta = a.h[(long long)s * a.hs + 1];
    if (!(beta > 0.0)) return;
    const long long lo = a.off[s] + (long long)blockIdx.x * kFsChunk;
    const long long hi = std::min(a.off[s + 1], lo + kFsChunk);
    for (long long e = lo + threadIdx.x; e < hi; e += kFsNT) a.V[e] = a.V[e] / beta;
}

// End of a cycle, one wavefront per active slab (restart below 64): y = H^-1 g
// over the cycle's n steps, into h.  The n x n triangle goes to LDS first;
// lane r holds row r's right-hand side, and for i = n-1 down to 0 the solved
// y_i (from lane i) is removed from every row above it at once.
constexpr int kBacksolveMaxM = kWave - 1;  // lanes 0..m write y_0..y_m
__global__ __launch_bounds__(kWave) void fs_backsolve_wave_kernel(FsArgs a) {
    extern __shared__ double Hs[];  // [n][n]
    const int s = blockIdx.x;
    if (!a.active[s]) return;
    const int m = a.m, n = a.jj[s], r = threadIdx.x;
    const double *H = a.H + (long long)s * (m + 1) * m;
    for (int e = r; e < n * n; e += kWave) Hs[e] = H[(long long)(e / n) * m + e % n];
    double t = r < n ? a.g[(long long)s * (m + 1) + r] : 0.0;
    __syncthreads();
    double yr = 0.0;
    for (int i = n - 1; i >= 0; --i) {
        const double yi = __shfl(t / Hs[i * n + i], i);
        if (r == i) yr = yi;
        if (r < i) t = fma(-Hs[r * n + i], yi, t);
    }
    if (r <= m) a.h[(long long)s * a.hs + r] = r < n ? yr : 0.0;
}

// The same for any restart, one thread per active slab, from global memory.
__global__ void fs_backsolve_kernel(FsArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_atm || !a.active[s]) return;
    const int m = a.m, n = a.jj[s];
    const double *H = a.H + (long long)s * (m + 1) * m;
    const double *g = a.g + (long long)s * (m + 1);
    double *y = a.h + (long long)s * a.hs;
    for (int i = n - 1; i >= 0; --i) {
        double t = g[i];
        for (int l = i + 1; l < n; ++l) t -= H[(long long)i * m + l] * y[l];
        y[i] = t / H[(long long)i * m + i];
    }
    for (int i = n; i <= m; ++i) y[i] = 0.0;
}

// x += sum_i y_i V_i over the active slabs.
__global__ __launch_bounds__(kFsNT) void fs_update_kernel(FsArgs a, double *x) {
    const int s = blockIdx.y;
    if (!a.active[s]) return;
    const double *y = a.h + (long long)s * a.hs;
    const int n = a.jj[s];
    const long long lo = a.off[s] + (long long)blockIdx.x * kFsChunk;
    const long long hi = std::min(a.off[s + 1], lo + kFsChunk);
    double v[kFsPerThread];
#pragma unroll
    for (int u = 0; u < kFsPerThread; ++u) {
        const long long e = lo + threadIdx.x + (long long)u * kFsNT;
        v[u] = e < hi ? x[e] : 0.0;
    }
#pragma unroll 4
    for (int i = 0; i < n; ++i) {
        const double *Vi = a.V + (long long)i * a.N;
#pragma unroll
        for (int u = 0; u < kFsPerThread; ++u) {
            const long long e = lo + threadIdx.x + (long long)u * kFsNT;
            if (e < hi) v[u] = fma(y[i], Vi[e], v[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < kFsPerThread; ++u) {
        const long long e = lo + threadIdx.x + (long long)u * kFsNT;
        if (e < hi) x[e] = v[u];
    }
}

// r = b - w into V_0 over the active slabs.
__global__ __launch_bounds__(kFsNT) void fs_residual_kernel(FsArgs a, const double *b,
                                                             const double *w) {
    const int s = blockIdx.y;
    if (!a.active[s]) return;
    const long long lo = a.off[s] + (long long)blockIdx.x * kFsChunk;
    const long long hi = std::min(a.off[s + 1], lo + kFsChunk);
    for (long long e = lo + threadIdx.x; e < hi; e += kFsNT) a.V[e] = b[e] - w[e];
}

// Restart test, one thread per slab: beta = ||r|| (in h[s][0]); converged
// slabs leave; the others get g = [beta, 0, ...] and a fresh cycle.  first:
// also records ||b|| (in resid) and starts the iteration counts.
__global__ void fs_restart_kernel(FsArgs a, int first, int maxit) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_atm || !a.active[s]) return;
    const double beta = sqrt(a.h[(long long)s * a.hs]);
    if (first) {
        a.bnorm[s] = sqrt(a.resid[s]);
        a.iters[s] = 0;
    }
    a.beta[s] = beta;
    a.jj[s] = 0;
    a.done[s] = 0;
    if (!(beta >= a.tol * a.bnorm[s]) || a.bnorm[s] == 0.0 || a.iters[s] >= maxit) {
        a.active[s] = 0;
        return;
    }
    double *g = a.g + (long long)s * (a.m + 1);
    g[0] = beta;
    for (int i = 1; i <= a.m; ++i) g[i] = 0.0;
    a.h[(long long)s * a.hs + 1] = beta;  // v_0 = r / beta
}

__global__ void fs_init_kernel(FsArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_atm) return;
    a.active[s] = 1;
    a.done[s] = 0;
    a.jj[s] = 0;
}

// ||b|| of each slab, kept in resid until the first restart.
__global__ void fs_keep_bnorm_kernel(FsArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_atm) return;
    a.resid[s] = a.h[(long long)s * a.hs];
}

// out = d .* in (mode 0), in ./ d (1) or out + in (2) over the whole vector
// (the Jacobi scaling of the generic solve; the refinement update).
__global__ void fs_mul_kernel(const double *d, const double *in, double *out, long long n,
                              int mode) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        out[e] = mode == 2 ? out[e] + in[e] : mode == 1 ? in[e] / d[e] : d[e] * in[e];
}

// r = b - w over the whole vector.
__global__ void fs_axpby_kernel(const double *b, const double *w, double *r, long long n) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        r[e] = b[e] - w[e];
}

}  // namespace

// GMRES(restart) for a block-diagonal operator whose slab s owns `per`
// entries per depth point; dinv (optional) preconditions from the right by
// diag(dinv): the solve runs on y with x = dinv .* y, starting from y0 =
// x0 ./ dinv, so that the residual tested is still b - A x.
int solve_seg_gmres(rt_handle *h, const SegOp &op,
                    long long per, const double *b_in,
                    const std::function<hipError_t(double *)> &own_rhs, double *x,
                    const double *dinv, rt_solve_info *info, hipStream_t st) {
    return solve_seg_gmres_tol(h, op, per, b_in, own_rhs, x, dinv, h->opt.rtol, h->opt.maxit, info,
                               st);
}

int solve_seg_gmres_tol(rt_handle *h, const SegOp &op,
                        long long per, const double *b_in,
                        const std::function<hipError_t(double *)> &own_rhs, double *x,
                        const double *dinv, double rtol, int maxit, rt_solve_info *info,
                        hipStream_t st) {
    const int m = h->opt.restart, n_atm = h->n_atm;
    const long long N = per * h->ns_total;
    const double *b = b_in;
    std::vector<long long> off(n_atm + 1, 0);
    int nchunk = 1;
    for (int s = 0; s < n_atm; ++s) {
        off[s + 1] = off[s] + per * h->ns[s];
        nchunk = std::max<int>(nchunk, (int)((per * h->ns[s] + kFsChunk - 1) / kFsChunk));
    }
    // workspace, kept by the handle for later calls
    FsArgs a{};
    a.n_atm = n_atm;
    a.nchunk = nchunk;
    a.m = m;
    a.N = N;
    a.tol = rtol;
    a.maxit = maxit;
    a.hs = 2 * (m + 1);
    double *w, *bown = nullptr;
    Carve cv(h, 0);
    cv.want((long long **)&a.off, n_atm + 1);
    cv.want(&a.V, (size_t)(m + 1) * N);
    cv.want(&w, N);
    if (!b) cv.want(&bown, N);
    cv.want(&a.part, (size_t)n_atm * nchunk * a.hs);
    cv.want(&a.h, (size_t)n_atm * a.hs);
    cv.want(&a.H, (size_t)n_atm * (m + 1) * m);
    cv.want(&a.Hu, (size_t)n_atm * (m + 1) * m);
    cv.want(&a.hc, (size_t)2 * n_atm * (m + 1));
    cv.want(&a.cs, (size_t)n_atm * m);
    cv.want(&a.sn, (size_t)n_atm * m);
    cv.want(&a.g, (size_t)n_atm * (m + 1));
    cv.want(&a.bnorm, n_atm);
    cv.want(&a.beta, n_atm);
    cv.want(&a.resid, n_atm);
    cv.want(&a.active, n_atm);
    cv.want(&a.done, n_atm);
    cv.want(&a.jj, n_atm);
    cv.want(&a.iters, n_atm);
    int *dflag;
    cv.want(&dflag, 1);
    if (!cv.commit()) return fail(RT_ENOMEM, "GMRES workspace allocation failed");
    if (!h->h_seg_flag && hipHostMalloc((void **)&h->h_seg_flag, sizeof(int)) != hipSuccess) {
        h->h_seg_flag = nullptr;
        return fail(RT_ENOMEM, "pinned host allocation failed");
    }
    volatile int *hflag = h->h_seg_flag;
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        return fail(RT_EDEVICE, "GMRES: event creation failed");
    auto release = [&] { (void)hipEventDestroy(ev); };
    hipError_t err = hipSuccess;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && err == hipSuccess) err = e;
        return err == hipSuccess;
    };
    ok(hipMemcpyAsync((void *)a.off, off.data(), sizeof(long long) * (n_atm + 1),
                      hipMemcpyHostToDevice, st));
    if (!b) {
        ok(own_rhs(bown));
        b = bown;
    }
    const int mgrid = (int)std::min<long long>((N + 255) / 256, 4096);
    // the preconditioned operator A diag(dinv), on y = x ./ dinv (the scaling
    // is done by the operator's kernels as they read v)
    auto apply = [&](const double *v, double *out) { return op(v, dinv, out); };
    if (dinv) hipLaunchKernelGGL(fs_mul_kernel, dim3(mgrid), dim3(256), 0, st, dinv, (const double *)x, x, N, 1);
    const dim3 seg(nchunk, n_atm), blk(kFsNT);
    const int tb = 64, tg = (n_atm + tb - 1) / tb;
    // whether any slab's flag is set: one int through pinned memory
    auto any_active = [&](const int *flags) {
        hipLaunchKernelGGL(fs_any_kernel, dim3(1), dim3(256), 0, st, flags, n_atm, dflag);
        ok(hipMemcpyAsync((void *)hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
        ok(hipStreamSynchronize(st));
        return err == hipSuccess && *hflag != 0;
    };
    hipLaunchKernelGGL(fs_init_kernel, dim3(tg), dim3(tb), 0, st, a);
    // ||b||, then r = b - K x
    hipLaunchKernelGGL(fs_norm2_kernel, seg, blk, 0, st, a, b);
    hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a, 1, 1);
    hipLaunchKernelGGL(fs_keep_bnorm_kernel, dim3(tg), dim3(tb), 0, st, a);
    bool first = true;
    int napply = 0;
    while (ok(hipGetLastError())) {
        ok(apply(x, w));
        ++napply;
        hipLaunchKernelGGL(fs_residual_kernel, seg, blk, 0, st, a, b, (const double *)w);
        hipLaunchKernelGGL(fs_norm2_kernel, seg, blk, 0, st, a, (const double *)a.V);
        hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a, 1, 1);
        hipLaunchKernelGGL(fs_restart_kernel, dim3(tg), dim3(tb), 0, st, a, first ? 1 : 0, maxit);
        first = false;
        if (!any_active(a.active)) break;
        // v_0 = r / beta (h[s][1] holds beta)
        hipLaunchKernelGGL(fs_scale_kernel, seg, blk, 0, st, a);
        // one reduction and one update per step (fs_dd_*), with the sums
        // added once apart from many chunks on
        const bool apart = nchunk > kFsFuseMaxChunks;
        auto reduce_update = [&](const double *wv, int j, int flush) {
            hipLaunchKernelGGL(fs_dd_dots_kernel, seg, blk, 0, st, a, wv, j);
            if (apart)
                hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a, 2 * j + 2,
                                   0);
            hipLaunchKernelGGL(fs_dd_update_kernel, seg, blk, 0, st, a, wv, j, flush,
                               apart ? 1 : 0);
            ok(hipGetLastError());
        };
        // Stop the cycle early once every slab's cycle has ended.  Every 8
        // steps the end flag is copied to pinned memory behind an event that
        // the following steps poll, so the host never drains the stream; a
        // host that reaches the next check first waits for that event, which
        // keeps it at most two checks ahead.  Steps run after the cycle ended
        // and before the flag is seen change nothing (their kernels skip
        // slabs out of their cycle).
        bool ended = false;  // every slab's cycle ended before step m
        bool pending = false;
        for (int j = 0; j < m && err == hipSuccess; ++j) {
            ok(apply(a.V + (long long)j * N, w));
            ++napply;
            reduce_update(w, j, 0);
            if (pending) {
                const hipError_t q = hipEventQuery(ev);
                if (q == hipSuccess) {
                    pending = false;
                    if (*hflag) {
                        ended = true;
                        break;
                    }
                } else if (q == hipErrorNotReady) {
                    (void)hipGetLastError();  // the copy is still running: no error
                } else {
                    ok(q);
                }
            }
            if ((j + 1) % 8 == 0 && j + 1 < m) {
                if (pending) {
                    // the host is a full check ahead: wait for the last one
                    // (the GPU still has the 8 steps since it queued)
                    ok(hipEventSynchronize(ev));
                    pending = false;
                    if (err == hipSuccess && *hflag) {
                        ended = true;
                        break;
                    }
                }
                hipLaunchKernelGGL(fs_ended_kernel, dim3(1), dim3(256), 0, st, a, dflag);
                ok(hipMemcpyAsync((void *)hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
                ok(hipEventRecord(ev, st));
                pending = true;
            }
        }
        // the last column of the cycle, for the slabs still in it
        if (!ended) reduce_update(nullptr, m, 1);
        if (m <= kBacksolveMaxM)
            hipLaunchKernelGGL(fs_backsolve_wave_kernel, dim3(n_atm), dim3(kWave),
                               sizeof(double) * m * m, st, a);
        else
            hipLaunchKernelGGL(fs_backsolve_kernel, dim3(tg), dim3(tb), 0, st, a);
        hipLaunchKernelGGL(fs_update_kernel, seg, blk, 0, st, a, x);
    }
    // back to x = dinv .* y, then the final explicit residuals b - A x
    if (dinv) hipLaunchKernelGGL(fs_mul_kernel, dim3(mgrid), dim3(256), 0, st, dinv, (const double *)x, x, N, 0);
    ok(op(x, nullptr, w));
    hipLaunchKernelGGL(fs_init_kernel, dim3(tg), dim3(tb), 0, st, a);
    hipLaunchKernelGGL(fs_residual_kernel, seg, blk, 0, st, a, b, (const double *)w);
    hipLaunchKernelGGL(fs_norm2_kernel, seg, blk, 0, st, a, (const double *)a.V);
    hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a, 1, 1);
    std::vector<double> hh((size_t)n_atm * a.hs), bn(n_atm);
    std::vector<int> its(n_atm);
    ok(hipMemcpyAsync(hh.data(), a.h, sizeof(double) * hh.size(), hipMemcpyDeviceToHost, st));
    ok(hipMemcpyAsync(bn.data(), a.bnorm, sizeof(double) * n_atm, hipMemcpyDeviceToHost, st));
    ok(hipMemcpyAsync(its.data(), a.iters, sizeof(int) * n_atm, hipMemcpyDeviceToHost, st));
    ok(hipStreamSynchronize(st));
    release();
    if (err != hipSuccess) return fail(RT_EDEVICE, std::string("GMRES: ") + hipGetErrorString(err));
    int worst = RT_OK;
    for (int s = 0; s < n_atm; ++s) {
        const double rel = bn[s] > 0.0 ? std::sqrt(hh[(size_t)s * a.hs]) / bn[s] : 0.0;
        const int status = rel < rtol ? RT_OK : RT_ENOCONV;
        worst = std::max(worst, status);
        if (info) {
            info[s].status = status;
            info[s].iterations = its[s];
            info[s].matvecs = napply + 1;  // the batch's applications, this slab's at most
            info[s].outer_steps = 0;
            info[s].relres = rel;
        }
    }
    if (worst != RT_OK) set_error("GMRES did not reach rtol within the iteration limit");
    return worst;
}

int solve_seg_refined(rt_handle *h, const SegOp &op, const SegOp &op_lo,
                      long long per, const double *b_in,
                      const std::function<hipError_t(double *)> &own_rhs, double *x,
                      const double *dinv, rt_solve_info *info, hipStream_t st) {
    const int n_atm = h->n_atm;
    const long long N = per * h->ns_total;
    std::vector<long long> off(n_atm + 1, 0);
    int nchunk = 1;
    for (int s = 0; s < n_atm; ++s) {
        off[s + 1] = off[s] + per * h->ns[s];
        nchunk = std::max<int>(nchunk, (int)((per * h->ns[s] + kFsChunk - 1) / kFsChunk));
    }
    // per-slab squared norms through the segmented reductions (m = 0: one row);
    // workspace kept by the handle for later calls
    FsArgs a{};
    a.n_atm = n_atm;
    a.nchunk = nchunk;
    a.m = 0;
    a.hs = 1;
    a.N = N;
    double *bown = nullptr, *r, *d, *w;
    Carve cv(h, 1);
    cv.want((long long **)&a.off, n_atm + 1);
    cv.want(&a.part, (size_t)n_atm * nchunk);
    cv.want(&a.h, n_atm);
    cv.want(&a.active, n_atm);
    if (!b_in) cv.want(&bown, N);
    cv.want(&r, N);
    cv.want(&d, N);
    cv.want(&w, N);
    if (!cv.commit()) return fail(RT_ENOMEM, "refinement workspace allocation failed");
    auto release = [] {};
    hipError_t err = hipSuccess;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && err == hipSuccess) err = e;
        return err == hipSuccess;
    };
    const std::vector<int> ones(n_atm, 1);
    ok(hipMemcpyAsync((void *)a.off, off.data(), sizeof(long long) * (n_atm + 1),
                      hipMemcpyHostToDevice, st));
    ok(hipMemcpyAsync(a.active, ones.data(), sizeof(int) * n_atm, hipMemcpyHostToDevice, st));
    const double *b = b_in;
    if (!b) {
        ok(own_rhs(bown));
        b = bown;
    }
    const dim3 seg(nchunk, n_atm), blk(kFsNT);
    const int mgrid = (int)std::min<long long>((N + 255) / 256, 4096);
    auto norms = [&](const double *v, std::vector<double> &out) {
        hipLaunchKernelGGL(fs_norm2_kernel, seg, blk, 0, st, a, v);
        hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a, 1, 1);
        ok(hipGetLastError());
        out.resize(n_atm);
        ok(hipMemcpyAsync(out.data(), a.h, sizeof(double) * n_atm, hipMemcpyDeviceToHost, st));
        ok(hipStreamSynchronize(st));
        for (double &v2 : out) v2 = std::sqrt(v2);
    };
    std::vector<double> bn, rn;
    norms(b, bn);
    std::vector<int> its(n_atm, 0);
    const double rtol = h->opt.rtol;
    int outer = 0, napply = 0, total = 0;
    bool done = false;
    while (err == hipSuccess) {
        // r = b - A x (FP64)
        ok(op(x, nullptr, w));
        ++napply;
        hipLaunchKernelGGL(fs_axpby_kernel, dim3(mgrid), dim3(256), 0, st, b, (const double *)w, r,
                           N);
        norms(r, rn);
        done = true;
        for (int s = 0; s < n_atm; ++s)
            if (!(bn[s] == 0.0 || rn[s] < rtol * bn[s])) done = false;
        if (done || err != hipSuccess || total >= h->opt.maxit) break;
        // d from the cheaper operator, from zero; slabs already converged
        // carry a tiny r and change x by a tiny d.  One tolerance for all
        // slabs: the tightest that the slabs still refining need
        double tol_in = 1.0;
        for (int s = 0; s < n_atm; ++s)
            if (bn[s] > 0.0 && !(rn[s] < rtol * bn[s]))
                tol_in = std::min(tol_in, kIrMargin * rtol * bn[s] / rn[s]);
        tol_in = std::max(tol_in, h->opt.inner_rtol);
        ok(fill(d, N, 0.0, st));
        std::vector<rt_solve_info> in(n_atm);
        const int rc = solve_seg_gmres_tol(h, op_lo, per, r, own_rhs, d, dinv, tol_in,
                                           h->opt.inner_maxit, in.data(), st);
        if (rc != RT_OK && rc != RT_ENOCONV) {
            release();
            return rc;
        }
        int most = 0;
        for (int s = 0; s < n_atm; ++s) {
            its[s] += in[s].iterations;
            most = std::max(most, in[s].iterations);
            napply += in[s].matvecs;
        }
        total += std::max(most, 1);  // every step counts toward maxit
        hipLaunchKernelGGL(fs_mul_kernel, dim3(mgrid), dim3(256), 0, st, (const double *)nullptr,
                           (const double *)d, x, N, 2);
        ok(hipGetLastError());
        ++outer;
    }
    release();
    if (err != hipSuccess) return fail(RT_EDEVICE, std::string("refinement: ") + hipGetErrorString(err));
    int worst = RT_OK;
    for (int s = 0; s < n_atm; ++s) {
        const double rel = bn[s] > 0.0 ? rn[s] / bn[s] : 0.0;
        const int status = rel < rtol ? RT_OK : RT_ENOCONV;
        worst = std::max(worst, status);
        if (info) {
            info[s].status = status;
            info[s].iterations = its[s];
            info[s].matvecs = napply;
            info[s].outer_steps = outer;
            info[s].relres = rel;
        }
    }
    if (worst != RT_OK) set_error("refinement did not reach rtol within the iteration limit");
    return worst;
}

int solve_field_gmres(rt_handle *h, const double *b, double *x, rt_solve_info *info,
                      hipStream_t st) {
    return solve_seg_gmres(
        h,
        [&](const double *in, const double *, double *out) {
            return apply_field_operator(h, in, out, st);  // unpreconditioned: no scaling
        },
        2LL * h->n_mu * h->n_nu, b, [&](double *bo) { return field_rhs(h, bo, st); }, x, nullptr,
        info, st);
}

}  // namespace rt
