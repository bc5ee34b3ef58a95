// rt_fieldsolve.hip -- GMRES(m) (Sect. 2.1) for the long-vector systems: the
// field-unknown system (Id - Lambda T J) I = Lambda T c + t (eq.
// crd_linear_system2) and the frequency-redistribution variant.
//
// The slabs are independent, so each slab's segment of the field vector is
// its own system with its own basis rows, Hessenberg matrix, Givens
// rotations and test ||b - K I|| / ||b|| < rtol, all kept on the device; the
// slabs advance in lock step and a converged slab stops updating.  Classical
// Gram-Schmidt applied twice, with segmented reductions: each workgroup sums
// a chunk of one slab's segment for all basis rows at once, and a second
// pass adds the chunks in a fixed order (deterministic).  No preconditioner:
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
    double *V;             // (m + 1) x N basis
    double *part;          // [n_atm][nchunk][m + 1] partial sums
    double *h;             // [n_atm][m + 1] current column / coefficients
    double *H;             // [n_atm][m + 1][m]
    double *cs, *sn, *g;   // [n_atm][m], [n_atm][m], [n_atm][m + 1]
    double *bnorm, *beta, *resid;  // [n_atm]
    int *active, *done;    // [n_atm]: still iterating; current cycle finished
    int *jj;               // [n_atm]: Arnoldi steps of the current cycle
    int *iters;            // [n_atm]
    double tol;
    int maxit;
};

__device__ inline bool working(const FsArgs &a, int s) { return a.active[s] && !a.done[s]; }

// part[s][c][i] = sum over chunk c of slab s of x[e] * V_i[e] (i < nv), or of
// x[e]^2 when V is NULL.  mode 1: all active slabs (restart); 0: working ones.
// Each lane keeps its entries of x in registers and every wavefront reduces
// whole rows (rows w, w + 4, ...) with a butterfly: no LDS, no barrier.
__global__ __launch_bounds__(kFsNT) void fs_dots_kernel(FsArgs a, const double *x, int nv,
                                                         const double *V, int mode) {
    const int s = blockIdx.y, c = blockIdx.x;
    if (!(mode ? a.active[s] : working(a, s))) return;
    const long long lo = a.off[s] + (long long)c * kFsChunk;
    const long long hi = std::min(a.off[s + 1], lo + kFsChunk);
    const int lane = threadIdx.x % kWave;
    double xv[kFsPerLane];
#pragma unroll
    for (int u = 0; u < kFsPerLane; ++u) {
        const long long e = lo + lane + (long long)u * kWave;
        xv[u] = e < hi ? x[e] : 0.0;
    }
    for (int i = threadIdx.x / kWave; i < nv; i += kFsNT / kWave) {
        const double *Vi = V ? V + (long long)i * a.N : x;
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kFsPerLane; ++u) {
            const long long e = lo + lane + (long long)u * kWave;
            acc = fma(xv[u], V ? (e < hi ? Vi[e] : 0.0) : xv[u], acc);
        }
        for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) a.part[((long long)s * a.nchunk + c) * (a.m + 1) + i] = acc;
    }
}

// h[s][i] = sum over the chunks of part[s][c][i]: one wavefront per row i,
// lane l adding chunks l, l + 64, ... in order, then a butterfly (a fixed
// order for a given chunk count: deterministic).
__global__ __launch_bounds__(1024) void fs_reduce_kernel(FsArgs a, int nv, int mode) {
    const int s = blockIdx.x;
    if (!(mode ? a.active[s] : working(a, s))) return;
    const int lane = threadIdx.x % kWave;
    const double *ps = a.part + (long long)s * a.nchunk * (a.m + 1);
    for (int i = threadIdx.x / kWave; i < nv; i += blockDim.x / kWave) {
        double t = 0.0;
        for (int c = lane; c < a.nchunk; c += kWave) t += ps[(long long)c * (a.m + 1) + i];
        for (int o = kWave / 2; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (lane == 0) a.h[(long long)s * (a.m + 1) + i] = t;
    }
}

// ---------------------------------------------------------------------------
// The Arnoldi step fused into three launches after the first pass's partial
// dot products (fs_dots_kernel into part): every workgroup of a slab first
// adds the partial sums of all chunks itself -- in the order fs_reduce_kernel
// uses, so every workgroup gets the same coefficients, bit for bit -- and then
// works on its chunk.
// (With many chunks that redundant sum costs more than a launch: from
// kFsFuseMaxChunks chunks on, fs_reduce_kernel adds them once into h first
// and fs_proj_kernel reads h; the sums are the same, bit for bit.)
//   fs_proj_kernel:   h = sum_c part, w -= sum_i h_i V_i on the chunk, H column
//                     (set or add), then the partial dot products of the new w
//                     with V_i (nv rows) or with itself (nv = 0) into `out`;
//   fs_close_kernel:  hn^2 = sum_c part (the norm), Givens (workgroup 0) and
//                     v_{j+1} = w / hn on the chunk.
// The dot products are taken from a copy of the chunk in LDS in the layout of
// fs_dots_kernel, so they add in the same order as that kernel's.
// ---------------------------------------------------------------------------

// the Givens part of step j for slab s (below)
__device__ void givens_step(const FsArgs &a, int s, int j);

// sum over the chunks of one slab's partial sums of row i (fs_reduce_kernel's
// order), by one wavefront
__device__ inline double chunk_sum(const FsArgs &a, const double *ps, int i, int lane) {
    double t = 0.0;
    for (int c = lane; c < a.nchunk; c += kWave) t += ps[(long long)c * (a.m + 1) + i];
    for (int o = kWave / 2; o > 0; o >>= 1) t += __shfl_xor(t, o);
    return t;
}

// the partial dot products of the chunk held in LDS (xs) with rows V_i,
// i < nv (or of the chunk with itself, nv = 0), as fs_dots_kernel computes them
__device__ inline void chunk_dots(const FsArgs &a, const double *xs, int nv, long long lo,
                                  long long hi, double *out) {
    const int lane = threadIdx.x % kWave;
    double xv[kFsPerLane];
#pragma unroll
    for (int u = 0; u < kFsPerLane; ++u) xv[u] = xs[lane + u * kWave];
    const int rows = nv > 0 ? nv : 1;
    for (int i = threadIdx.x / kWave; i < rows; i += kFsNT / kWave) {
        const double *Vi = a.V + (long long)i * a.N;
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kFsPerLane; ++u) {
            const long long e = lo + lane + (long long)u * kWave;
            acc = fma(xv[u], nv > 0 ? (e < hi ? Vi[e] : 0.0) : xv[u], acc);
        }
        for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) out[i] = acc;
    }
}

__global__ __launch_bounds__(kFsNT) void fs_proj_kernel(FsArgs a, double *w, int nv, int j,
                                                         int first, const double *in,
                                                         double *out, int next_nv) {
    __shared__ double hs[RT_MAX_RESTART + 1];
    __shared__ double xs[kFsChunk];
    const int s = blockIdx.y, c = blockIdx.x;
    if (!working(a, s)) return;
    const int lane = threadIdx.x % kWave;
    if (in) {
        const double *ps = in + (long long)s * a.nchunk * (a.m + 1);
        for (int i = threadIdx.x / kWave; i < nv; i += kFsNT / kWave) {
            const double t = chunk_sum(a, ps, i, lane);
            if (lane == 0) hs[i] = t;
        }
    } else {  // already added by fs_reduce_kernel (the same order)
        for (int i = threadIdx.x; i < nv; i += kFsNT) hs[i] = a.h[(long long)s * (a.m + 1) + i];
    }
    __syncthreads();
    const long long lo = a.off[s] + (long long)c * kFsChunk;
    const long long hi = std::min(a.off[s + 1], lo + kFsChunk);
    double v[kFsPerThread];
#pragma unroll
    for (int u = 0; u < kFsPerThread; ++u) {
        const long long e = lo + threadIdx.x + (long long)u * kFsNT;
        v[u] = e < hi ? w[e] : 0.0;
    }
#pragma unroll 4
    for (int i = 0; i < nv; ++i) {
        const double cf = -hs[i];
        const double *Vi = a.V + (long long)i * a.N;
#pragma unroll
        for (int u = 0; u < kFsPerThread; ++u) {
            const long long e = lo + threadIdx.x + (long long)u * kFsNT;
            if (e < hi) v[u] = fma(cf, Vi[e], v[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < kFsPerThread; ++u) {
        const long long e = lo + threadIdx.x + (long long)u * kFsNT;
        if (e < hi) w[e] = v[u];
        xs[threadIdx.x + u * kFsNT] = v[u];
    }
    if (c == 0 && threadIdx.x < nv) {
        double *Hc = a.H + (long long)s * (a.m + 1) * a.m + (long long)threadIdx.x * a.m + j;
        *Hc = first ? hs[threadIdx.x] : *Hc + hs[threadIdx.x];
    }
    __syncthreads();
    chunk_dots(a, xs, next_nv, lo, hi, out + ((long long)s * a.nchunk + c) * (a.m + 1));
}

__global__ __launch_bounds__(kFsNT) void fs_close_kernel(FsArgs a, const double *w, int j,
                                                          const double *in) {
    __shared__ double shn;
    const int s = blockIdx.y, c = blockIdx.x;
    if (!a.active[s]) return;
    if (a.done[s] && a.jj[s] != j + 1) return;  // finished before this step
    if (threadIdx.x < kWave) {
        const double t = chunk_sum(a, in + (long long)s * a.nchunk * (a.m + 1), 0, threadIdx.x);
        if (threadIdx.x == 0) shn = t;
    }
    __syncthreads();
    const double hn = sqrt(shn);
    if (c == 0 && threadIdx.x == 0) {
        // the rotations of fs_givens_kernel, with h_{j+1,j} = hn
        a.h[(long long)s * (a.m + 1)] = shn;
        givens_step(a, s, j);
    }
    if (!(hn > 0.0)) return;
    const long long lo = a.off[s] + (long long)c * kFsChunk;
    const long long hi = std::min(a.off[s + 1], lo + kFsChunk);
    for (long long e = lo + threadIdx.x; e < hi; e += kFsNT)
        a.V[(long long)(j + 1) * a.N + e] = w[e] / hn;
}

// Step j's last part for slab s: h_{j+1,j} = ||w|| (its square in h[s][0]),
// previous rotations on column j, the new rotation, g, the residual
// estimate; v_{j+1} = w / h_{j+1,j} is left to the caller.
__device__ void givens_step(const FsArgs &a, int s, int j) {
    const int m = a.m;
    double *H = a.H + (long long)s * (m + 1) * m;
    double *cs = a.cs + (long long)s * m, *sn = a.sn + (long long)s * m;
    double *g = a.g + (long long)s * (m + 1);
    const double hn = sqrt(a.h[(long long)s * (m + 1)]);
    H[(long long)(j + 1) * m + j] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * H[(long long)i * m + j] + sn[i] * H[(long long)(i + 1) * m + j];
        H[(long long)(i + 1) * m + j] = -sn[i] * H[(long long)i * m + j] + cs[i] * H[(long long)(i + 1) * m + j];
        H[(long long)i * m + j] = t;
    }
    const double hjj = H[(long long)j * m + j];
    const double den = sqrt(hjj * hjj + hn * hn);
    cs[j] = den > 0.0 ? hjj / den : 1.0;
    sn[j] = den > 0.0 ? hn / den : 0.0;
    H[(long long)j * m + j] = den;
    H[(long long)(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    a.resid[s] = fabs(g[j + 1]);
    a.jj[s] = j + 1;
    a.iters[s] += 1;
    a.h[(long long)s * (m + 1) + 1] = hn;  // for the normalization
    if (a.resid[s] < a.tol * a.bnorm[s] || hn == 0.0 || j + 1 == m || a.iters[s] >= a.maxit)
        a.done[s] = 1;
}

__global__ __launch_bounds__(kFsNT) void fs_scale_kernel(FsArgs a, const double *w, int j) {
    const int s = blockIdx.y;
    if (!a.active[s]) return;
    if (a.done[s] && a.jj[s] != j + 1) return;  // finished before this step
    const double hn = a.h[(long long)s * (a.m + 1) + 1];
    if (!(hn > 0.0)) return;
    const long long lo = a.off[s] + (long long)blockIdx.x * kFsChunk;
    const long long hi = std::min(a.off[s + 1], lo + kFsChunk);
    for (long long e = lo + threadIdx.x; e < hi; e += kFsNT)
        a.V[(long long)(j + 1) * a.N + e] = w[e] / hn;
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
    if (r <= m) a.h[(long long)s * (m + 1) + r] = r < n ? yr : 0.0;
}

// The same for any restart, one thread per active slab, from global memory.
__global__ void fs_backsolve_kernel(FsArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_atm || !a.active[s]) return;
    const int m = a.m, n = a.jj[s];
    const double *H = a.H + (long long)s * (m + 1) * m;
    const double *g = a.g + (long long)s * (m + 1);
    double *y = a.h + (long long)s * (m + 1);
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
    const double *y = a.h + (long long)s * (a.m + 1);
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
    const double beta = sqrt(a.h[(long long)s * (a.m + 1)]);
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
    a.h[(long long)s * (a.m + 1) + 1] = beta;  // v_0 = r / beta
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
    a.resid[s] = a.h[(long long)s * (a.m + 1)];
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
    double *w, *bown = nullptr, *part2;
    Carve cv(h, 0);
    cv.want((long long **)&a.off, n_atm + 1);
    cv.want(&a.V, (size_t)(m + 1) * N);
    cv.want(&w, N);
    if (!b) cv.want(&bown, N);
    cv.want(&a.part, (size_t)n_atm * nchunk * (m + 1));
    cv.want(&part2, (size_t)n_atm * nchunk * (m + 1));
    cv.want(&a.h, (size_t)n_atm * (m + 1));
    cv.want(&a.H, (size_t)n_atm * (m + 1) * m);
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
    if (!cv.commit()) return fail(RT_ENOMEM, "GMRES workspace allocation failed");
    auto release = [] {};
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
    std::vector<int> act(n_atm);
    auto any_active = [&](const int *flags) {
        ok(hipMemcpyAsync(act.data(), flags, sizeof(int) * n_atm, hipMemcpyDeviceToHost, st));
        ok(hipStreamSynchronize(st));
        for (int v : act)
            if (v) return true;
        return false;
    };
    hipLaunchKernelGGL(fs_init_kernel, dim3(tg), dim3(tb), 0, st, a);
    // ||b||, then r = b - K x
    hipLaunchKernelGGL(fs_dots_kernel, seg, blk, 0, st, a, b, 1, (const double *)nullptr, 1);
    hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a, 1, 1);
    hipLaunchKernelGGL(fs_keep_bnorm_kernel, dim3(tg), dim3(tb), 0, st, a);
    bool first = true;
    int napply = 0;
    while (ok(hipGetLastError())) {
        ok(apply(x, w));
        ++napply;
        hipLaunchKernelGGL(fs_residual_kernel, seg, blk, 0, st, a, b, (const double *)w);
        hipLaunchKernelGGL(fs_dots_kernel, seg, blk, 0, st, a, (const double *)a.V, 1,
                           (const double *)nullptr, 1);
        hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a, 1, 1);
        hipLaunchKernelGGL(fs_restart_kernel, dim3(tg), dim3(tb), 0, st, a, first ? 1 : 0, maxit);
        first = false;
        if (!any_active(a.active)) break;
        // v_0 = r / beta (h[s][1] holds beta)
        hipLaunchKernelGGL(fs_scale_kernel, seg, blk, 0, st, a, (const double *)a.V, -1);
        for (int j = 0; j < m && err == hipSuccess; ++j) {
            const double *vj = a.V + (long long)j * N;
            ok(apply(vj, w));
            ++napply;
            // classical Gram-Schmidt twice: first-pass dots; first projection
            // fused with the second-pass dots; second projection fused with
            // the norm's partial sums; Givens and the new basis vector
            hipLaunchKernelGGL(fs_dots_kernel, seg, blk, 0, st, a, (const double *)w, j + 1,
                               (const double *)a.V, 0);
            if (nchunk <= kFsFuseMaxChunks) {
                hipLaunchKernelGGL(fs_proj_kernel, seg, blk, 0, st, a, w, j + 1, j, 1,
                                   (const double *)a.part, part2, j + 1);
                hipLaunchKernelGGL(fs_proj_kernel, seg, blk, 0, st, a, w, j + 1, j, 0,
                                   (const double *)part2, a.part, 0);
            } else {
                FsArgs a2 = a;
                a2.part = part2;
                hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a, j + 1, 0);
                hipLaunchKernelGGL(fs_proj_kernel, seg, blk, 0, st, a, w, j + 1, j, 1,
                                   (const double *)nullptr, part2, j + 1);
                hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a2, j + 1, 0);
                hipLaunchKernelGGL(fs_proj_kernel, seg, blk, 0, st, a, w, j + 1, j, 0,
                                   (const double *)nullptr, a.part, 0);
            }
            hipLaunchKernelGGL(fs_close_kernel, seg, blk, 0, st, a, (const double *)w, j,
                               (const double *)a.part);
            ok(hipGetLastError());
            if ((j + 1) % 8 == 0 && j + 1 < m) {
                // stop the cycle early once every slab's cycle has ended
                std::vector<int> d(n_atm), ac(n_atm);
                ok(hipMemcpyAsync(d.data(), a.done, sizeof(int) * n_atm, hipMemcpyDeviceToHost, st));
                ok(hipMemcpyAsync(ac.data(), a.active, sizeof(int) * n_atm, hipMemcpyDeviceToHost, st));
                ok(hipStreamSynchronize(st));
                bool all = true;
                for (int s = 0; s < n_atm; ++s)
                    if (ac[s] && !d[s]) all = false;
                if (all) break;
            }
        }
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
    hipLaunchKernelGGL(fs_dots_kernel, seg, blk, 0, st, a, (const double *)a.V, 1,
                       (const double *)nullptr, 1);
    hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a, 1, 1);
    std::vector<double> hh((size_t)n_atm * (m + 1)), bn(n_atm);
    std::vector<int> its(n_atm);
    ok(hipMemcpyAsync(hh.data(), a.h, sizeof(double) * hh.size(), hipMemcpyDeviceToHost, st));
    ok(hipMemcpyAsync(bn.data(), a.bnorm, sizeof(double) * n_atm, hipMemcpyDeviceToHost, st));
    ok(hipMemcpyAsync(its.data(), a.iters, sizeof(int) * n_atm, hipMemcpyDeviceToHost, st));
    ok(hipStreamSynchronize(st));
    release();
    if (err != hipSuccess) return fail(RT_EDEVICE, std::string("GMRES: ") + hipGetErrorString(err));
    int worst = RT_OK;
    for (int s = 0; s < n_atm; ++s) {
        const double rel = bn[s] > 0.0 ? std::sqrt(hh[(size_t)s * (m + 1)]) / bn[s] : 0.0;
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
        hipLaunchKernelGGL(fs_dots_kernel, seg, blk, 0, st, a, v, 1, (const double *)nullptr, 1);
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
