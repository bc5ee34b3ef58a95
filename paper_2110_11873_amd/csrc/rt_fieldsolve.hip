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

constexpr int kFsNT = 256;
constexpr int kFsChunk = 1024;  // vector entries per workgroup
constexpr int kFsPerThread = kFsChunk / kFsNT;
constexpr int kFsPerLane = kFsChunk / kWave;

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

// w -= sum_i h[s][i] V_i over the working slabs' segments; the column of H
// accumulates h (first pass: set, second: add).
__global__ __launch_bounds__(kFsNT) void fs_axpy_kernel(FsArgs a, double *w, int nv, int j,
                                                         int first) {
    const int s = blockIdx.y;
    if (!working(a, s)) return;
    const double *hs = a.h + (long long)s * (a.m + 1);
    const long long lo = a.off[s] + (long long)blockIdx.x * kFsChunk;
    const long long hi = std::min(a.off[s + 1], lo + kFsChunk);
    double v[kFsPerThread];
#pragma unroll
    for (int u = 0; u < kFsPerThread; ++u) {
        const long long e = lo + threadIdx.x + (long long)u * kFsNT;
        v[u] = e < hi ? w[e] : 0.0;
    }
    for (int i = 0; i < nv; ++i) {
        const double c = -hs[i];
        const double *Vi = a.V + (long long)i * a.N;
#pragma unroll
        for (int u = 0; u < kFsPerThread; ++u) {
            const long long e = lo + threadIdx.x + (long long)u * kFsNT;
            if (e < hi) v[u] = fma(c, Vi[e], v[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < kFsPerThread; ++u) {
        const long long e = lo + threadIdx.x + (long long)u * kFsNT;
        if (e < hi) w[e] = v[u];
    }
    if (blockIdx.x == 0 && threadIdx.x < nv) {
        double *Hc = a.H + (long long)s * (a.m + 1) * a.m + (long long)threadIdx.x * a.m + j;
        *Hc = first ? hs[threadIdx.x] : *Hc + hs[threadIdx.x];
    }
}

// Step j's last part, one thread per slab: h_{j+1,j} = ||w|| (in h[s][0]),
// previous rotations on column j, the new rotation, g, the residual
// estimate; v_{j+1} = w / h_{j+1,j} is left to fs_scale_kernel.
__global__ void fs_givens_kernel(FsArgs a, int j) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_atm || !working(a, s)) return;
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

// End of a cycle, one thread per active slab: y = H^-1 g (back substitution
// over the cycle's steps), into h.
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
int solve_seg_gmres(rt_handle *h, const std::function<hipError_t(const double *, double *)> &op,
                    long long per, const double *b_in,
                    const std::function<hipError_t(double *)> &own_rhs, double *x,
                    const double *dinv, rt_solve_info *info, hipStream_t st) {
    return solve_seg_gmres_tol(h, op, per, b_in, own_rhs, x, dinv, h->opt.rtol, h->opt.maxit, info,
                               st);
}

int solve_seg_gmres_tol(rt_handle *h, const std::function<hipError_t(const double *, double *)> &op,
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
    // workspace, released at the end of the call
    std::vector<void *> bufs;
    auto get = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        bufs.push_back(p);
        return p;
    };
    auto release = [&]() {
        for (void *p : bufs) (void)hipFree(p);
    };
    FsArgs a{};
    a.n_atm = n_atm;
    a.nchunk = nchunk;
    a.m = m;
    a.N = N;
    a.tol = rtol;
    a.maxit = maxit;
    a.off = (long long *)get(sizeof(long long) * (n_atm + 1));
    a.V = (double *)get(sizeof(double) * (size_t)(m + 1) * N);
    double *w = (double *)get(sizeof(double) * N);
    double *bown = b ? nullptr : (double *)get(sizeof(double) * N);
    double *tmp = dinv ? (double *)get(sizeof(double) * N) : nullptr;
    a.part = (double *)get(sizeof(double) * (size_t)n_atm * nchunk * (m + 1));
    a.h = (double *)get(sizeof(double) * (size_t)n_atm * (m + 1));
    a.H = (double *)get(sizeof(double) * (size_t)n_atm * (m + 1) * m);
    a.cs = (double *)get(sizeof(double) * (size_t)n_atm * m);
    a.sn = (double *)get(sizeof(double) * (size_t)n_atm * m);
    a.g = (double *)get(sizeof(double) * (size_t)n_atm * (m + 1));
    a.bnorm = (double *)get(sizeof(double) * n_atm);
    a.beta = (double *)get(sizeof(double) * n_atm);
    a.resid = (double *)get(sizeof(double) * n_atm);
    a.active = (int *)get(sizeof(int) * n_atm);
    a.done = (int *)get(sizeof(int) * n_atm);
    a.jj = (int *)get(sizeof(int) * n_atm);
    a.iters = (int *)get(sizeof(int) * n_atm);
    for (void *p : bufs)
        if (!p) {
            release();
            return fail(RT_ENOMEM, "GMRES workspace allocation failed");
        }
    if (!a.off || !a.V || !w || (!b && !bown) || (dinv && !tmp) || !a.part || !a.h || !a.H || !a.cs || !a.sn ||
        !a.g || !a.bnorm || !a.beta || !a.resid || !a.active || !a.done || !a.jj || !a.iters) {
        release();
        return fail(RT_ENOMEM, "GMRES workspace allocation failed");
    }
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
    // the preconditioned operator A diag(dinv), on y = x ./ dinv
    auto apply = [&](const double *v, double *out) {
        if (!dinv) return op(v, out);
        hipLaunchKernelGGL(fs_mul_kernel, dim3(mgrid), dim3(256), 0, st, dinv, v, tmp, N, 0);
        hipError_t e = hipGetLastError();
        return e != hipSuccess ? e : op(tmp, out);
    };
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
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(fs_dots_kernel, seg, blk, 0, st, a, (const double *)w, j + 1,
                                   (const double *)a.V, 0);
                hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a, j + 1, 0);
                hipLaunchKernelGGL(fs_axpy_kernel, seg, blk, 0, st, a, w, j + 1, j,
                                   pass == 0 ? 1 : 0);
            }
            hipLaunchKernelGGL(fs_dots_kernel, seg, blk, 0, st, a, (const double *)w, 1,
                               (const double *)nullptr, 0);
            hipLaunchKernelGGL(fs_reduce_kernel, dim3(n_atm), dim3(1024), 0, st, a, 1, 0);
            hipLaunchKernelGGL(fs_givens_kernel, dim3(tg), dim3(tb), 0, st, a, j);
            hipLaunchKernelGGL(fs_scale_kernel, seg, blk, 0, st, a, (const double *)w, j);
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
        hipLaunchKernelGGL(fs_backsolve_kernel, dim3(tg), dim3(tb), 0, st, a);
        hipLaunchKernelGGL(fs_update_kernel, seg, blk, 0, st, a, x);
    }
    // back to x = dinv .* y, then the final explicit residuals b - A x
    if (dinv) hipLaunchKernelGGL(fs_mul_kernel, dim3(mgrid), dim3(256), 0, st, dinv, (const double *)x, x, N, 0);
    ok(op(x, w));
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

int solve_seg_refined(rt_handle *h, const std::function<hipError_t(const double *, double *)> &op,
                      const std::function<hipError_t(const double *, double *)> &op_lo,
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
    std::vector<void *> bufs;
    auto get = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        bufs.push_back(p);
        return p;
    };
    auto release = [&]() {
        for (void *p : bufs) (void)hipFree(p);
    };
    // per-slab squared norms through the segmented reductions (m = 0: one row)
    FsArgs a{};
    a.n_atm = n_atm;
    a.nchunk = nchunk;
    a.m = 0;
    a.N = N;
    a.off = (long long *)get(sizeof(long long) * (n_atm + 1));
    a.part = (double *)get(sizeof(double) * (size_t)n_atm * nchunk);
    a.h = (double *)get(sizeof(double) * n_atm);
    a.active = (int *)get(sizeof(int) * n_atm);
    double *bown = b_in ? nullptr : (double *)get(sizeof(double) * N);
    double *r = (double *)get(sizeof(double) * N);
    double *d = (double *)get(sizeof(double) * N);
    double *w = (double *)get(sizeof(double) * N);
    if (!a.off || !a.part || !a.h || !a.active || (!b_in && !bown) || !r || !d || !w) {
        release();
        return fail(RT_ENOMEM, "refinement workspace allocation failed");
    }
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
        ok(op(x, w));
        ++napply;
        hipLaunchKernelGGL(fs_axpby_kernel, dim3(mgrid), dim3(256), 0, st, b, (const double *)w, r,
                           N);
        norms(r, rn);
        done = true;
        for (int s = 0; s < n_atm; ++s)
            if (!(bn[s] == 0.0 || rn[s] < rtol * bn[s])) done = false;
        if (done || err != hipSuccess || total >= h->opt.maxit) break;
        // d from the cheaper operator, from zero; slabs already converged
        // carry a tiny r and change x by a tiny d
        ok(fill(d, N, 0.0, st));
        std::vector<rt_solve_info> in(n_atm);
        const int rc = solve_seg_gmres_tol(h, op_lo, per, r, own_rhs, d, dinv, h->opt.inner_rtol,
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
        h, [&](const double *in, double *out) { return apply_field_operator(h, in, out, st); },
        2LL * h->n_mu * h->n_nu, b, [&](double *bo) { return field_rhs(h, bo, st); }, x, nullptr,
        info, st);
}

}  // namespace rt
