// rt_api.hip -- host runtime behind include/rt.h: validation, launch
// planning, device memory, setup kernels, and the C entry points.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "rt_internal.h"

#ifndef RT_SWEEP_SOURCE_HASH
#define RT_SWEEP_SOURCE_HASH "unknown"
#endif

namespace rt {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

hipError_t launch_scale(const double *v, const double *d, double *z, long long n, hipStream_t s);
int run_solver(rt_handle *h, int kind, const double *b, double *x, rt_solve_info *info,
               hipStream_t s);

namespace {

bool finite(double v) { return std::isfinite(v); }

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

std::string idx(const char *name, long long i) {
    return std::string(name) + "[" + std::to_string(i) + "]";
}

// Validation of the problem and options.  Pure host code: no HIP call.
// On success fills the positive half of the symmetric direction set.
int validate(const rt_problem *p, const rt_options *o, std::vector<double> &mu_pos,
             std::vector<double> &w_pos, std::vector<int> *mu_index = nullptr) {
    if (!p) return fail(RT_EINVAL, "problem is NULL");
    if (p->n_atm < 1) return fail(RT_EINVAL, "n_atm must be >= 1");
    if (!p->ns || !p->tau || !p->mu || !p->w_mu || !p->w_nu || !p->phi || !p->opac || !p->eps ||
        !p->W2)
        return fail(RT_EINVAL, "a required problem array is NULL");
    long long total = 0;
    for (int a = 0; a < p->n_atm; ++a) {
        if (p->ns[a] < 2 || p->ns[a] > RT_MAX_NS)
            return fail(RT_EINVAL, idx("ns", a) + " must be in [2, " +
                                       std::to_string(RT_MAX_NS) + "]");
        total += p->ns[a];
    }
    if (total > (1LL << 30)) return fail(RT_EINVAL, "too many depth points");
    long long off = 0;
    for (int a = 0; a < p->n_atm; ++a) {
        for (int k = 0; k < p->ns[a]; ++k) {
            const double t = p->tau[off + k];
            if (!finite(t)) return fail(RT_EINVAL, idx("tau", off + k) + " is not finite");
            if (k > 0 && !(t > p->tau[off + k - 1]))
                return fail(RT_EINVAL, idx("tau", off + k) + " is not strictly increasing");
        }
        off += p->ns[a];
    }
    if (p->n_mu < 2 || p->n_mu % 2 != 0 || p->n_mu > 4096)
        return fail(RT_EINVAL, "n_mu must be even, >= 2");
    double wsum = 0.0;
    for (int m = 0; m < p->n_mu; ++m) {
        if (!finite(p->mu[m]) || p->mu[m] == 0.0 || std::fabs(p->mu[m]) > 1.0)
            return fail(RT_EINVAL, idx("mu", m) + " must be finite, nonzero, |mu| <= 1");
        if (!finite(p->w_mu[m]) || !(p->w_mu[m] > 0.0))
            return fail(RT_EINVAL, idx("w_mu", m) + " must be finite and > 0");
        wsum += p->w_mu[m];
    }
    if (std::fabs(wsum - 2.0) > 1e-10)
        return fail(RT_EINVAL, "w_mu must sum to 2 (quadrature of (1/2) int dmu on [-1,1])");
    std::vector<int> order(p->n_mu);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int i, int j) { return p->mu[i] < p->mu[j]; });
    const int M = p->n_mu / 2;
    mu_pos.assign(M, 0.0);
    w_pos.assign(M, 0.0);
    for (int i = 0; i < M; ++i) {
        const int lo = order[M - 1 - i], hi = order[M + i];
        const double mn = p->mu[lo], mp = p->mu[hi];
        if (!(mp > 0.0) || !(mn < 0.0) || std::fabs(mp + mn) > 1e-12 * std::fabs(mp))
            return fail(RT_EINVAL, "mu must be symmetric: every mu > 0 needs a -mu partner");
        if (std::fabs(p->w_mu[lo] - p->w_mu[hi]) > 1e-12 * p->w_mu[hi])
            return fail(RT_EINVAL, "w_mu must be equal for mu and -mu");
        mu_pos[i] = mp;
        w_pos[i] = p->w_mu[hi];
        if (mu_index) {  // where the pair sits in the caller's mu array
            mu_index->resize(2 * M);
            (*mu_index)[2 * i] = lo;
            (*mu_index)[2 * i + 1] = hi;
        }
    }
    if (p->n_nu < 1 || p->n_nu > (1 << 20)) return fail(RT_EINVAL, "n_nu must be >= 1");
    for (int q = 0; q < p->n_nu; ++q)
        if (!finite(p->w_nu[q]) || p->w_nu[q] < 0.0)
            return fail(RT_EINVAL, idx("w_nu", q) + " must be finite and >= 0");
    for (int a = 0; a < p->n_atm; ++a) {
        double sw = 0.0;
        for (int q = 0; q < p->n_nu; ++q) {
            const long long e = (long long)a * p->n_nu + q;
            if (!finite(p->phi[e]) || p->phi[e] < 0.0)
                return fail(RT_EINVAL, idx("phi", e) + " must be finite and >= 0");
            if (!finite(p->opac[e]) || !(p->opac[e] > 0.0))
                return fail(RT_EINVAL, idx("opac", e) + " must be finite and > 0");
            sw += p->w_nu[q] * p->phi[e];
        }
        if (!(sw > 0.0)) return fail(RT_EINVAL, "sum of w_nu * phi must be > 0 for every slab");
        if (!finite(p->eps[a]) || p->eps[a] < 0.0 || p->eps[a] > 1.0)
            return fail(RT_EINVAL, idx("eps", a) + " must be in [0, 1]");
        if (!finite(p->W2[a])) return fail(RT_EINVAL, idx("W2", a) + " is not finite");
        if (p->I_bot && !finite(p->I_bot[a]))
            return fail(RT_EINVAL, idx("I_bot", a) + " is not finite");
    }
    if (p->B)
        for (long long k = 0; k < total; ++k)
            if (!finite(p->B[k])) return fail(RT_EINVAL, idx("B", k) + " is not finite");
    if (p->formal_solver < RT_FS_DELO_LINEAR || p->formal_solver > RT_FS_DELO_PARABOLIC)
        return fail(RT_EINVAL,
                    "formal_solver must be RT_FS_DELO_LINEAR, RT_FS_TRAPEZOIDAL, "
                    "RT_FS_IMPLICIT_EULER or RT_FS_DELO_PARABOLIC");
    if (o) {
        if (o->precision != RT_PREC_FP64 && o->precision != RT_PREC_MIXED)
            return fail(RT_EINVAL, "options.precision must be RT_PREC_FP64 or RT_PREC_MIXED");
        if (o->restart < 1 || o->restart > RT_MAX_RESTART)
            return fail(RT_EINVAL, "options.restart must be in [1, RT_MAX_RESTART]");
        if (o->maxit < 0) return fail(RT_EINVAL, "options.maxit must be >= 0");
        if (!(o->rtol > 0.0) || !finite(o->rtol)) return fail(RT_EINVAL, "options.rtol must be > 0");
        if (!(o->inner_rtol > 0.0) || !(o->inner_rtol < 1.0))
            return fail(RT_EINVAL, "options.inner_rtol must be in (0, 1)");
        if (o->max_outer < 1) return fail(RT_EINVAL, "options.max_outer must be >= 1");
        if (o->inner_maxit < 1) return fail(RT_EINVAL, "options.inner_maxit must be >= 1");
        if (o->chunk != 0 && !sweep_chunk_supported(o->chunk, false))
            return fail(RT_EINVAL, "options.chunk must be 0, 4, 8, 16 or 32");
        if (o->check_every < 1) return fail(RT_EINVAL, "options.check_every must be >= 1");
        if (o->prefetch < 0 || o->prefetch > 3)
            return fail(RT_EINVAL, "options.prefetch must be in [0, 3]");
        if (o->wave_batches < 0 || o->wave_batches > 64)
            return fail(RT_EINVAL, "options.wave_batches must be in [0, 64]");
        if (o->sweep_waves != 0 && o->sweep_waves != 4 && o->sweep_waves != 8)
            return fail(RT_EINVAL, "options.sweep_waves must be 0, 4 or 8");
        if (o->sweep_waves == 8 && o->chunk > 8)
            return fail(RT_EINVAL, "options.sweep_waves = 8 needs chunk <= 8");
        if (o->graphs != 0 && o->graphs != 1) return fail(RT_EINVAL, "options.graphs must be 0 or 1");
        if (o->precond < RT_PC_JACOBI || o->precond > RT_PC_SSOR)
            return fail(RT_EINVAL, "options.precond must be RT_PC_JACOBI, RT_PC_SOR or RT_PC_SSOR");
        if (!(o->omega > 0.0 && o->omega < 2.0))
            return fail(RT_EINVAL, "options.omega must lie in (0, 2)");
        if (o->coef_mode < RT_COEF_AUTO || o->coef_mode > RT_COEF_RECOMPUTE_FP32)
            return fail(RT_EINVAL, "options.coef_mode must be one of the RT_COEF_* values");
        if (o->autotune != 0 && o->autotune != 1)
            return fail(RT_EINVAL, "options.autotune must be 0 or 1");
    }
    return RT_OK;
}

// ---- stored launch plans (the autotuner's cache, read by rt_setup) --------
// Key of a problem shape: architecture, precision, formal solver, directions,
// frequencies, slabs, deepest slab and a 64-bit FNV-1a hash of the depth
// counts -- the features the sweep's launch plan depends on.
std::string plan_key(const rt_problem *p, int precision, const std::string &arch) {
    unsigned long long f = 0xcbf29ce484222325ULL;
    int ns_max = 0;
    for (int a = 0; a < p->n_atm; ++a) {
        const unsigned int v = (unsigned int)p->ns[a];
        for (int b = 0; b < 4; ++b) {
            f ^= (v >> (8 * b)) & 0xffu;
            f *= 0x100000001b3ULL;
        }
        ns_max = std::max(ns_max, p->ns[a]);
    }
    char hex[17];
    std::snprintf(hex, sizeof hex, "%016llx", f);
    std::ostringstream k;
    k << arch << '|' << (precision == RT_PREC_MIXED ? "mixed" : "fp64") << '|' << p->formal_solver
      << '|' << p->n_mu << '|' << p->n_nu << '|' << p->n_atm << '|' << ns_max << '|' << hex;
    return k.str();
}

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "";
    }
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}

// The plan file: options.plan_file, else $RT_TUNE_PLANS, else
// tuned_plans.txt in the directory of this library.
std::string plan_file_path(const rt_options &o) {
    if (o.plan_file && o.plan_file[0]) return o.plan_file;
    const char *env = std::getenv("RT_TUNE_PLANS");
    if (env && env[0]) return env;
    Dl_info info;
    if (dladdr((void *)&plan_key, &info) && info.dli_fname) {
        std::string lib = info.dli_fname;
        const size_t slash = lib.rfind('/');
        return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) +
               "/tuned_plans.txt";
    }
    return "tuned_plans.txt";
}

// Apply the stored plan for this problem to the options the caller left
// automatic (0).  Returns 0 when none is stored, 1 when the plan was made
// with the sweep sources this library was built from, 2 when with other sources.
int apply_stored_plan(const rt_problem *p, rt_options *o, const std::string &arch) {
    std::ifstream in(plan_file_path(*o));
    if (!in) return 0;
    const std::string key = plan_key(p, o->precision, arch);
    std::string line;
    while (std::getline(in, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream ls(line);
        std::string k, src;
        int chunk, waves, pf, nb, cm;
        if (!(ls >> k >> chunk >> waves >> pf >> nb >> cm >> src) || k != key) continue;
        if (o->chunk == 0) o->chunk = chunk;
        if (o->sweep_waves == 0) o->sweep_waves = waves;
        if (o->prefetch == 0) o->prefetch = pf;
        if (o->wave_batches == 0) o->wave_batches = nb;
        if (o->coef_mode == RT_COEF_AUTO) o->coef_mode = cm;
        return src == RT_SWEEP_SOURCE_HASH ? 1 : 2;
    }
    return 0;
}

// Coefficient modes (kCoef*) of the FP64 and FP32 sweeps for options.coef_mode.
void resolve_coef_modes(int coef_mode, int *cm64, int *cm32) {
    switch (coef_mode) {
        case RT_COEF_PAIRS: *cm64 = *cm32 = kCoefPairs; return;
        case RT_COEF_RECOMPUTE: *cm64 = *cm32 = kCoefRecompute; return;
        case RT_COEF_RECOMPUTE_FP32:
            *cm64 = kCoefW;
            *cm32 = kCoefRecompute;
            return;
        default:  // RT_COEF_STREAM_W and RT_COEF_AUTO
            *cm64 = *cm32 = kCoefW;
    }
}

int chunks_for(int ns, int L) {
    const int x = ns - 1;
    int C = kMinChunks;
    while (C < kWave && C * L < x) C <<= 1;
    return C;
}

// Chunk length: the largest L whose lane count fills the chip (about two
// waves per SIMD) -- longer chunks mean fewer scan steps and partial sums --
// else the shortest, for the most parallelism on small problems.
int auto_chunk(const std::vector<int> &ns, int rays) {
    const long long target = 256LL * 4 * kWave * 2;
    int best = 4;
    for (int L : {4, 8}) {
        bool fits = true;
        long long lanes = 0;
        for (int n : ns) {
            const int C = chunks_for(n, L);
            if ((long long)C * L < n - 1) fits = false;
            lanes += (long long)rays * C;
        }
        if (fits && lanes >= target) best = L;
    }
    // a slab deeper than 64 * best intervals needs longer chunks
    for (int n : ns)
        while (best < 32 && (long long)kWave * best < n - 1) best *= 2;
    return best;
}

// The tile geometry of one slab for a plan of longest chunk L: chunks per
// ray, chunk length, long chunks, rays per wave-batch, wave-batches per
// direction and tile entries per wave-batch.
struct SlabTiles {
    int C, Leff, nlong, G, nwb, bstride;
};
SlabTiles slab_tiles(int ns, int L, int n_nu) {
    SlabTiles t;
    t.C = chunks_for(ns, L);
    t.Leff = chunk_len(ns, t.C, L);
    // chunk lengths Leff and Leff - 1 tile the ns - 1 intervals exactly
    // when Leff is ceil((ns - 1) / C); otherwise (lengths rounded up to
    // a compiled one) all chunks are long and the last ones end past the
    // slab's bottom in identity steps
    t.nlong = t.C;
    if (chunk_len_step(L) == 1) {
        const int r = (ns - 1) - t.C * (t.Leff - 1);
        if (r >= 1 && r <= t.C) t.nlong = r;
    }
    t.G = kWave / t.C;
    t.nwb = (n_nu + t.G - 1) / t.G;
    t.bstride = (t.Leff - 1) * kWave + (t.G * t.nlong + 15) / 16 * 16;
    return t;
}

// The sweep addresses the tiles of one (slab, direction) through 32-bit
// buffer offsets, in entries of up to 16 bytes (FP64 pairs): reject plans
// whose tiles of one direction exceed 2^31 - 1 bytes.
int check_tile_range(const std::vector<int> &ns, int L, int n_nu) {
    for (size_t a = 0; a < ns.size(); ++a) {
        const SlabTiles t = slab_tiles(ns[a], L, n_nu);
        if ((long long)t.nwb * t.bstride * 16 > 2147483647LL)
            return fail(RT_EINVAL, idx("ns", (long long)a) +
                                       ": the coefficient tiles of one direction exceed 2 GiB "
                                       "(too many frequencies for this depth grid)");
    }
    return RT_OK;
}

template <typename T>
int dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return RT_OK;
    if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(RT_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) +
                                   " bytes failed");
    }
    return RT_OK;
}

template <typename T>
int h2d(T *dst, const T *src, size_t count) {
    if (count == 0) return RT_OK;
    if (hipMemcpy(dst, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return fail(RT_EDEVICE, "host to device copy failed");
    return RT_OK;
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return RT_OK;
    return fail(RT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

static SweepArgs sweep_args(rt_handle *h, const double *in, const double *scale, double *out,
                            const int *mask, bool fp32, int mode) {
    SweepArgs a{};
    a.atm = plan_atm(h);
    a.blk = plan_blk(h);
    const int cm = coef_mode_of(h, fp32);
    a.coef = cm == kCoefPairs ? (fp32 ? (const void *)h->d_coef32 : (const void *)h->d_coef64)
                              : (fp32 ? (const void *)h->d_w32 : (const void *)h->d_w64);
    a.q = h->d_qt;
    a.kt = h->d_kt;
    a.dtau = h->d_dtau;
    a.fs = h->fs;
    a.dirc = h->d_dirc;
    a.Qs = h->d_Qs;
    a.sig_in = in;
    a.scale = scale;
    a.sig_out = out;
    a.partial = h->d_partial;
    a.mask = mask;
    a.B = h->d_B;
    a.mode = mode;
    a.part_f32 = fp32 ? 1 : 0;
    return a;
}

hipError_t apply_sweep(rt_handle *h, const double *in, const double *scale, const int *mask,
                       bool fp32, hipStream_t s) {
    const SweepArgs a = sweep_args(h, in, scale, nullptr, mask, fp32, 0);
    int W;
    bool pf;
    sweep_config(h, fp32, &W, &pf);
    return launch_sweep(h->L, W, pf, fp32, coef_mode_of(h, fp32), a, plan_blocks(h), h->ns_max,
                        s);
}

hipError_t apply_operator_into(rt_handle *h, const double *in, double *out, double *partial,
                               hipStream_t s) {
    SweepArgs a = sweep_args(h, in, nullptr, out, nullptr, false, 0);
    a.partial = partial;
    int W;
    bool pf;
    sweep_config(h, false, &W, &pf);
    hipError_t e = launch_sweep(h->L, W, pf, false, coef_mode_of(h, false), a, plan_blocks(h),
                                h->ns_max, s);
    if (e != hipSuccess) return e;
    return launch_finalize(a, h->n_atm, h->ns_max, plan_nblk_max(h), s);
}

hipError_t apply_operator(rt_handle *h, const double *in, const double *scale, double *out,
                          const int *mask, bool fp32, int mode, hipStream_t s) {
    if (h->fs == RT_FS_DELO_PARABOLIC) return apply_ray_operator(h, in, scale, out, mask, mode, s);
    const SweepArgs a = sweep_args(h, in, scale, out, mask, fp32, mode);
    int W;
    bool pf;
    sweep_config(h, fp32, &W, &pf);
    hipError_t e = launch_sweep(h->L, W, pf, fp32, coef_mode_of(h, fp32), a, plan_blocks(h),
                                h->ns_max, s);
    if (e != hipSuccess) return e;
    return launch_finalize(a, h->n_atm, h->ns_max, plan_nblk_max(h), s);
}

void clear_graphs(rt_handle *h) {
    for (auto &g : h->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

int ensure_workspace(rt_handle *h) {
    const int m = h->opt.restart;
    if (h->d_V && h->ws_restart == m) return RT_OK;
    clear_graphs(h);  // captured with the old basis address
    (void)hipFree(h->d_V);
    h->d_V = nullptr;
    const long long N = h->n_unk;
    int rc;
    if ((rc = dalloc(&h->d_V, (size_t)(m + 1) * N)) != RT_OK) return rc;
    if (!h->d_H) {
        // restart-independent buffers, sized for the largest restart; all or
        // none (a failure frees the ones already made, so a later call starts
        // over rather than finding d_H without the rest)
        const int mm = RT_MAX_RESTART;
        void **group[] = {(void **)&h->d_H,     (void **)&h->d_cs,    (void **)&h->d_sn,
                          (void **)&h->d_g,     (void **)&h->d_w,     (void **)&h->d_r,
                          (void **)&h->d_rh,    (void **)&h->d_p,     (void **)&h->d_v,
                          (void **)&h->d_s,     (void **)&h->d_t,     (void **)&h->d_cq,
                          (void **)&h->d_state, (void **)&h->d_active, (void **)&h->d_cycle,
                          (void **)&h->d_count};
        auto undo = [&](int code) {
            for (void **q : group) {
                if (*q) (void)hipFree(*q);
                *q = nullptr;
            }
            return code;
        };
        if ((rc = dalloc(&h->d_H, (size_t)h->n_atm * (mm + 1) * mm)) != RT_OK) return undo(rc);
        if ((rc = dalloc(&h->d_cs, (size_t)h->n_atm * mm)) != RT_OK) return undo(rc);
        if ((rc = dalloc(&h->d_sn, (size_t)h->n_atm * mm)) != RT_OK) return undo(rc);
        if ((rc = dalloc(&h->d_g, (size_t)h->n_atm * (mm + 1))) != RT_OK) return undo(rc);
        double **vecs[] = {&h->d_w, &h->d_r, &h->d_rh, &h->d_p, &h->d_v, &h->d_s, &h->d_t, &h->d_cq};
        for (double **v : vecs)
            if ((rc = dalloc(v, (size_t)N)) != RT_OK) return undo(rc);
        if ((rc = dalloc(&h->d_state, (size_t)2 * h->n_atm)) != RT_OK) return undo(rc);
        if ((rc = dalloc(&h->d_active, (size_t)2 * h->n_atm)) != RT_OK) return undo(rc);
        if ((rc = dalloc(&h->d_cycle, (size_t)h->n_atm)) != RT_OK) return undo(rc);
        if ((rc = dalloc(&h->d_count, 1)) != RT_OK) return undo(rc);
        if (!h->h_count && hipHostMalloc((void **)&h->h_count, sizeof(int)) != hipSuccess) {
            h->h_count = nullptr;
            return undo(fail(RT_ENOMEM, "pinned host allocation failed"));
        }
    }
    h->ws_restart = m;
    return RT_OK;
}

}  // namespace rt

using namespace rt;

extern "C" {

void rt_default_options(rt_options *o) {
    if (!o) return;
    o->precision = RT_PREC_FP64;
    o->restart = 30;
    o->maxit = 10000;
    o->rtol = 1e-10;
    o->inner_rtol = 3e-4;
    o->inner_maxit = 200;
    o->max_outer = 30;
    o->chunk = 0;
    o->wave_batches = 0;
    o->prefetch = 0;
    o->sweep_waves = 0;
    o->graphs = 0;
    o->precond = RT_PC_JACOBI;
    o->omega = 1.0;
    o->check_every = 16;
    o->coef_mode = RT_COEF_AUTO;
    o->autotune = 0;
    o->plan_file = nullptr;
}

const char *rt_last_error(void) { return g_err.c_str(); }

int rt_num_unknowns(const rt_handle *h) { return h ? h->n_unk : 0; }

void rt_destroy(rt_handle *h) {
    if (!h) return;
    void *ptrs[] = {h->d_tau,   h->d_B,     h->d_opac,    h->d_phi,     h->d_mu_pos, h->d_w_pos,
                    h->d_w_nu,  h->d_pt_atm, h->d_atm,    h->d_blk,     h->d_rayc,   h->d_coef64,
                    h->d_atm_tail, h->d_blk_tail,
                    h->d_q,     h->d_qt,      h->d_dirc,    h->d_Qs,
                    h->d_coef32, h->d_partial, h->d_diag,  h->d_dinv,   h->d_b,
                    h->d_V,     h->d_H,     h->d_cs,      h->d_sn,      h->d_g,      h->d_w,
                    h->d_r,     h->d_rh,    h->d_p,       h->d_v,       h->d_s,      h->d_t,
                    h->d_cq,    h->d_state, h->d_active,  h->d_cycle,   h->d_count,
                    h->d_ew,    h->d_asm_dg, h->d_asm_sc, h->d_asm_task, h->d_A,
                    h->d_pz,    h->d_ones,  h->d_LU,      h->d_piv,     h->d_sing,
                    h->d_rpart, h->d_mu_idx, h->d_fsig, h->d_Rw,   h->d_Rw_bf, h->d_prd_Jm,
                    h->d_prd_J, h->d_prd_diag, h->d_prd_dinv, h->d_w64, h->d_w32, h->d_kt,
                    h->d_dtau, h->seg_ws[0], h->seg_ws[1], h->d_lu_order};
    clear_graphs(h);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    for (hipEvent_t e : h->gev)
        if (e) (void)hipEventDestroy(e);
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (h->h_count) (void)hipHostFree(h->h_count);
    if (h->h_seg_flag) (void)hipHostFree(h->h_seg_flag);
    delete h;
}

int rt_setup(rt_handle **out, const rt_problem *p, const rt_options *o) {
    if (!out) return fail(RT_EINVAL, "handle pointer is NULL");
    *out = nullptr;
    rt_options opt;
    rt_default_options(&opt);
    if (o) opt = *o;
    std::vector<double> mu_pos, w_pos;
    std::vector<int> mu_index;
    int rc = validate(p, &opt, mu_pos, w_pos, &mu_index);
    if (rc != RT_OK) return rc;

    // ---- device
    int dev = 0, ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(RT_EDEVICE, "no HIP device available");
    }
    if (hipGetDevice(&dev) != hipSuccess) return fail(RT_EDEVICE, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(RT_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(RT_EDEVICE, std::string("this library is built for gfx950, device is ") +
                                    prop.gcnArchName);

    int plan_status = 0;
    if (opt.autotune) {
        const rt_options asked = opt;
        plan_status = apply_stored_plan(p, &opt, device_arch());
        // a stored plan that does not fit these options or slabs is not applied
        bool fits = true;
        for (int a = 0; a < p->n_atm && opt.chunk; ++a)
            fits = fits && (long long)kWave * opt.chunk >= p->ns[a] - 1;
        if (plan_status && (!fits || validate(p, &opt, mu_pos, w_pos, &mu_index) != RT_OK)) {
            opt = asked;
            plan_status = 0;
            rc = validate(p, &opt, mu_pos, w_pos, &mu_index);
            if (rc != RT_OK) return rc;
        }
    }

    rt_handle *h = new rt_handle();
    h->device = dev;
    h->opt = opt;
    h->plan_status = plan_status;
    resolve_coef_modes(opt.coef_mode, &h->cm64, &h->cm32);
    h->n_atm = p->n_atm;
    h->n_mu = p->n_mu;
    h->M = p->n_mu / 2;
    h->n_nu = p->n_nu;
    h->fs = p->formal_solver;
    h->normalize = p->normalize_profile != 0;
    h->ns.assign(p->ns, p->ns + p->n_atm);
    h->doff.resize(h->n_atm);
    int acc = 0;
    for (int a = 0; a < h->n_atm; ++a) {
        h->doff[a] = acc;
        acc += h->ns[a];
        h->ns_max = std::max(h->ns_max, h->ns[a]);
    }
    h->ns_total = acc;
    h->n_unk = 2 * acc;

    // ---- plan: chunks, wave-batches, blocks, tiles, partial sums
    const int rays = h->M * h->n_nu;
    h->L = opt.chunk ? opt.chunk : auto_chunk(h->ns, rays);
    for (int n : h->ns)
        if ((long long)kWave * h->L < n - 1) {
            delete h;
            return fail(RT_EINVAL, "options.chunk too short for ns (need 64 * chunk >= ns - 1)");
        }
    if ((rc = check_tile_range(h->ns, h->L, h->n_nu)) != RT_OK) {
        delete h;
        return rc;
    }
    long long coef = 0, part = 0, qt = 0, dense = 0, ew = 0, part_t = 0;
    int blk = 0, blk_t = 0;
    h->nblk_max = h->nblk_max_tail = 0;
    std::vector<AtmDesc> atm_t(h->n_atm);
    std::vector<BlockDesc> blk_t_h;
    // Waves per block and wave-batches per wave.  A block never mixes
    // directions.  Big batches: one block per (slab, direction), the fewest
    // partial sums; small problems: about 48 blocks in all, for parallelism.
    h->W = opt.sweep_waves ? opt.sweep_waves : sweep_waves(h->L, false);
    const long long dirs_total = (long long)h->n_atm * h->M;
    const int blocks_per_dir = (int)std::max<long long>(1, (48 + dirs_total - 1) / dirs_total);
    h->atm_h.resize(h->n_atm);
    for (int a = 0; a < h->n_atm; ++a) {
        AtmDesc d{};
        d.ns = h->ns[a];
        d.doff = h->doff[a];
        const SlabTiles t = slab_tiles(d.ns, h->L, h->n_nu);
        d.C = t.C;
        d.Leff = t.Leff;
        d.nlong = t.nlong;
        d.G = t.G;
        d.n_nu = h->n_nu;
        d.nwb = t.nwb;
        d.bstride = t.bstride;
        d.ray_off = a * rays;
        int nb = (d.nwb + h->W * blocks_per_dir - 1) / (h->W * blocks_per_dir);
        nb = std::min(std::max(nb, 1), 32);
        if (opt.wave_batches > 0) nb = opt.wave_batches;
        const int wb_per_block = h->W * nb;
        const int blk_per_dir = (d.nwb + wb_per_block - 1) / wb_per_block;
        d.nblk = h->M * blk_per_dir;
        d.blk_first = blk;
        d.coef_off = coef;
        d.part_off = part;
        d.q_off = qt;
        d.a_off = dense;
        d.ew_off = ew;
        dense += 4LL * d.ns * d.ns;
        ew += (long long)(d.ns - 1) * rays;
        d.eps = p->eps[a];
        d.xi = 1.0 - p->eps[a];
        d.W2 = p->W2[a];
        d.Ibot = p->I_bot ? p->I_bot[a] : (p->B ? p->B[d.doff + d.ns - 1] : 1.0);
        for (int m = 0; m < h->M; ++m) {
            for (int bb = 0; bb < blk_per_dir; ++bb) {
                BlockDesc bd{};
                bd.atm = a;
                bd.m = m;
                bd.wb_first = bb * wb_per_block;
                bd.wb_count = std::min(wb_per_block, d.nwb - bd.wb_first);
                bd.slot = m * blk_per_dir + bb;
                h->blk_h.push_back(bd);
            }
        }
        h->NB = nb;
        // the tail plan: the same tiles, at most kTailWb wave-batches per
        // wave (a plan the caller fixed is kept for every cycle)
        {
            const int nbt = opt.wave_batches > 0 ? nb : std::min(nb, kTailWb);
            const int wbt = h->W * nbt;
            const int bpd = (d.nwb + wbt - 1) / wbt;
            AtmDesc dt = d;
            dt.nblk = h->M * bpd;
            dt.blk_first = blk_t;
            dt.part_off = part_t;
            for (int m = 0; m < h->M; ++m) {
                for (int bb = 0; bb < bpd; ++bb) {
                    BlockDesc bd{};
                    bd.atm = a;
                    bd.m = m;
                    bd.wb_first = bb * wbt;
                    bd.wb_count = std::min(wbt, d.nwb - bd.wb_first);
                    bd.slot = m * bpd + bb;
                    blk_t_h.push_back(bd);
                }
            }
            blk_t += dt.nblk;
            part_t += (long long)dt.nblk * 2 * d.ns;
            atm_t[a] = dt;
        }
        blk += d.nblk;
        h->nblk_max = std::max(h->nblk_max, d.nblk);
        h->nblk_max_tail = std::max(h->nblk_max_tail, atm_t[a].nblk);
        coef += (long long)h->M * d.nwb * d.bstride;
        qt += (long long)h->M * d.nwb * d.G;
        part += (long long)d.nblk * 2 * d.ns;
        h->atm_h[a] = d;
    }
    h->n_blocks = blk;
    // longest blocks first (work ~ wave-batches x chunk length, the same
    // lane count per batch); ties keep slab order
    auto order_blocks = [&](std::vector<BlockDesc> &list) {
        std::stable_sort(list.begin(), list.end(), [&](const BlockDesc &x, const BlockDesc &y) {
            return (long long)x.wb_count * h->atm_h[x.atm].Leff >
                   (long long)y.wb_count * h->atm_h[y.atm].Leff;
        });
        {
            // XCD-aware order: workgroups are handed to the 8 XCDs in turn by
            // index, and the blocks of one slab stage the same sources, so each
            // slab's run of blocks goes to one XCD (indices 8 apart, one L2) and
            // consecutive runs to consecutive XCDs -- the longest-first order
            // kept per group of 8 runs.  Applied when the runs fill the XCDs
            // evenly (equal-size runs, a multiple of 8 of them).
            constexpr int kXcd = 8;
            std::vector<std::vector<BlockDesc>> q(kXcd);
            size_t i = 0;
            int run = 0;
            while (i < list.size()) {
                size_t j = i;
                while (j < list.size() && list[j].atm == list[i].atm) ++j;
                for (size_t k = i; k < j; ++k) q[run % kXcd].push_back(list[k]);
                ++run;
                i = j;
            }
            bool even = true;
            for (int x = 1; x < kXcd; ++x) even = even && q[x].size() == q[0].size();
            if (even && !q[0].empty()) {
                std::vector<BlockDesc> out;
                out.reserve(list.size());
                for (size_t k = 0; k < q[0].size(); ++k)
                    for (int x = 0; x < kXcd; ++x) out.push_back(q[x][k]);
                list.swap(out);
            }
        }
    };
    order_blocks(h->blk_h);
    // the tail plan only where it differs (not for the three-point solver,
    // whose operator does not use the sweep blocks)
    const bool tail_plan = blk_t != blk && h->fs != RT_FS_DELO_PARABOLIC;
    if (tail_plan) {
        order_blocks(blk_t_h);
        h->n_blocks_tail = blk_t;
    }
    h->n_qt = qt;
    h->n_pairs = coef;
    h->n_partial = tail_plan ? std::max(part, part_t) : part;
    h->n_partial_main = part;
    h->n_dense = dense;
    h->n_ew = ew;

    // ---- device memory
    std::vector<int> pt_atm(acc);
    for (int a = 0; a < h->n_atm; ++a)
        std::fill(pt_atm.begin() + h->doff[a], pt_atm.begin() + h->doff[a] + h->ns[a], a);
    std::vector<double> B(acc, 1.0);
    if (p->B) std::copy(p->B, p->B + acc, B.begin());
    const size_t nphi = (size_t)h->n_atm * h->n_nu;
#define RT_TRY(x)            \
    do {                     \
        int _rc = (x);       \
        if (_rc != RT_OK) {  \
            rt_destroy(h);   \
            return _rc;      \
        }                    \
    } while (0)
    RT_TRY(dalloc(&h->d_tau, acc));
    RT_TRY(dalloc(&h->d_B, acc));
    RT_TRY(dalloc(&h->d_opac, nphi));
    RT_TRY(dalloc(&h->d_phi, nphi));
    RT_TRY(dalloc(&h->d_mu_pos, h->M));
    RT_TRY(dalloc(&h->d_mu_idx, (size_t)2 * h->M));
    RT_TRY(dalloc(&h->d_fsig, (size_t)2 * acc));
    RT_TRY(dalloc(&h->d_w_pos, h->M));
    RT_TRY(dalloc(&h->d_w_nu, h->n_nu));
    RT_TRY(dalloc(&h->d_pt_atm, acc));
    RT_TRY(dalloc(&h->d_atm, h->n_atm));
    RT_TRY(dalloc(&h->d_blk, h->n_blocks));
    RT_TRY(dalloc(&h->d_rayc, (size_t)h->n_atm * rays));
    RT_TRY(dalloc(&h->d_q, (size_t)h->n_atm * rays));
    RT_TRY(dalloc(&h->d_qt, (size_t)h->n_qt));
    RT_TRY(dalloc(&h->d_dirc, (size_t)h->M));
    RT_TRY(dalloc(&h->d_Qs, (size_t)h->n_atm));
    // the coefficient tiles the handle's sweeps stream, (kappa, 1 / kappa) per
    // ray and the depth steps for those that derive coefficients
    if (h->cm64 == kCoefPairs) RT_TRY(dalloc(&h->d_coef64, h->n_pairs));
    if (h->cm32 == kCoefPairs) RT_TRY(dalloc(&h->d_coef32, h->n_pairs));
    if (h->cm64 == kCoefW) RT_TRY(dalloc(&h->d_w64, h->n_pairs));
    if (h->cm32 == kCoefW) RT_TRY(dalloc(&h->d_w32, h->n_pairs));
    const bool derive = h->cm64 != kCoefPairs || h->cm32 != kCoefPairs;
    if (derive) {
        RT_TRY(dalloc(&h->d_kt, (size_t)h->n_qt));
        RT_TRY(dalloc(&h->d_dtau, acc));
        std::vector<double> dtau(acc, 0.0);
        for (int a = 0; a < h->n_atm; ++a)
            for (int k = 0; k + 1 < h->ns[a]; ++k)
                dtau[h->doff[a] + k] = p->tau[h->doff[a] + k + 1] - p->tau[h->doff[a] + k];
        RT_TRY(h2d(h->d_dtau, dtau.data(), acc));
    }
    RT_TRY(dalloc(&h->d_partial, std::max<long long>(h->n_partial, 1)));
    RT_TRY(dalloc(&h->d_diag, h->n_unk));
    RT_TRY(dalloc(&h->d_dinv, h->n_unk));
    RT_TRY(dalloc(&h->d_b, h->n_unk));
    if (h->fs == RT_FS_DELO_PARABOLIC)
        RT_TRY(dalloc(&h->d_rpart, (size_t)ray_slots(h) * 2 * acc));
    RT_TRY(h2d(h->d_tau, p->tau, acc));
    RT_TRY(h2d(h->d_B, B.data(), acc));
    RT_TRY(h2d(h->d_opac, p->opac, nphi));
    RT_TRY(h2d(h->d_phi, p->phi, nphi));
    RT_TRY(h2d(h->d_mu_pos, mu_pos.data(), h->M));
    RT_TRY(h2d(h->d_mu_idx, mu_index.data(), (size_t)2 * h->M));
    RT_TRY(h2d(h->d_w_pos, w_pos.data(), h->M));
    RT_TRY(h2d(h->d_w_nu, p->w_nu, h->n_nu));
    RT_TRY(h2d(h->d_pt_atm, pt_atm.data(), acc));
    RT_TRY(h2d(h->d_atm, h->atm_h.data(), h->n_atm));
    RT_TRY(h2d(h->d_blk, h->blk_h.data(), h->n_blocks));
    if (tail_plan) {
        RT_TRY(dalloc(&h->d_atm_tail, h->n_atm));
        RT_TRY(dalloc(&h->d_blk_tail, h->n_blocks_tail));
        RT_TRY(h2d(h->d_atm_tail, atm_t.data(), h->n_atm));
        RT_TRY(h2d(h->d_blk_tail, blk_t_h.data(), h->n_blocks_tail));
    }

    // ---- precompute: ray constants, tile coefficients, D and D^-1, b
    hipStream_t s = nullptr;
    RT_TRY(hip_check(launch_ray_setup(h->n_atm, h->d_atm, h->d_mu_pos, h->d_w_pos, h->M,
                                      h->d_w_nu, h->d_phi, h->n_nu, h->normalize, h->d_rayc,
                                      h->d_q, h->d_dirc, h->d_Qs, s),
                     "ray setup launch"));
    RT_TRY(hip_check(launch_coef_build(h->n_blocks, h->W, h->d_atm, h->d_blk, h->d_tau, h->d_opac,
                                       h->d_mu_pos, h->fs, h->d_q, h->d_coef64, h->d_coef32,
                                       h->d_w64, h->d_w32, h->d_qt, h->d_kt, s),
                     "coefficient launch"));
    RT_TRY(hip_check(launch_diag(acc, h->d_pt_atm, h->d_atm, h->d_tau, h->d_opac, h->d_mu_pos,
                                 h->d_rayc, h->M, h->n_nu, h->fs, h->d_diag, h->d_dinv, s),
                     "diagonal launch"));
    RT_TRY(hip_check(apply_operator(h, nullptr, nullptr, h->d_b, nullptr, false, 1, s),
                     "right-hand side launch"));
    RT_TRY(hip_check(hipDeviceSynchronize(), "setup"));
    // the frequency-redistribution variant, when the problem carries R
    if (p->R) RT_TRY(rt_set_redistribution(h, p->R));
#undef RT_TRY
    *out = h;
    return RT_OK;
}

int rt_apply_op(rt_handle *h, const double *sigma_in, double *sigma_out, void *stream) {
    if (!h || !sigma_in || !sigma_out) return fail(RT_EINVAL, "NULL handle or vector");
    if (!aligned16(sigma_in) || !aligned16(sigma_out))
        return fail(RT_EINVAL, "vectors must be 16-byte aligned");
    return hip_check(apply_operator(h, sigma_in, nullptr, sigma_out, nullptr, false, 0,
                                    (hipStream_t)stream),
                     "rt_apply_op");
}

int rt_apply_op_fp32(rt_handle *h, const double *sigma_in, double *sigma_out, void *stream) {
    if (!h || !sigma_in || !sigma_out) return fail(RT_EINVAL, "NULL handle or vector");
    if (!aligned16(sigma_in) || !aligned16(sigma_out))
        return fail(RT_EINVAL, "vectors must be 16-byte aligned");
    return hip_check(apply_operator(h, sigma_in, nullptr, sigma_out, nullptr, true, 0,
                                    (hipStream_t)stream),
                     "rt_apply_op_fp32");
}

int rt_precond_jacobi(rt_handle *h, const double *v, double *z, void *stream) {
    if (!h || !v || !z) return fail(RT_EINVAL, "NULL handle or vector");
    if (!aligned16(v) || !aligned16(z)) return fail(RT_EINVAL, "vectors must be 16-byte aligned");
    return hip_check(launch_scale(v, h->d_dinv, z, h->n_unk, (hipStream_t)stream),
                     "rt_precond_jacobi");
}

int rt_get_rhs(rt_handle *h, double *b, void *stream) {
    if (!h || !b) return fail(RT_EINVAL, "NULL handle or vector");
    return hip_check(hipMemcpyAsync(b, h->d_b, sizeof(double) * h->n_unk,
                                    hipMemcpyDeviceToDevice, (hipStream_t)stream),
                     "rt_get_rhs");
}

int rt_get_jacobi_diag(rt_handle *h, double *d, void *stream) {
    if (!h || !d) return fail(RT_EINVAL, "NULL handle or vector");
    return hip_check(hipMemcpyAsync(d, h->d_diag, sizeof(double) * h->n_unk,
                                    hipMemcpyDeviceToDevice, (hipStream_t)stream),
                     "rt_get_jacobi_diag");
}

int rt_solve_gmres(rt_handle *h, const double *b, double *x, rt_solve_info *info, void *stream) {
    if (!h || !x) return fail(RT_EINVAL, "NULL handle or x");
    if (!aligned16(x) || (b && !aligned16(b))) return fail(RT_EINVAL, "vectors must be 16-byte aligned");
    return run_solver(h, 0, b, x, info, (hipStream_t)stream);
}

int rt_solve_bicgstab(rt_handle *h, const double *b, double *x, rt_solve_info *info,
                      void *stream) {
    if (!h || !x) return fail(RT_EINVAL, "NULL handle or x");
    if (!aligned16(x) || (b && !aligned16(b))) return fail(RT_EINVAL, "vectors must be 16-byte aligned");
    return run_solver(h, 1, b, x, info, (hipStream_t)stream);
}

int rt_solve_richardson(rt_handle *h, const double *b, double *x, rt_solve_info *info,
                        void *stream) {
    if (!h || !x) return fail(RT_EINVAL, "NULL handle or x");
    if (!aligned16(x) || (b && !aligned16(b))) return fail(RT_EINVAL, "vectors must be 16-byte aligned");
    return run_solver(h, 2, b, x, info, (hipStream_t)stream);
}

int rt_solve_cgs(rt_handle *h, const double *b, double *x, rt_solve_info *info, void *stream) {
    if (!h || !x) return fail(RT_EINVAL, "NULL handle or x");
    if (!aligned16(x) || (b && !aligned16(b))) return fail(RT_EINVAL, "vectors must be 16-byte aligned");
    return run_solver(h, 3, b, x, info, (hipStream_t)stream);
}

// Sweep-plan introspection for tests and benchmarks (not in the public header).
int rt_plan_info(const rt_handle *h, int *chunk_L, int *n_blocks, long long *n_pairs,
                 long long *n_intervals) {
    if (!h) return fail(RT_EINVAL, "NULL handle");
    if (chunk_L) *chunk_L = h->L;
    if (n_blocks) *n_blocks = h->n_blocks;
    if (n_pairs) *n_pairs = h->n_pairs;
    if (n_intervals) {
        long long s = 0;
        for (int n : h->ns) s += (long long)(n - 1) * h->M * h->n_nu;
        *n_intervals = s;
    }
    return RT_OK;
}

int rt_sweep_config(const rt_handle *h, int fp32, int *waves, int *prefetch) {
    if (!h) return fail(RT_EINVAL, "NULL handle");
    int W;
    bool pf;
    sweep_config(h, fp32 != 0, &W, &pf);
    if (waves) *waves = W;
    if (prefetch) *prefetch = pf ? 1 : 0;
    return RT_OK;
}

int rt_tuned_plan_status(const rt_handle *h) { return h ? h->plan_status : 0; }

int rt_get_options(const rt_handle *h, rt_options *o) {
    if (!h || !o) return fail(RT_EINVAL, "NULL handle or output");
    *o = h->opt;
    o->plan_file = nullptr;  // the caller's string is not kept
    return RT_OK;
}

const char *rt_sweep_source_hash(void) { return RT_SWEEP_SOURCE_HASH; }

int rt_plan_key(const rt_problem *p, int precision, const char *arch, char *buf, int buflen) {
    if (!p || !p->ns || p->n_atm < 1 || !buf || buflen < 1)
        return fail(RT_EINVAL, "NULL problem or buffer");
    const std::string a = arch ? std::string(arch) : device_arch();
    if (a.empty()) return fail(RT_EDEVICE, "no device to take the architecture from");
    const std::string k = plan_key(p, precision, a);
    if ((int)k.size() + 1 > buflen) return fail(RT_EINVAL, "buffer too short for the plan key");
    std::memcpy(buf, k.c_str(), k.size() + 1);
    return RT_OK;
}

int rt_sweep_coef_mode(const rt_handle *h, int fp32, int *mode) {
    if (!h || !mode) return fail(RT_EINVAL, "NULL handle or output");
    *mode = coef_mode_of(h, fp32 != 0);
    return RT_OK;
}

int rt_solve_lu(rt_handle *h, const double *b, double *x, rt_solve_info *info, void *stream) {
    if (!h || !x) return fail(RT_EINVAL, "NULL handle or x");
    if (!aligned16(x) || (b && !aligned16(b))) return fail(RT_EINVAL, "vectors must be 16-byte aligned");
    return run_solver(h, 4, b, x, info, (hipStream_t)stream);
}

int rt_precond_apply(rt_handle *h, const double *v, double *z, void *stream) {
    if (!h || !v || !z) return fail(RT_EINVAL, "NULL handle or vector");
    if (!aligned16(v) || !aligned16(z)) return fail(RT_EINVAL, "vectors must be 16-byte aligned");
    const hipStream_t s = (hipStream_t)stream;
    if (h->opt.precond == RT_PC_JACOBI)
        return hip_check(launch_scale(v, h->d_dinv, z, h->n_unk, s), "rt_precond_apply");
    const int rc = ensure_dense(h, s);
    if (rc != RT_OK) return rc;
    return hip_check(precond_tri(h, v, z, nullptr, s), "rt_precond_apply");
}

int rt_assembled_size(const rt_handle *h, long long *count) {
    if (!h || !count) return fail(RT_EINVAL, "NULL handle or count");
    *count = h->n_dense;
    return RT_OK;
}

int rt_assemble(rt_handle *h, double *A_out, void *stream) {
    if (!h || !A_out) return fail(RT_EINVAL, "NULL handle or output");
    if (h->fs == RT_FS_DELO_PARABOLIC)
        return fail(RT_EINVAL, "rt_assemble supports the two-point formal solvers only");
    if (!aligned16(A_out)) return fail(RT_EINVAL, "output must be 16-byte aligned");
    return assemble(h, A_out, (hipStream_t)stream);
}

int rt_field_size(const rt_handle *h, long long *count) {
    if (!h || !count) return fail(RT_EINVAL, "NULL handle or count");
    *count = 2LL * h->n_mu * h->n_nu * h->ns_total;
    return RT_OK;
}

int rt_apply_op_field(rt_handle *h, const double *I_in, double *I_out, void *stream) {
    if (!h || !I_in || !I_out) return fail(RT_EINVAL, "NULL handle or vector");
    if (I_in == I_out) return fail(RT_EINVAL, "I_in and I_out must not alias");
    return hip_check(apply_field_operator(h, I_in, I_out, (hipStream_t)stream), "rt_apply_op_field");
}

int rt_get_rhs_field(rt_handle *h, double *b_field, void *stream) {
    if (!h || !b_field) return fail(RT_EINVAL, "NULL handle or vector");
    return hip_check(field_rhs(h, b_field, (hipStream_t)stream), "rt_get_rhs_field");
}

int rt_solve_field_gmres(rt_handle *h, const double *b_field, double *I, rt_solve_info *info,
                         void *stream) {
    if (!h || !I) return fail(RT_EINVAL, "NULL handle or I");
    if (b_field == I) return fail(RT_EINVAL, "b_field and I must not alias");
    return solve_field_gmres(h, b_field, I, info, (hipStream_t)stream);
}

int rt_set_redistribution(rt_handle *h, const double *R) {
    if (!h || !R) return fail(RT_EINVAL, "NULL handle or R");
    const long long n = (long long)h->n_atm * h->n_nu * h->n_nu;
    for (long long e = 0; e < n; ++e)
        if (!std::isfinite(R[e])) return fail(RT_EINVAL, "R must be finite");
    // R(p, q) w_q stored transposed ([slab][q][p]), the form the contraction reads
    const int nnu = h->n_nu;
    std::vector<double> w_nu(nnu), Rw(n);
    if (hipMemcpy(w_nu.data(), h->d_w_nu, sizeof(double) * nnu, hipMemcpyDeviceToHost) !=
        hipSuccess)
        return fail(RT_EDEVICE, "reading the frequency weights failed");
    for (long long s0 = 0; s0 < n; s0 += (long long)nnu * nnu)
        for (int pp = 0; pp < nnu; ++pp)
            for (int q = 0; q < nnu; ++q)
                Rw[s0 + (long long)q * nnu + pp] = R[s0 + (long long)pp * nnu + q] * w_nu[q];
    if (!h->d_Rw && hipMalloc((void **)&h->d_Rw, sizeof(double) * n) != hipSuccess) {
        h->d_Rw = nullptr;
        (void)hipGetLastError();
        return fail(RT_ENOMEM, "device allocation of R failed");
    }
    if (hipMemcpy(h->d_Rw, Rw.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess)
        return fail(RT_EDEVICE, "upload of R failed");
    // the bf16 split of R(p, q) w_q, row-major with zero-padded rows: hi =
    // bf16(x), lo = bf16(x - hi), both rounded to nearest even from FP32
    const int nqp = (nnu + 31) / 32 * 32;
    const long long nbf = (long long)h->n_atm * nnu * nqp;
    auto to_bf16 = [](float f) {
        unsigned u;
        std::memcpy(&u, &f, sizeof u);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (unsigned short)(u >> 16);
    };
    auto from_bf16 = [](unsigned short b) {
        const unsigned u = (unsigned)b << 16;
        float f;
        std::memcpy(&f, &u, sizeof f);
        return f;
    };
    std::vector<unsigned short> bf(2 * nbf, 0);
    for (int a = 0; a < h->n_atm; ++a)
        for (int pp = 0; pp < nnu; ++pp)
            for (int q = 0; q < nnu; ++q) {
                const long long s0 = (long long)a * nnu * nnu;
                const float x = (float)Rw[s0 + (long long)q * nnu + pp];
                const unsigned short hi = to_bf16(x);
                const long long e = ((long long)a * nnu + pp) * nqp + q;
                bf[e] = hi;
                bf[nbf + e] = to_bf16(x - from_bf16(hi));
            }
    if (!h->d_Rw_bf && hipMalloc((void **)&h->d_Rw_bf, sizeof(unsigned short) * 2 * nbf) != hipSuccess) {
        h->d_Rw_bf = nullptr;
        (void)hipGetLastError();
        return fail(RT_ENOMEM, "device allocation of the bf16 split of R failed");
    }
    h->prd_nqp = nqp;
    if (hipMemcpy(h->d_Rw_bf, bf.data(), sizeof(unsigned short) * 2 * nbf, hipMemcpyHostToDevice) !=
        hipSuccess)
        return fail(RT_EDEVICE, "upload of the bf16 split of R failed");
    h->prd_ready = false;  // the diagonal depends on R
    return RT_OK;
}

int rt_prd_size(const rt_handle *h, long long *count) {
    if (!h || !count) return fail(RT_EINVAL, "NULL handle or count");
    *count = 2LL * h->n_nu * h->ns_total;
    return RT_OK;
}

int rt_apply_op_prd(rt_handle *h, const double *sigma_in, double *sigma_out, void *stream) {
    if (!h || !sigma_in || !sigma_out) return fail(RT_EINVAL, "NULL handle or vector");
    const int rc = ensure_prd(h, (hipStream_t)stream);
    if (rc != RT_OK) return rc;
    return hip_check(apply_prd_operator(h, sigma_in, sigma_out, (hipStream_t)stream),
                     "rt_apply_op_prd");
}

int rt_apply_op_prd_bf16x3(rt_handle *h, const double *sigma_in, double *sigma_out, void *stream) {
    if (!h || !sigma_in || !sigma_out) return fail(RT_EINVAL, "NULL handle or vector");
    const int rc = ensure_prd(h, (hipStream_t)stream);
    if (rc != RT_OK) return rc;
    return hip_check(apply_prd_operator(h, sigma_in, sigma_out, (hipStream_t)stream, true),
                     "rt_apply_op_prd_bf16x3");
}

int rt_get_rhs_prd(rt_handle *h, double *b, void *stream) {
    if (!h || !b) return fail(RT_EINVAL, "NULL handle or vector");
    const int rc = ensure_prd(h, (hipStream_t)stream);
    if (rc != RT_OK) return rc;
    return hip_check(apply_prd_operator(h, nullptr, b, (hipStream_t)stream), "rt_get_rhs_prd");
}

int rt_get_jacobi_diag_prd(rt_handle *h, double *d, void *stream) {
    if (!h || !d) return fail(RT_EINVAL, "NULL handle or vector");
    const int rc = ensure_prd(h, (hipStream_t)stream);
    if (rc != RT_OK) return rc;
    return hip_check(hipMemcpyAsync(d, h->d_prd_diag, sizeof(double) * 2 * h->n_nu * h->ns_total,
                                    hipMemcpyDeviceToDevice, (hipStream_t)stream),
                     "rt_get_jacobi_diag_prd");
}

int rt_solve_prd_gmres(rt_handle *h, const double *b, double *x, rt_solve_info *info,
                       void *stream) {
    if (!h || !x) return fail(RT_EINVAL, "NULL handle or x");
    if (b == x) return fail(RT_EINVAL, "b and x must not alias");
    return solve_prd_gmres(h, b, x, info, (hipStream_t)stream);
}

int rt_sigma_from_field(rt_handle *h, const double *I, double *sigma, void *stream) {
    if (!h || !I || !sigma) return fail(RT_EINVAL, "NULL handle or vector");
    return hip_check(field_sigma(h, I, sigma, 1, (hipStream_t)stream), "rt_sigma_from_field");
}

// Validation only, without touching the device (tests of the error paths).
int rt_validate(const rt_problem *p, const rt_options *o) {
    std::vector<double> mp, wp;
    rt_options opt;
    rt_default_options(&opt);
    if (o) opt = *o;
    int rc = validate(p, &opt, mp, wp);
    if (rc != RT_OK) return rc;
    // the plan checks rt_setup makes before any device call
    const std::vector<int> ns(p->ns, p->ns + p->n_atm);
    const int L = opt.chunk ? opt.chunk : auto_chunk(ns, (p->n_mu / 2) * p->n_nu);
    for (int n : ns)
        if ((long long)kWave * L < n - 1)
            return fail(RT_EINVAL, "options.chunk too short for ns (need 64 * chunk >= ns - 1)");
    return check_tile_range(ns, L, p->n_nu);
}

}  // extern "C"
