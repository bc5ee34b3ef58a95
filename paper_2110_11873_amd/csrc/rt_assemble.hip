// rt_assemble.hip -- dense assembly of A = Id - J Lambda T on gfx950.
//
// Sect. 3.3 assembles A column by column, applying Algorithm 1 to the unit
// vectors; a point source at depth j leaves the intensity zero upwind of j
// and only decays downwind of it (Sect. 4.4).  Here the columns of a block of
// 64 source depths are built together by a multi-source sweep:
//
//  * lane j of every wavefront owns source column j; a wavefront owns one
//    |mu| and up to RG frequencies of it and keeps their intensities
//    I_r(k; j) in registers, pre-multiplied by the ray weight q_r;
//  * walking k downwind from the block, a ray's intensity picks up the
//    source at k = j (through c_k of the interval entering j) and at
//    k = j + 1 (through c_u), then only decays: I *= E;
//  * the wavefront sums its rays in registers, so its row k is
//    sum_p q_p Lambda_p(k, j); the T^2_0 weights of its |mu| turn that into
//    the three moments sum q Lambda, sum q T1 Lambda, sum q (T1^2 + T2^2)
//    Lambda that make up the 2x2 block of A at (k, j) (eqs. J00/J02 with
//    S_I = s00 + T1 s20, S_Q = T2 s20), and the wavefronts of a workgroup
//    add theirs in LDS in a fixed order once per depth step.
//
// The downward rays give the lower triangle (k > j), the upward rays -- the
// same code on the reversed depth order -- the upper one; the 2x2 blocks on
// the diagonal receive both and are written by a separate pass.  When a
// workgroup cannot hold every ray, the rays are split into slices whose
// moments are stored apart and added, in slice order, by a combine pass.
// Nothing is accumulated with atomics: the result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "rt_coef.h"
#include "rt_internal.h"

namespace rt {

namespace {

struct AsmTask {
    int atm;    // slab
    int dir;    // 0: mu < 0 (downward, lower triangle), 1: mu > 0 (upward, upper)
    int jblk;   // block of 64 source depths, in the direction's depth order
    int slice;  // ray slice
};

struct AsmArgs {
    const AtmDesc *atm;
    const AsmTask *task;
    const double2 *ew;       // (E, w) per slab, interval and ray
    const RayConst *rayc;
    const double2 *dirc;     // per |mu|: (T1, T1^2 + T2^2)
    double *A;               // final A, or the raw moments of slice 0
    double *sc;              // raw moments of slices 1.. (stride sc_stride)
    long long sc_stride;
    double *dg;              // [slice][dir][ns_total][3] moments of the diagonal blocks
    int ns_total;
    int n_nu, M;
    int cpm;                 // wavefronts (frequency groups) per |mu|
    int nw;                  // wavefronts per workgroup
    int slices;
};

// (E, w) per (slab, interval i = 1..ns-1 between depths i-1 and i, ray
// r = m n_nu + p), at ew_off + (i - 1) (M n_nu) + r.
__global__ void ew_table_kernel(const AtmDesc *atm, const double *tau, const double *opac,
                                const double *mu_pos, int M, int n_nu, int fs, double2 *ew) {
    const AtmDesc at = atm[blockIdx.y];
    const int R = M * n_nu;
    const long long n = (long long)(at.ns - 1) * R;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / R) + 1, r = (int)(e % R);
        const int m = r / n_nu, p = r % n_nu;
        const double kap = opac[(long long)blockIdx.y * n_nu + p] / mu_pos[m];
        const double d = kap * (tau[at.doff + i] - tau[at.doff + i - 1]);
        double E, w;
        step_ew(fs, d, E, w);
        ew[at.ew_off + e] = make_double2(E, w);
    }
}

// One workgroup per task: NT / 64 wavefronts of RG ray slots each.  LDS:
// E of the current and next step, and for the first 65 steps the injections
// q c_k (at k = j) and q c_u (at k = j + 1), double-buffered; the wave
// moments of the current and previous step.
template <int RG, int NT>
__global__ __launch_bounds__(NT) void assemble_kernel(AsmArgs g) {
    static_assert(RG % 2 == 0, "rays are read in pairs");
    extern __shared__ double smem[];
    const AsmTask t = g.task[blockIdx.x];
    const AtmDesc at = g.atm[t.atm];
    const int ns = at.ns, R = g.M * g.n_nu;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nrs = g.nw * RG;           // ray slots of the workgroup (<= NT)
    double *eb = smem;                   // [2][nrs] E
    double *ab = eb + 2 * nrs;           // [2][nrs] q c_k
    double *bb = ab + 2 * nrs;           // [2][nrs] q c_u
    double *part = bb + 2 * nrs;         // [2][nw][3][64]

    // slot s = w RG + i holds frequency p = (c % cpm) RG + i of |mu| m = c / cpm,
    // c = slice nw + w; slots past the last ray have q = 0 and E = 1
    const int nchunks = g.M * g.cpm;
    const int my_slot = threadIdx.x;
    int my_ray = -1;
    if (my_slot < nrs) {
        const int c = t.slice * g.nw + my_slot / RG;
        const int p = (c % g.cpm) * RG + my_slot % RG;
        if (c < nchunks && p < g.n_nu) my_ray = (c / g.cpm) * g.n_nu + p;
    }
    const double my_q = my_ray >= 0 ? g.rayc[at.ray_off + my_ray].q : 0.0;
    // (E, w) of the interval entering depth k of the direction's order; depth
    // 0 has none: (1, 1), so that c_k = 1 - w = 0 there
    auto ew_at = [&](int k) -> double2 {
        if (k <= 0 || my_ray < 0) return make_double2(1.0, 1.0);
        const int row = t.dir == 0 ? k - 1 : ns - 1 - k;
        return g.ew[at.ew_off + (long long)row * R + my_ray];
    };
    auto stage = [&](int buf, double2 v, bool inj) {
        eb[buf * nrs + my_slot] = v.x;
        if (inj) {
            ab[buf * nrs + my_slot] = my_q * (1.0 - v.y);  // c_k = 1 - w
            bb[buf * nrs + my_slot] = my_q * (v.y - v.x);  // c_u = w - E
        }
    };

    const int c = t.slice * g.nw + wave;
    const double2 tw = g.dirc[c < nchunks ? c / g.cpm : 0];  // (T1, T1^2 + T2^2)
    const int j0 = t.jblk * kWave;
    const int j = j0 + lane;
    const int nsteps = ns - j0;

    double It[RG];
#pragma unroll
    for (int i = 0; i < RG; ++i) It[i] = 0.0;

    if (my_slot < nrs) stage(0, ew_at(j0), true);
    __syncthreads();

    // One depth step: advance every ray of the wavefront to depth k, write
    // the wavefront's moments, stage the next step's coefficients, then sum
    // the wavefronts and store row k.  INJ: sources j0..j0+63 enter at
    // k = j (through c_k) and k = j + 1 (through c_u).
    auto step = [&](int st, auto inj_tag) {
        constexpr bool INJ = decltype(inj_tag)::value;
        const int k = j0 + st;
        const int cur = st & 1;
        const bool pre = my_slot < nrs && st + 1 < nsteps;
        double2 nxt = make_double2(1.0, 1.0);
        if (pre) nxt = ew_at(k + 1);  // loaded during this step

        const double *e = eb + cur * nrs + wave * RG;
        double acc0 = 0.0, acc1 = 0.0;
        if constexpr (INJ) {
#pragma clang fp contract(off)
            const double *a = ab + cur * nrs + wave * RG;
            const double *b = bb + cur * nrs + wave * RG;
            // 0/1 per lane: no branch and no select on the loaded values
            const double fa = k == j ? 1.0 : 0.0, fb = k == j + 1 ? 1.0 : 0.0;
#pragma unroll
            for (int i = 0; i < RG; i += 2) {
                const double2 e2 = *reinterpret_cast<const double2 *>(e + i);
                const double2 a2 = *reinterpret_cast<const double2 *>(a + i);
                const double2 b2 = *reinterpret_cast<const double2 *>(b + i);
                It[i] = fma(e2.x, It[i], fma(fa, a2.x, fb * b2.x));
                It[i + 1] = fma(e2.y, It[i + 1], fma(fa, a2.y, fb * b2.y));
                acc0 += It[i];
                acc1 += It[i + 1];
            }
        } else {
            // no contraction of the product into the sum: the product is the
            // new state, and a fused form would keep E live to recompute it
#pragma clang fp contract(off)
#pragma unroll
            for (int i = 0; i < RG; i += 2) {
                const double2 e2 = *reinterpret_cast<const double2 *>(e + i);
                It[i] *= e2.x;
                It[i + 1] *= e2.y;
                acc0 += It[i];
                acc1 += It[i + 1];
            }
        }
        const double acc = acc0 + acc1;
        double *pp = part + (cur * g.nw + wave) * 3 * kWave;
        pp[lane] = acc;
        pp[kWave + lane] = acc * tw.x;
        pp[2 * kWave + lane] = acc * tw.y;
        if (pre) stage(cur ^ 1, nxt, st + 1 <= kWave);
        __syncthreads();

        // (moment, column) pairs over the workgroup's threads (a workgroup of
        // fewer than three wavefronts takes several pairs per thread)
        for (int idx = threadIdx.x; idx < 3 * kWave; idx += blockDim.x) {
            const int mom = idx / kWave, l = idx % kWave;
            const int jj = j0 + l;
            if (jj <= k && jj < ns) {
                double v = 0.0;
#pragma unroll 4
                for (int w = 0; w < g.nw; ++w) v += part[((cur * g.nw + w) * 3 + mom) * kWave + l];
                const int K = t.dir == 0 ? k : ns - 1 - k;
                const int J = t.dir == 0 ? jj : ns - 1 - jj;
                if (K == J) {
                    g.dg[(((long long)t.slice * 2 + t.dir) * g.ns_total + at.doff + K) * 3 + mom] = v;
                } else {
                    const long long N = 2LL * ns;
                    const long long base = 2LL * K * N + 2LL * J;
                    if (g.slices == 1) {
                        double *A = g.A + at.a_off;
                        if (mom == 0) {
                            A[base] = -at.xi * v;
                        } else if (mom == 1) {
                            A[base + 1] = -at.xi * v;
                            A[base + N] = -at.xi * at.W2 * v;
                        } else {
                            A[base + N + 1] = -at.xi * at.W2 * v;
                        }
                    } else {
                        double *buf = (t.slice == 0 ? g.A : g.sc + (t.slice - 1) * g.sc_stride) +
                                      at.a_off;
                        buf[base + (mom == 0 ? 0 : mom == 1 ? 1 : N + 1)] = v;
                    }
                }
            }
        }
    };
    const int ninj = min(nsteps, kWave + 1);
    for (int st = 0; st < ninj; ++st) step(st, std::true_type{});
    for (int st = ninj; st < nsteps; ++st) step(st, std::false_type{});
}

// Off-diagonal 2x2 blocks from the slices' raw moments (slices > 1).
__global__ void assemble_combine_kernel(AsmArgs g) {
    const AtmDesc at = g.atm[blockIdx.y];
    const long long ns = at.ns, N = 2 * ns;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < ns * ns;
         e += (long long)gridDim.x * blockDim.x) {
        const long long K = e / ns, J = e % ns;
        if (K == J) continue;
        const long long base = at.a_off + 2 * K * N + 2 * J;
        double v0 = g.A[base], v1 = g.A[base + 1], v2 = g.A[base + N + 1];
        for (int s = 1; s < g.slices; ++s) {
            const double *b = g.sc + (s - 1) * g.sc_stride;
            v0 += b[base];
            v1 += b[base + 1];
            v2 += b[base + N + 1];
        }
        g.A[base] = -at.xi * v0;
        g.A[base + 1] = -at.xi * v1;
        g.A[base + N] = -at.xi * at.W2 * v1;
        g.A[base + N + 1] = -at.xi * at.W2 * v2;
    }
}

// The 2x2 blocks on the diagonal: both directions, all slices, plus Id.
__global__ void assemble_diag_kernel(AsmArgs g, const int *pt_atm) {
    const int kk = blockIdx.x * blockDim.x + threadIdx.x;
    if (kk >= g.ns_total) return;
    const AtmDesc at = g.atm[pt_atm[kk]];
    const long long K = kk - at.doff, N = 2LL * at.ns;
    double v[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < g.slices; ++s)
        for (int d = 0; d < 2; ++d)
            for (int mom = 0; mom < 3; ++mom)
                v[mom] += g.dg[(((long long)s * 2 + d) * g.ns_total + kk) * 3 + mom];
    double *A = g.A + at.a_off + 2 * K * N + 2 * K;
    A[0] = 1.0 - at.xi * v[0];
    A[1] = -at.xi * v[1];
    A[N] = -at.xi * at.W2 * v[1];
    A[N + 1] = 1.0 - at.xi * at.W2 * v[2];
}

// Compiled variants: ray slots per wavefront and workgroup size.  Up to 24
// slots the intensities and the loop's temporaries fit 128 VGPRs (16
// wavefronts per workgroup); 52 and 64 slots fit 256 VGPRs (8 wavefronts).
// Every thread stages at most one slot's coefficients, so a wavefront holds
// at most 64 slots.
struct AsmVariant {
    int rg, nt;
};
constexpr AsmVariant kVariants[] = {{8, 1024}, {16, 1024}, {24, 1024}, {52, 512}, {64, 512}};
static_assert(kVariants[4].rg <= kWave, "one staged slot per thread");

size_t asm_lds_bytes(int nw, int rg) {
    const size_t nrs = (size_t)nw * rg;
    return (6 * nrs + 2 * (size_t)nw * 3 * kWave) * sizeof(double);
}

template <int RG, int NT>
hipError_t launch_variant(const AsmArgs &a, int ntasks, hipStream_t s) {
    const size_t lds = asm_lds_bytes(a.nw, RG);
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void *)assemble_kernel<RG, NT>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((assemble_kernel<RG, NT>), dim3(ntasks), dim3(kWave * a.nw), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_assemble(int rg, const AsmArgs &a, int ntasks, hipStream_t s) {
    switch (rg) {
        case 8: return launch_variant<8, 1024>(a, ntasks, s);
        case 16: return launch_variant<16, 1024>(a, ntasks, s);
        case 24: return launch_variant<24, 1024>(a, ntasks, s);
        case 52: return launch_variant<52, 512>(a, ntasks, s);
        default: return launch_variant<64, 512>(a, ntasks, s);
    }
}

template <typename T>
int alloc(T **p, size_t count) {
    if (count == 0) count = 1;
    if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(RT_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) +
                                   " bytes for the dense assembly failed");
    }
    return RT_OK;
}

// Plan the assembly once per handle: frequency groups of RG rays per
// wavefront (the fewest slices, then the smallest RG), wavefronts per
// workgroup, the task list (longest walks first) and the workspace.
int plan_assembly(rt_handle *h, hipStream_t s) {
    if (h->d_asm_task) return RT_OK;
    // the fewest slices, then the fewest empty ray slots, then the smaller variant
    int best_rg = 0, best_slices = 0, best_nw = 0;
    long long best_waste = 0;
    for (const AsmVariant &v : kVariants) {
        const int maxw = v.nt / kWave;
        const int cpm = (h->n_nu + v.rg - 1) / v.rg;
        const int chunks = h->M * cpm;
        const int slices = (chunks + maxw - 1) / maxw;
        const int nw = (chunks + slices - 1) / slices;
        const long long waste = (long long)slices * nw * v.rg - (long long)h->M * h->n_nu;
        if (!best_rg || slices < best_slices || (slices == best_slices && waste < best_waste)) {
            best_rg = v.rg;
            best_slices = slices;
            best_nw = nw;
            best_waste = waste;
        }
    }
    h->asm_rg = best_rg;
    h->asm_cpm = (h->n_nu + best_rg - 1) / best_rg;
    h->asm_slices = best_slices;
    h->asm_nw = best_nw;
    std::vector<AsmTask> tasks;
    for (int a = 0; a < h->n_atm; ++a)
        for (int d = 0; d < 2; ++d)
            for (int jb = 0; jb * kWave < h->ns[a]; ++jb)
                for (int sl = 0; sl < best_slices; ++sl) tasks.push_back(AsmTask{a, d, jb, sl});
    std::stable_sort(tasks.begin(), tasks.end(), [&](const AsmTask &x, const AsmTask &y) {
        return h->ns[x.atm] - kWave * x.jblk > h->ns[y.atm] - kWave * y.jblk;
    });
    h->asm_tasks = (int)tasks.size();
    int rc;
    // the task list is set on the handle last: it marks the plan as made, so
    // a failure frees whatever this call allocated and a later call starts over
    AsmTask *dt = nullptr;
    auto undo = [&](int code) {
        for (void **q : {(void **)&dt, (void **)&h->d_ew, (void **)&h->d_asm_dg,
                         (void **)&h->d_asm_sc}) {
            if (*q) (void)hipFree(*q);
            *q = nullptr;
        }
        return code;
    };
    if ((rc = alloc(&dt, tasks.size())) != RT_OK) return undo(rc);
    if (hipMemcpy(dt, tasks.data(), tasks.size() * sizeof(AsmTask), hipMemcpyHostToDevice) !=
        hipSuccess)
        return undo(fail(RT_EDEVICE, "assembly task upload failed"));
    if ((rc = alloc(&h->d_ew, (size_t)h->n_ew)) != RT_OK) return undo(rc);
    if ((rc = alloc(&h->d_asm_dg, (size_t)best_slices * 2 * h->ns_total * 3)) != RT_OK)
        return undo(rc);
    if (best_slices > 1 &&
        (rc = alloc(&h->d_asm_sc, (size_t)(best_slices - 1) * h->n_dense)) != RT_OK)
        return undo(rc);
    h->d_asm_task = dt;
    int ns_max_m1 = 1;
    for (int n : h->ns) ns_max_m1 = std::max(ns_max_m1, n - 1);
    const long long per = (long long)ns_max_m1 * h->M * h->n_nu;
    const dim3 grid((unsigned)std::min<long long>((per + 255) / 256, 4096), h->n_atm);
    hipLaunchKernelGGL(ew_table_kernel, grid, dim3(256), 0, s, h->d_atm, h->d_tau, h->d_opac,
                       h->d_mu_pos, h->M, h->n_nu, h->fs, h->d_ew);
    if (hipGetLastError() != hipSuccess) return fail(RT_EDEVICE, "assembly coefficient launch failed");
    return RT_OK;
}

}  // namespace

int assemble(rt_handle *h, double *A, hipStream_t s) {
    int rc = plan_assembly(h, s);
    if (rc != RT_OK) return rc;
    AsmArgs g{};
    g.atm = h->d_atm;
    g.task = static_cast<const AsmTask *>(h->d_asm_task);
    g.ew = h->d_ew;
    g.rayc = h->d_rayc;
    g.dirc = h->d_dirc;
    g.A = A;
    g.sc = h->d_asm_sc;
    g.sc_stride = h->n_dense;
    g.dg = h->d_asm_dg;
    g.ns_total = h->ns_total;
    g.n_nu = h->n_nu;
    g.M = h->M;
    g.cpm = h->asm_cpm;
    g.nw = h->asm_nw;
    g.slices = h->asm_slices;
    if (launch_assemble(h->asm_rg, g, h->asm_tasks, s) != hipSuccess)
        return fail(RT_EDEVICE, "assembly launch failed");
    if (g.slices > 1) {
        long long nsq = 1;
        for (int n : h->ns) nsq = std::max(nsq, (long long)n * n);
        const dim3 grid((unsigned)std::min<long long>((nsq + 255) / 256, 4096), h->n_atm);
        hipLaunchKernelGGL(assemble_combine_kernel, grid, dim3(256), 0, s, g);
        if (hipGetLastError() != hipSuccess) return fail(RT_EDEVICE, "assembly combine launch failed");
    }
    hipLaunchKernelGGL(assemble_diag_kernel, dim3((h->ns_total + 255) / 256), dim3(256), 0, s, g,
                       (const int *)h->d_pt_atm);
    if (hipGetLastError() != hipSuccess) return fail(RT_EDEVICE, "assembly diagonal launch failed");
    return RT_OK;
}

}  // namespace rt
