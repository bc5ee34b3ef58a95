// rt_sweep_kernel.h -- the fused T + Lambda + J sweep (device templates).
//
// Included by the translation units that instantiate it for one arithmetic
// type each (rt_sweep_f32.hip, rt_sweep_f64.hip), so the many compiled
// variants build in parallel.
//
// T: arithmetic type of the recurrences and accumulators (double, or float
// inside the mixed-precision inner solve).  L: the longest chunk of the plan.
// A block runs the body compiled for its slab's chunk count C (8, 16, 32 or
// 64) and chunk length LE (one of the lengths chunk_len allows for L): every
// loop over a chunk and every lane-scan level is straight-line code.  W: waves
// per block.  PF: 1 = the next ray batch of a wave is loaded while the
// current one is computed.  CM: where a step's coefficients (E, w) come from
// (kCoefPairs: both streamed from the tiles; kCoefW: w streamed, E = 1 - w d
// derived; kCoefRecompute: both computed from d), d = kappa dtau the optical
// step of the interval, kappa = r_p / |mu| per ray, dtau per interval.  Each
// block writes the 2 ns quadrature sums of its rays to its own slot of
// `partial`; the finalize pass adds the slots of a slab in block order and
// applies sigma_out = z - xi [J00, W2 J20].
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "rt_internal.h"

namespace rt {
namespace sweep {

template <typename T>
struct Pair;
template <>
struct Pair<double> {
    using type = double2;
};
template <>
struct Pair<float> {
    using type = float2;
};

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRawBufferWord3 = 0x00020000;  // gfx9 buffer descriptor: raw 32-bit data

__device__ inline void load_pair(__amdgpu_buffer_rsrc_t r, int voff, int soff, float2 &o) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    o.x = __uint_as_float(v.x);
    o.y = __uint_as_float(v.y);
}
__device__ inline void load_pair(__amdgpu_buffer_rsrc_t r, int voff, int soff, double2 &o) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    o.x = __hiloint2double((int)v.y, (int)v.x);
    o.y = __hiloint2double((int)v.w, (int)v.z);
}
__device__ inline double load_f64(__amdgpu_buffer_rsrc_t r, int voff) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0);
    return __hiloint2double((int)v.y, (int)v.x);
}
// single coefficients (the w-only tiles)
__device__ inline void load_pair(__amdgpu_buffer_rsrc_t r, int voff, int soff, float &o) {
    o = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ inline void load_pair(__amdgpu_buffer_rsrc_t r, int voff, int soff, double &o) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    o = __hiloint2double((int)v.y, (int)v.x);
}
__device__ inline double2 load_f64x2(__amdgpu_buffer_rsrc_t r, int voff) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
    return make_double2(__hiloint2double((int)v.y, (int)v.x), __hiloint2double((int)v.w, (int)v.z));
}

// --------------------------------------------------------------------------
// Step coefficients computed in the sweep (kCoefRecompute), from the optical
// step d of the interval and its reciprocal rd.  Every formal solver here
// has w = (1 - E) / d:
//   DELO-linear  E = e^{-d},               w = (1 - e^{-d}) / d;
//   trapezoidal  E = (1 - d/2)/(1 + d/2),  w = 1 / (1 + d/2);
//   implicit Euler E = w = 1 / (1 + d).
// Below d = 0.1 the DELO-linear w comes from its Taylor series
// sum_{n>=0} (-d)^n / (n+1)!, 6 terms in FP32 and 11 in FP64 (the first
// omitted term is below 3e-10 and 3e-20 relative there).
// --------------------------------------------------------------------------
template <typename T>
struct WSeries;
template <>
struct WSeries<float> {
    static constexpr int n = 6;
};
template <>
struct WSeries<double> {
    static constexpr int n = 11;
};
struct WSeriesCoef {
    double c[12];
};
constexpr WSeriesCoef make_w_series() {
    WSeriesCoef s{};
    double fact = 1.0;  // (n + 1)!
    for (int n = 0; n < 12; ++n) {
        fact *= (n + 1);
        s.c[n] = ((n % 2 == 0) ? 1.0 : -1.0) / fact;
    }
    return s;
}
constexpr WSeriesCoef c_w_series = make_w_series();

__device__ inline float exp_neg(float d) { return __expf(-d); }
__device__ inline double exp_neg(double d) { return exp(-d); }
__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double recip(double x) { return 1.0 / x; }

template <typename T>
__device__ inline void delo_ew(T d, T rd, T &E, T &w) {
    constexpr int n = WSeries<T>::n;
    T s = (T)c_w_series.c[n - 1];
#pragma unroll
    for (int t = n - 2; t >= 0; --t) s = fma(s, d, (T)c_w_series.c[t]);
    E = exp_neg(d);
    const T big = ((T)1 - E) * rd;
    w = d < (T)0.1 ? s : big;
}

// --------------------------------------------------------------------------
// Cross-lane moves.  DPP (data-parallel primitives) move a register between
// lanes inside the VALU: row_shr:d / row_shl:d shift within rows of 16 lanes,
// row_bcast:15 / :31 broadcast lane 15 of a row (lane 31) to the next row(s),
// row_newbcast:15 broadcasts lane 15 of a row over the same row, wave_shr:1 /
// wave_shl:1 shift the whole wave by one lane.  Lanes with no source lane,
// and rows outside ROWS, receive `old`.
// --------------------------------------------------------------------------
constexpr int kRowShr = 0x110, kRowShl = 0x100, kWaveShr1 = 0x138, kWaveShl1 = 0x130,
              kRowBcast15 = 0x142, kRowBcast31 = 0x143, kRowNewBcast15 = 0x15F;

template <int CTRL, int ROWS>
__device__ inline float dpp(float v, float old) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ inline double dpp(double v, double old) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROWS,
                                               0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROWS,
                                               0xF, false);
    return __hiloint2double(hi, lo);
}
// As dpp, for values whose lanes without a source are never used (no old
// value to set up).
template <int CTRL>
__device__ inline float dpp_any(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ inline double dpp_any(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ inline float read_lane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double read_lane(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// A chunk's map x -> P x + (U, V) preceded by the map (pP, pU, pV) of the
// chunks the radiation crosses before it.
template <typename T>
__device__ inline void compose(T &P, T &U, T &V, T pP, T pU, T pV) {
    U = fma(P, pU, U);
    V = fma(P, pV, V);
    P = P * pP;
}
template <int CTRL, int ROWS, typename T>
__device__ inline void scan_level(T &P, T &U, T &V) {
    compose(P, U, V, dpp<CTRL, ROWS>(P, (T)1), dpp<CTRL, ROWS>(U, (T)0),
            dpp<CTRL, ROWS>(V, (T)0));
}

// Compose with the map held by (sP, sU, sV) in the lane CTRL points to.
template <int CTRL, int ROWS, typename T>
__device__ inline void scan_level_from(T &P, T &U, T &V, T sP, T sU, T sV) {
    compose(P, U, V, dpp<CTRL, ROWS>(sP, (T)1), dpp<CTRL, ROWS>(sU, (T)0),
            dpp<CTRL, ROWS>(sV, (T)0));
}

// The same level in FP32 as three DPP-sourced VALU operations: the neighbour's
// U, V and P are read through the DPP operand, and lanes with no source lane
// (or in rows not enabled) are not written, i.e. keep their own map, which is
// the composition with the identity.  The leading s_nop covers the wait
// states a DPP read needs after a VALU write of its source (2) or of EXEC
// (5); the trailing one covers a DPP read of the outputs right after.
#define RT_DPP_SCAN_F32(P, U, V, CTL)                                     \
    asm("s_nop 4\n\t"                                                     \
        "v_fmac_f32_dpp %1, %1, %0 " CTL "\n\t"                           \
        "v_fmac_f32_dpp %2, %2, %0 " CTL "\n\t"                           \
        "v_mul_f32_dpp %0, %0, %0 " CTL "\n\t"                            \
        "s_nop 1"                                                         \
        : "+v"(P), "+v"(U), "+v"(V))

template <int CTRL, int ROWS>
__device__ inline void scan_level(float &P, float &U, float &V) {
    if constexpr (CTRL == kRowShr + 1) RT_DPP_SCAN_F32(P, U, V, "row_shr:1 row_mask:0xf bank_mask:0xf");
    else if constexpr (CTRL == kRowShr + 2) RT_DPP_SCAN_F32(P, U, V, "row_shr:2 row_mask:0xf bank_mask:0xf");
    else if constexpr (CTRL == kRowShr + 4) RT_DPP_SCAN_F32(P, U, V, "row_shr:4 row_mask:0xf bank_mask:0xf");
    else if constexpr (CTRL == kRowShr + 8) RT_DPP_SCAN_F32(P, U, V, "row_shr:8 row_mask:0xf bank_mask:0xf");
    else if constexpr (CTRL == kRowShl + 1) RT_DPP_SCAN_F32(P, U, V, "row_shl:1 row_mask:0xf bank_mask:0xf");
    else if constexpr (CTRL == kRowShl + 2) RT_DPP_SCAN_F32(P, U, V, "row_shl:2 row_mask:0xf bank_mask:0xf");
    else if constexpr (CTRL == kRowShl + 4) RT_DPP_SCAN_F32(P, U, V, "row_shl:4 row_mask:0xf bank_mask:0xf");
    else if constexpr (CTRL == kRowShl + 8) RT_DPP_SCAN_F32(P, U, V, "row_shl:8 row_mask:0xf bank_mask:0xf");
    else if constexpr (CTRL == kRowBcast15 && ROWS == 0xA) RT_DPP_SCAN_F32(P, U, V, "row_bcast:15 row_mask:0xa bank_mask:0xf");
    else if constexpr (CTRL == kRowBcast31 && ROWS == 0xC) RT_DPP_SCAN_F32(P, U, V, "row_bcast:31 row_mask:0xc bank_mask:0xf");
    else static_assert(CTRL < 0, "no FP32 scan level for this DPP control");
}
template <>
__device__ inline void scan_level_from<kRowNewBcast15, 0x5, float>(float &P, float &U, float &V,
                                                                  float sP, float sU, float sV) {
    asm("s_nop 4\n\t"
        "v_fmac_f32_dpp %1, %4, %0 row_newbcast:15 row_mask:0x5 bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %5, %0 row_newbcast:15 row_mask:0x5 bank_mask:0xf\n\t"
        "v_mul_f32_dpp %0, %3, %0 row_newbcast:15 row_mask:0x5 bank_mask:0xf\n\t"
        "s_nop 1"
        : "+v"(P), "+v"(U), "+v"(V)
        : "v"(sP), "v"(sU), "v"(sV));
}
#undef RT_DPP_SCAN_F32

// Inclusive scans over the C chunks of every ray of the wave (lane layout of
// lane_chunk): forward, the lane of chunk c ends with the map of chunks 0..c
// (downward rays); backward, with the map of chunks c..C-1 (upward rays).
// Row shifts by 1, 2, 4, 8 lanes are chunk shifts by 1, 2, 4, 8 / s.
template <int C, typename T>
__device__ inline void scan_forward(T &P, T &U, T &V) {
    if constexpr (C >= 16) scan_level<kRowShr + 1, 0xF>(P, U, V);
    if constexpr (C >= 8) scan_level<kRowShr + 2, 0xF>(P, U, V);
    if constexpr (C >= 4) scan_level<kRowShr + 4, 0xF>(P, U, V);
    if constexpr (C >= 2) scan_level<kRowShr + 8, 0xF>(P, U, V);
    if constexpr (C >= 32) scan_level<kRowBcast15, 0xA>(P, U, V);  // rows 1, 3 <- lane 15 of 0, 2
    if constexpr (C == 64) scan_level<kRowBcast31, 0xC>(P, U, V);  // rows 2, 3 <- lane 31
}
template <int C, typename T>
__device__ inline void scan_backward(T &P, T &U, T &V, int lane) {
    if constexpr (C >= 16) scan_level<kRowShl + 1, 0xF>(P, U, V);
    if constexpr (C >= 8) scan_level<kRowShl + 2, 0xF>(P, U, V);
    if constexpr (C >= 4) scan_level<kRowShl + 4, 0xF>(P, U, V);
    if constexpr (C >= 2) scan_level<kRowShl + 8, 0xF>(P, U, V);
    if constexpr (C >= 32) {
        // rows 0 and 2 take the first lane of rows 1 and 3: the wave shifted
        // left by one lane puts lanes 16 and 48 at lanes 15 and 47, which are
        // then broadcast over rows 0 and 2 (only those two lanes of the shift
        // are read, and both have a source)
        scan_level_from<kRowNewBcast15, 0x5>(P, U, V, dpp_any<kWaveShl1>(P), dpp_any<kWaveShl1>(U),
                                             dpp_any<kWaveShl1>(V));
    }
    if constexpr (C == 64) {  // lanes 0..31 take lane 32
        const T rP = read_lane(P, 32), rU = read_lane(U, 32), rV = read_lane(V, 32);
        const bool lo = lane < 32;
        compose(P, U, V, lo ? rP : (T)1, lo ? rU : (T)0, lo ? rV : (T)0);
    }
}

// The value held by chunk c - 1 (from_prev) or c + 1 (from_next) of the same
// ray; `old` where there is no such chunk.
template <int C, typename T>
__device__ inline T from_prev(T v, T old, int c) {
    if constexpr (C >= 32) {
        const T x = dpp<kWaveShr1, 0xF>(v, old);
        return c == 0 ? old : x;
    } else {
        return dpp<kRowShr + 16 / C, 0xF>(v, old);
    }
}
template <int C, typename T>
__device__ inline T from_next(T v, T old, int c) {
    if constexpr (C >= 32) {
        const T x = dpp<kWaveShl1, 0xF>(v, old);
        return c == C - 1 ? old : x;
    } else {
        return dpp<kRowShl + 16 / C, 0xF>(v, old);
    }
}

// One wave's share of a block: the ray batches wb_first + wave + t * W of
// direction bd.m of slab bd.atm, whose chunk count is C and chunk length LE.
template <typename T, int LE, int C, int W, int PF, int CM>
__device__ __forceinline__ void sweep_rays(const SweepArgs &a, const BlockDesc &bd,
                                           const AtmDesc &at, int wave, int lane, T *sacc,
                                           const T *src) {
    using P2 = typename Pair<T>::type;
    // one tile entry: the (E, w) pair, or w alone
    using Ent = typename std::conditional<CM == kCoefPairs, P2, T>::type;
    const int ns = at.ns;
    const int c = lane_chunk(lane, C), g = lane_slot(lane, C);
    // the chunk: first depth point s0, len = LE or LE - 1 intervals (a short
    // chunk's step LE - 1 is the zero-length identity: its end point repeats)
    const int nlong = at.nlong;
    const bool longc = c < nlong;
    const int s0 = c * (LE - 1) + min(c, nlong);
    const int len = longc ? LE : LE - 1;

    // The sweep carries the deviation D = I - S of the intensity from the
    // local source: with E + c_u = 1 - c_k = w the step becomes
    //   D_k = E D_u + w (S_u - S_k),
    // which only accumulates differences of the source, so its rounding stays
    // small against J even where I ~ S (thermalized layers, the FP32 sweep of
    // the mixed-precision solve).  The source part sum q S is added exactly,
    // in FP64, by the finalize pass.
    //
    // Sources s00, s20 at the chunk's points from the block's copy in LDS
    // (zero past the slab); dl[i] = S(point i) - S(point i + 1); top/bottom:
    // sources at the slab's first and last point, for the boundary deviations.
    T dl0[LE], dl2[LE];
    {
        const P2 *src2 = reinterpret_cast<const P2 *>(src);
        P2 sv[LE + 1];
#pragma unroll
        for (int i = 0; i <= LE; ++i) {
            const int k = s0 + min(i, len);
            sv[i] = src2[min(k, ns - 1)];
            if (k >= ns) sv[i].x = sv[i].y = (T)0;
        }
#pragma unroll
        for (int i = 0; i < LE; ++i) {
            dl0[i] = sv[i].x - sv[i + 1].x;
            dl2[i] = sv[i].y - sv[i + 1].y;
        }
    }
    const T top0 = src[0], top2 = src[1], bot0 = src[2 * (ns - 1)], bot2 = src[2 * (ns - 1) + 1];

    // the optical-depth steps dtau of the chunk's intervals (and their
    // reciprocals), for the modes that derive coefficients: zero for the
    // zero-length step of a short chunk and for steps past the bottom, whose
    // d = 0 makes them the identity (E = w = 1)
    T dt[LE], rdt[LE];
    if constexpr (CM != kCoefPairs) {
#pragma unroll
        for (int i = 0; i < LE; ++i) {
            const int j = s0 + i;
            const bool on = i < len && j < ns - 1;
            dt[i] = on ? (T)a.dtau[at.doff + min(j, ns - 2)] : (T)0;
            if constexpr (CM == kCoefRecompute) rdt[i] = on ? (T)1 / dt[i] : (T)0;
        }
    }

    // AU = sum_rays q (D from s00), AV = sum_rays q (D from s20), by point;
    // every ray of the block has the same direction, so the T factors are
    // applied once at the end
    T AU[LE + 1], AV[LE + 1];
#pragma unroll
    for (int i = 0; i <= LE; ++i) AU[i] = AV[i] = (T)0;

    // deviations entering the slab: I = 0 at the top; I = Ibot (right-hand
    // side) or 0 (operator) at the bottom, whose entry point is the last
    // chunk's end point -- a point of the slab or past it (source zero)
    const T inflow = (a.mode == 1) ? (T)at.Ibot : (T)0;
    const T topD0 = -top0, topD2 = -top2;
    const bool bottom_on_grid = C * (LE - 1) + nlong == ns - 1;
    const T botD0 = inflow - (bottom_on_grid ? bot0 : (T)0);
    const T botD2 = -(bottom_on_grid ? bot2 : (T)0);
    // the top point's downward deviation is the top inflow's; a bottom point
    // that ends the last chunk has the bottom inflow's upward deviation
    const T ftop = (c == 0) ? (T)1 : (T)0;
    const T fbot = (c == C - 1 && bottom_on_grid) ? (T)1 : (T)0;

    // this direction's tiles and ray weights, read through buffer
    // descriptors that end at the block's last batch: a load of a batch past
    // it (the prefetch beyond a wave's last batch) returns zeros and fetches
    // nothing, so every load is unconditional and the compiler can keep the
    // next batch's loads in flight across the current batch's work.  Batch
    // and lane offsets in a register, the step offset in a scalar register.
    const int bend = bd.wb_first + bd.wb_count;
    const int bbytes = at.bstride * (int)sizeof(Ent);  // one wave-batch of tile entries
    const Ent *tiles = reinterpret_cast<const Ent *>(a.coef) + at.coef_off +
                       (long long)bd.m * at.nwb * at.bstride;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)tiles, 0, CM == kCoefRecompute ? 0 : bend * bbytes, kRawBufferWord3);
    const long long rdir = at.q_off + (long long)bd.m * at.nwb * at.G;
    const __amdgpu_buffer_rsrc_t qrsrc =
        __builtin_amdgcn_make_buffer_rsrc((void *)(a.q + rdir), 0, bend * at.G * 8, kRawBufferWord3);
    // per ray (kappa, 1 / kappa), laid out as the weights; zero for padding rays
    const double2 *kdir = CM == kCoefPairs ? reinterpret_cast<const double2 *>(a.q) : a.kt + rdir;
    const __amdgpu_buffer_rsrc_t krsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)kdir, 0, CM == kCoefPairs ? 0 : bend * at.G * 16, kRawBufferWord3);
    const int voff = lane * (int)sizeof(Ent);
    // the packed last step: short chunks read from past the descriptor's
    // range (zeros, no memory access) and take the identity below
    constexpr int kNoLoad = 1 << 30;
    const int voff_last =
        longc ? ((LE - 1) * kWave + g * nlong + c) * (int)sizeof(Ent) : kNoLoad;

    auto load_batch = [&](int b, Ent (&cn)[LE], double &qn, double2 &kn) {
        if constexpr (CM != kCoefRecompute) {
            const int vo = voff + b * bbytes;
#pragma unroll
            for (int i = 0; i + 1 < LE; ++i)
                load_pair(rsrc, vo, i * kWave * (int)sizeof(Ent), cn[i]);
            load_pair(rsrc, voff_last + b * bbytes, 0, cn[LE - 1]);
        }
        qn = load_f64(qrsrc, (b * at.G + g) * 8);
        if constexpr (CM == kCoefW) kn.x = load_f64(krsrc, (b * at.G + g) * 16);
        if constexpr (CM == kCoefRecompute) kn = load_f64x2(krsrc, (b * at.G + g) * 16);
    };

    auto process = [&](Ent (&cn)[LE], double qd, double2 kd) {
        const T q = (T)qd;
        // the steps' (E, w)
        T Es[LE], ws[LE];
        if constexpr (CM == kCoefPairs) {
#pragma unroll
            for (int i = 0; i < LE; ++i) {
                Es[i] = cn[i].x;
                ws[i] = cn[i].y;
            }
            if (!longc) Es[LE - 1] = ws[LE - 1] = (T)1;  // zero-length step
        } else if constexpr (CM == kCoefW) {
            const T kap = (T)kd.x;
#pragma unroll
            for (int i = 0; i < LE; ++i) ws[i] = cn[i];
            if (!longc) ws[LE - 1] = (T)1;  // zero-length step (its d is 0)
#pragma unroll
            for (int i = 0; i < LE; ++i) Es[i] = fma(-ws[i], kap * dt[i], (T)1);
        } else {
            const T kap = (T)kd.x, rkap = (T)kd.y;
            if (a.fs == RT_FS_DELO_LINEAR) {
#pragma unroll
                for (int i = 0; i < LE; ++i) delo_ew(kap * dt[i], rkap * rdt[i], Es[i], ws[i]);
            } else if (a.fs == RT_FS_TRAPEZOIDAL) {
#pragma unroll
                for (int i = 0; i < LE; ++i) {
                    const T d = kap * dt[i];
                    ws[i] = recip(fma((T)0.5, d, (T)1));
                    Es[i] = fma(-ws[i], d, (T)1);
                }
            } else {  // implicit Euler
#pragma unroll
                for (int i = 0; i < LE; ++i) Es[i] = ws[i] = recip(fma(kap, dt[i], (T)1));
            }
        }
        // one pass over the chunk with zero inflow in both directions: the
        // local deviations go into the quadrature at once.  p = w (S_u - S_k)
        // is formed once per step and source and serves both directions; the
        // running transmissions Td[i] = E_0..E_i, Tu[i] = E_i..E_{LE-1} are
        // kept for the inflow term added after the scan
        T p0[LE], p2[LE], Td[LE], Tu[LE];
#pragma unroll
        for (int i = 0; i < LE; ++i) {
            p0[i] = ws[i] * dl0[i];
            p2[i] = ws[i] * dl2[i];
        }
        T dU = p0[0], dV = p2[0];
        Td[0] = Es[0];
        AU[1] = fma(q, dU, AU[1]);
        AV[1] = fma(q, dV, AV[1]);
#pragma unroll
        for (int i = 1; i < LE; ++i) {
            dU = fma(Es[i], dU, p0[i]);
            dV = fma(Es[i], dV, p2[i]);
            Td[i] = Td[i - 1] * Es[i];
            AU[i + 1] = fma(q, dU, AU[i + 1]);
            AV[i + 1] = fma(q, dV, AV[i + 1]);
        }
        T uU = -p0[LE - 1], uV = -p2[LE - 1];
        Tu[LE - 1] = Es[LE - 1];
        AU[LE - 1] = fma(q, uU, AU[LE - 1]);
        AV[LE - 1] = fma(q, uV, AV[LE - 1]);
#pragma unroll
        for (int i = LE - 2; i >= 0; --i) {
            uU = fma(Es[i], uU, -p0[i]);
            uV = fma(Es[i], uV, -p2[i]);
            Tu[i] = Tu[i + 1] * Es[i];
            AU[i] = fma(q, uU, AU[i]);
            AV[i] = fma(q, uV, AV[i]);
        }

        // lane scans of the chunk maps D_out = P D_in + e: downward chunks
        // compose in chunk order, upward ones in reverse order
        T Pd = Td[LE - 1], Pu = Tu[0];
        scan_forward<C>(Pd, dU, dV);
        scan_backward<C>(Pu, uU, uV, lane);
        // deviations at the chunk's entry points: the boundary deviation
        // carried through the chunks above (down) or below (up) -- the value
        // at the end of the neighbouring chunk -- or the boundary's own
        const T qdU = q * from_prev<C, T>(fma(Pd, topD0, dU), topD0, c);
        const T qdV = q * from_prev<C, T>(fma(Pd, topD2, dV), topD2, c);
        const T quU = q * from_next<C, T>(fma(Pu, botD0, uU), botD0, c);
        const T quV = q * from_next<C, T>(fma(Pu, botD2, uV), botD2, c);

        // inflow terms: D_true = D_local + T * D_in at every point of the chunk
#pragma unroll
        for (int i = 0; i < LE; ++i) {
            AU[i + 1] = fma(Td[i], qdU, AU[i + 1]);
            AV[i + 1] = fma(Td[i], qdV, AV[i + 1]);
            AU[i] = fma(Tu[i], quU, AU[i]);
            AV[i] = fma(Tu[i], quV, AV[i]);
        }
        AU[0] = fma(ftop, qdU, AU[0]);
        AV[0] = fma(ftop, qdV, AV[0]);
        AU[LE] = fma(fbot, quU, AU[LE]);
        AV[LE] = fma(fbot, quV, AV[LE]);
    };

    const int b0 = bd.wb_first + wave;
    if constexpr (PF == 0) {
        for (int b = b0; b < bend; b += W) {
            Ent cn[LE];
            double qn;
            double2 kn = make_double2(0.0, 0.0);
            load_batch(b, cn, qn, kn);
            process(cn, qn, kn);
        }
    } else {
        // two register sets, each loaded one batch ahead of its use
        Ent cA[LE], cB[LE];
        double qA, qB;
        double2 kA = make_double2(0.0, 0.0), kB = kA;
        load_batch(b0, cA, qA, kA);
        for (int b = b0; b < bend; b += 2 * W) {
            load_batch(b + W, cB, qB, kB);
            process(cA, qA, kA);
            if (b + W >= bend) break;
            load_batch(b + 2 * W, cA, qA, kA);
            process(cB, qB, kB);
        }
    }

    // sum over the rays of the wave that share chunk c: lanes that differ in
    // the slot bits (above the chunk bits for C >= 16; the low log2(16 / C)
    // bits and the row bits otherwise)
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const bool slot_bit = (C >= 16) ? (off >= C) : (off < 16 / C || off >= 16);
        if (slot_bit) {
#pragma unroll
            for (int i = 0; i <= LE; ++i) {
                AU[i] += __shfl_xor(AU[i], off);
                AV[i] += __shfl_xor(AV[i], off);
            }
        }
    }
    // the downward value at a chunk's end point belongs to the next chunk's first point
    AU[0] += from_prev<C>(AU[LE], (T)0, c);
    AV[0] += from_prev<C>(AV[LE], (T)0, c);
    const T bU = AU[LE], bV = AV[LE];

    // J00 = AU + T1 AV, J20 = T1 AU + (T1^2 + T2^2) AV for this direction
    const double2 tf = a.dirc[bd.m];
    const T t1 = (T)tf.x, t12 = (T)tf.y;

    // block totals of the 2 ns quadrature sums, stored in the sweep's type
    // (an FP32 sweep's sums are FP32 values: half the bytes, the same numbers)
    const int nthr = kWave * W;
    T *mine = reinterpret_cast<T *>(a.partial) + at.part_off + (long long)bd.slot * 2 * ns;
    if (a.rows) {
        // one LDS row per wave, then a fixed-order sum over the rows
        T *row = sacc + (long long)wave * 2 * ns;
        if (g == 0) {
#pragma unroll
            for (int i = 0; i < LE; ++i) {
                const int k = s0 + i;
                if (k < ns && i < len) {
                    row[2 * k] = AU[i] + t1 * AV[i];
                    row[2 * k + 1] = t1 * AU[i] + t12 * AV[i];
                }
            }
            if (c == C - 1 && bottom_on_grid) {
                row[2 * (ns - 1)] = bU + t1 * bV;
                row[2 * (ns - 1) + 1] = t1 * bU + t12 * bV;
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 2 * ns; e += nthr) {
            T s = sacc[e];
            for (int w = 1; w < W; ++w) s += sacc[(long long)w * 2 * ns + e];
            mine[e] = s;
        }
    } else {
        // one shared row, filled wave after wave (fixed order)
        for (int e = threadIdx.x; e < 2 * ns; e += nthr) sacc[e] = (T)0;
        __syncthreads();
        for (int w = 0; w < W; ++w) {
            if (wave == w && g == 0) {
#pragma unroll
                for (int i = 0; i < LE; ++i) {
                    const int k = s0 + i;
                    if (k < ns && i < len) {
                        sacc[2 * k] += AU[i] + t1 * AV[i];
                        sacc[2 * k + 1] += t1 * AU[i] + t12 * AV[i];
                    }
                }
                if (c == C - 1 && bottom_on_grid) {
                    sacc[2 * (ns - 1)] += bU + t1 * bV;
                    sacc[2 * (ns - 1) + 1] += t1 * bU + t12 * bV;
                }
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < 2 * ns; e += nthr) mine[e] = sacc[e];
    }
}

template <typename T, int L, int W, int PF, int CM, int LE, int C>
__device__ __forceinline__ void dispatch_c(const SweepArgs &a, const BlockDesc &bd,
                                           const AtmDesc &at, int wave, int lane, T *sacc,
                                           const T *src) {
    if constexpr (C <= kWave) {
        if (at.C == C) {
            sweep_rays<T, LE, C, W, PF, CM>(a, bd, at, wave, lane, sacc, src);
            return;
        }
        dispatch_c<T, L, W, PF, CM, LE, 2 * C>(a, bd, at, wave, lane, sacc, src);
    }
}
template <typename T, int L, int W, int PF, int CM, int LE>
__device__ __forceinline__ void dispatch_le(const SweepArgs &a, const BlockDesc &bd,
                                            const AtmDesc &at, int wave, int lane, T *sacc,
                                            const T *src) {
    if constexpr (LE <= L) {
        if (at.Leff == LE) {
            dispatch_c<T, L, W, PF, CM, LE, kMinChunks>(a, bd, at, wave, lane, sacc, src);
            return;
        }
        dispatch_le<T, L, W, PF, CM, LE + chunk_len_step(L)>(a, bd, at, wave, lane, sacc, src);
    }
}

// Waves per SIMD the register allocation is held to, for the bodies of chunk
// length 8 that stream w: 5 in FP32 (96 registers, a handful spilled) and 3
// in FP64 (168 registers, about 20 spilled; left alone it takes 244 and runs
// two waves per SIMD, 3-6% slower).  The recomputing bodies would spill more.
template <typename T, int L, int CM>
struct MinWaves {
    static constexpr int value =
        (L == 8 && CM == kCoefW) ? (sizeof(T) == 4 ? 5 : 3) : 1;
};

// LDS: the quadrature rows (a.rows ? W : 1) x 2 ns_max values of type T, then
// the slab's sources (2 ns values of type T, scaled) at byte a.src_lds.
template <typename T, int L, int W, int PF, int CM>
__global__ __launch_bounds__(kWave *W)
__attribute__((amdgpu_waves_per_eu(MinWaves<T, L, CM>::value, 8))) void sweep_kernel(SweepArgs a) {
    extern __shared__ unsigned char smem_raw[];
    const BlockDesc bd = a.blk[blockIdx.x];
    if (a.mask && a.mask[bd.atm] == 0) return;  // uniform over the block
    const AtmDesc at = a.atm[bd.atm];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    T *src = reinterpret_cast<T *>(smem_raw + a.src_lds);
    {
        // the slab's sources z = scale .* sigma_in in type T (zero: no source)
        const long long vbase = 2LL * at.doff;
        for (int k = threadIdx.x; k < at.ns; k += kWave * W) {
            double2 v = make_double2(0.0, 0.0);
            if (a.sig_in) {
                v = *reinterpret_cast<const double2 *>(a.sig_in + vbase + 2LL * k);
                if (a.scale) {
                    const double2 sc = *reinterpret_cast<const double2 *>(a.scale + vbase + 2LL * k);
                    v.x *= sc.x;
                    v.y *= sc.y;
                }
            }
            src[2 * k] = (T)v.x;
            src[2 * k + 1] = (T)v.y;
        }
        __syncthreads();
    }
    dispatch_le<T, L, W, PF, CM, chunk_len_min(L)>(a, bd, at, wave, lane,
                                                   reinterpret_cast<T *>(smem_raw), src);
}

// Launch for one (T, L, CM): waves per block by register footprint, LDS
// layout, prefetch choice (compiled for the streamed pairs only).
template <typename T, int L, int W, int CM>
hipError_t launch_tw(SweepArgs a, bool pf, int nblocks, int ns_max, hipStream_t s) {
    const size_t row = 2 * (size_t)ns_max * sizeof(T);
    a.rows = ((W + 1) * row <= (size_t)kSweepLdsBudget) ? 1 : 0;
    a.src_lds = (int)(a.rows ? W * row : row);
    const size_t lds = a.src_lds + row;
    if constexpr (L <= 8 && CM == kCoefPairs) {
        if (pf) {
            hipLaunchKernelGGL((sweep_kernel<T, L, W, 1, CM>), dim3(nblocks), dim3(kWave * W), lds,
                               s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((sweep_kernel<T, L, W, 0, CM>), dim3(nblocks), dim3(kWave * W), lds, s, a);
    return hipGetLastError();
}

template <typename T, int L, int CM>
hipError_t launch(const SweepArgs &a, int W, bool pf, int nblocks, int ns_max, hipStream_t s) {
    if constexpr (L <= 8) {
        if (W == 8) return launch_tw<T, L, 8, CM>(a, pf, nblocks, ns_max, s);
    }
    return launch_tw<T, L, 4, CM>(a, pf, nblocks, ns_max, s);
}

// All chunk lengths of one (T, CM).
template <typename T, int CM>
hipError_t launch_any(int L, int W, bool pf, const SweepArgs &a, int nblocks, int ns_max,
                      hipStream_t s) {
    switch (L) {
        case 4: return launch<T, 4, CM>(a, W, pf, nblocks, ns_max, s);
        case 8: return launch<T, 8, CM>(a, W, pf, nblocks, ns_max, s);
        case 16: return launch<T, 16, CM>(a, W, pf, nblocks, ns_max, s);
        case 32: return launch<T, 32, CM>(a, W, pf, nblocks, ns_max, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace sweep
}  // namespace rt
