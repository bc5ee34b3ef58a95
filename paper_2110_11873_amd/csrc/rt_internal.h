// rt_internal.h -- internal types shared by the host runtime and the kernels
// of the gfx950 library behind include/rt.h.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "rt.h"
#include "rt_ext.h"

namespace rt {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kSweepLdsBudget = 64 * 1024;  // bytes of LDS a sweep block may use
constexpr int kKrylovThreads = 256;
constexpr int kKrylovEPT = (2 * RT_MAX_NS + kKrylovThreads - 1) / kKrylovThreads;

// Per-slab launch plan of the formal-solver sweep.  A ray is one (|mu_m|, nu_p)
// pair; its depth recurrence is split into C chunks, one chunk per lane,
// G = 64 / C rays per wavefront ("wave-batch").  The first nlong chunks have
// Leff intervals, the others Leff - 1: a short chunk's last step is a
// zero-length interval (the identity), which is neither stored nor loaded.
// Wave-batches never mix directions: batch b of direction m holds the rays
// p = b*G + g.
struct AtmDesc {
    int ns;         // depth points
    int doff;       // first depth point of the slab in concatenated arrays
    int C;          // chunks per ray (power of two, <= 64)
    int Leff;       // intervals of a long chunk (chunk_len; <= the kernel's L)
    int G;          // rays per wave-batch
    int n_nu;       // frequencies: rays per direction
    int nwb;        // wave-batches per direction
    int ray_off;    // first ray of the slab in the ray tables (rays m*n_nu + p)
    int blk_first;  // first sweep block of the slab
    int nblk;       // sweep blocks of the slab
    int nlong;      // chunks of Leff intervals (the rest have Leff - 1)
    int bstride;    // coefficient pairs per wave-batch: Leff - 1 rows of 64 lanes,
                    // then the long chunks' last steps, packed (padded to 16)
    long long q_off;     // first entry of the slab's tile-ordered weights
    long long coef_off;  // first coefficient pair of the slab's tiles
    long long part_off;  // first partial sum of the slab's blocks
    long long a_off;     // first entry of the slab's block of the assembled A
    long long ew_off;    // first entry of the slab's rows of the assembly coefficient table
    double xi;      // 1 - eps
    double W2;      // polarizability
    double eps;     // thermalization
    double Ibot;    // bottom inflow for mu > 0
};

// One sweep block: direction m of slab atm; wave w of a block of W waves
// handles wave-batches wb_first + w + t * W, t = 0, 1, ..., while below
// wb_first + wb_count, and writes its quadrature sums to partial-sum slot
// `slot` of the slab.  The block list is ordered by decreasing work, so the
// in-order dispatch of workgroups starts the longest ones first.
struct BlockDesc {
    int atm;
    int m;
    int wb_first;
    int wb_count;
    int slot;
    int pad[3];
};

// Quadrature weight of a ray (applied to both directions of the +-mu pair)
// and its products with the T^2_0 factors: q, q T1, q (T1^2 + T2^2).
struct RayConst {
    double q, qt1, qt12, pad;
};

// Where the sweep takes a step's coefficients (E, w) from: both streamed
// from the tiles, w streamed and E = 1 - w d derived, or both computed from
// the optical step d = kappa dtau (kappa = r_p / |mu| per ray, dtau per
// interval).
constexpr int kCoefPairs = 0;
constexpr int kCoefW = 1;
constexpr int kCoefRecompute = 2;

struct SweepArgs {
    const AtmDesc *atm;
    const BlockDesc *blk;
    const void *coef;        // tile-ordered step coefficients: (E, w) pairs or w (type T)
    const double *q;         // tile-ordered quadrature weights (see q_off)
    const double2 *kt;       // tile-ordered (kappa, 1 / kappa) per ray, as q
    const double *dtau;      // per depth point: tau_{k+1} - tau_k (0 at a slab's last point)
    const double2 *dirc;     // per direction: (T1, T1^2 + T2^2)
    const double4 *Qs;       // per slab: sums over all rays of q, q T1, q (T1^2 + T2^2)
    const double *sig_in;    // FP64 input, NULL = zero source
    const double *scale;     // optional elementwise scaling of sig_in
    double *sig_out;         // FP64 output
    double *partial;         // per-block partial quadrature sums (float values when part_f32)
    const int *mask;         // optional per-slab activity mask
    const double *B;         // Planck function (right-hand-side mode)
    int mode;                // 0: sigma_out = z - xi [J00, W2 J20]
                             // 1: sigma_out = xi [J00, W2 J20] + [eps B, 0],
                             //    with the bottom inflow and no source
    int rows;                // 1: one LDS row per wave (W * 2 ns_max values),
                             // 0: one shared row filled wave after wave
    int src_lds;             // byte offset of the sources in the sweep's LDS (set at launch)
    int fs;                  // formal solver (coefficients computed in the sweep)
    int part_f32;            // 1: the partial sums are FP32 (written by an FP32 sweep)
};

// --------------------------------------------------------------------------
// Lane layout of a wave-batch.  A ray's C chunks sit C lanes apart in chunk
// order; for C < 16 the chunks of one ray are spread over a row of 16 lanes
// with stride s = 16 / C (s rays interleaved per row), for C >= 16 a ray
// fills C consecutive lanes.  Either way a DPP shift by s lanes inside a row
// (or a row broadcast across rows) moves data from chunk c to chunk c + 1 of
// the same ray, and lanes whose source would be another ray's chunk have no
// source at all, so the lane scans need no masks.
// --------------------------------------------------------------------------
__host__ __device__ inline int lane_chunk(int lane, int C) {
    return C >= 16 ? (lane & (C - 1)) : ((lane & 15) / (16 / C));
}
__host__ __device__ inline int lane_slot(int lane, int C) {
    if (C >= 16) return lane / C;
    const int s = 16 / C;
    return (lane >> 4) * s + (lane & (s - 1));
}


// Chunk counts of a plan: powers of two from kMinChunks to 64 (short slabs
// get identity-padded chunks rather than fewer of them, so the sweep has one
// lane layout per chunk count it is compiled for).
constexpr int kMinChunks = 8;
// The tail plan: GMRES cycles that start with at most kTailSlabs slabs still
// iterating sweep with at most kTailWb wave-batches per wave, so those slabs
// spread over more workgroups (the main plan, made for the whole batch, gives
// a long slab one workgroup per direction).
constexpr int kTailSlabs = 128;
constexpr int kTailWb = 8;

// Chunk lengths compiled for a plan of longest chunk L: L/2+1 .. L for L <= 8,
// L/2 + L/8, L/2 + 2L/8, .. L for L >= 16.  A slab's chunk length is
// ceil((ns - 1) / C) rounded up to one of them (the extra steps are identity
// padding).
constexpr int chunk_len_step(int L) { return L >= 16 ? L / 8 : 1; }
constexpr int chunk_len_min(int L) { return L / 2 + chunk_len_step(L); }

// Waves per sweep block for a chunk length and precision (automatic choice).
int sweep_waves(int L, bool fp32);

// Launch helpers (rt_sweep.hip).  launch_sweep writes the per-block partial
// quadrature sums; launch_finalize turns them into sigma_out.
hipError_t launch_sweep(int L, int W, bool pf, bool fp32, int cm, const SweepArgs &a,
                        int nblocks, int ns_max, hipStream_t s);
#define RT_SWEEP_LAUNCHER(name)                                                              \
    hipError_t name(int L, int W, bool pf, const SweepArgs &a, int nblocks, int ns_max, \
                    hipStream_t s)
RT_SWEEP_LAUNCHER(launch_sweep_f32);
RT_SWEEP_LAUNCHER(launch_sweep_f64);
RT_SWEEP_LAUNCHER(launch_sweep_f32_w);
RT_SWEEP_LAUNCHER(launch_sweep_f64_w);
RT_SWEEP_LAUNCHER(launch_sweep_f32_rc);
RT_SWEEP_LAUNCHER(launch_sweep_f64_rc);
#undef RT_SWEEP_LAUNCHER
// The coefficient mode (kCoef*) of a handle's FP32 or FP64 sweeps.
int coef_mode_of(const rt_handle *h, bool fp32);
// Launch configuration of the sweep for a handle: waves per block and whether
// the next ray batch is loaded during the current one.
void sweep_config(const rt_handle *h, bool fp32, int *W, bool *pf);
// nblk_max: the most blocks of one slab in the plan a.atm describes (it sets
// how many lanes share a point).
hipError_t launch_finalize(const SweepArgs &a, int n_atm, int ns_max, int nblk_max,
                           hipStream_t s);
// Tile-ordered step coefficients of the modes that stream them (any output
// may be NULL: not built), the tile-ordered weights and (kappa, 1 / kappa).
hipError_t launch_coef_build(int nblocks, int W, const AtmDesc *atm, const BlockDesc *blk,
                             const double *tau, const double *opac, const double *mu_pos, int fs,
                             const double *qray, double2 *coef64, float2 *coef32, double *w64,
                             float *w32, double *qtile, double2 *ktile, hipStream_t s);
hipError_t launch_ray_setup(int n_atm, const AtmDesc *atm, const double *mu_pos,
                            const double *w_pos, int M, const double *w_nu, const double *phi,
                            int n_nu, int normalize, RayConst *rayc, double *q, double2 *dirc,
                            double4 *Qs, hipStream_t s);
hipError_t launch_diag(int npts, const int *pt_atm, const AtmDesc *atm, const double *tau,
                       const double *opac, const double *mu_pos, const RayConst *rayc, int M,
                       int n_nu, int fs, double *diag, double *dinv, hipStream_t s);
bool sweep_chunk_supported(int L, bool fp32);
// Chunk length of a slab of ns points split into C chunks, for a plan of
// longest chunk L: ceil((ns - 1) / C) rounded up to a length the sweep is
// compiled for.
int chunk_len(int ns, int C, int L);

// Dense assembly of A (rt_assemble.hip).  Writes every slab's (2 ns)^2 block,
// row-major, at a_off; the coefficient table and scratch live in the handle.
int assemble(rt_handle *h, double *A, hipStream_t s);

// SOR / SSOR on the assembled A (rt_dense.hip): out = P^-1 in for the slabs
// whose mask is set (all if NULL), and out = P in.  ensure_dense assembles the
// handle's A on first use.
hipError_t precond_tri(const rt_handle *h, const double *in, double *out, const int *mask,
                       hipStream_t s);
hipError_t precond_tri_mult(const rt_handle *h, const double *in, double *out, hipStream_t s);
hipError_t fill(double *v, long long n, double c, hipStream_t s);
int ensure_dense(rt_handle *h, hipStream_t s);
// Dense LU with partial pivoting of every slab's assembled A (once per
// handle), and x = A^-1 b from the factors.
int lu_factor(rt_handle *h, hipStream_t s);
hipError_t lu_solve(const rt_handle *h, const double *b, double *x, hipStream_t s);

// Mixed-precision refinement: the inner solve of A d = r only has to bring
// ||r - A d|| below rtol ||b||.  Asking for kIrMargin rtol ||b|| is a
// relative tolerance of kIrMargin rtol ||b|| / ||r|| on the inner solve; where
// that is looser than inner_rtol (the last refinement step) the inner solve
// stops there instead of reducing the residual by the full inner_rtol.
constexpr double kIrMargin = 0.5;

// Krylov state kept on the device, one entry per slab.
struct KState {
    double bnorm;     // ||b||
    double beta;      // last explicit residual norm
    double resid;     // GMRES residual estimate |g_{j+1}|
    double rho, alpha, omega, rho_old;  // BiCGSTAB scalars
    double relres;    // final explicit relative residual
    int status;       // RT_OK / RT_ENOCONV / RT_EBREAKDOWN
    int iters;        // iterations counted for maxit
    int matvecs;      // applications of A
    int inner;        // GMRES: Arnoldi steps in the current cycle
    int outer;        // mixed precision: refinement steps
    int half_done;    // BiCGSTAB: converged at the half step
    int pad0, pad1;
    double tol_next;  // mixed precision: relative tolerance the next inner solve needs
};

}  // namespace rt

// The handle (opaque to C callers).
struct rt_handle {
    int device = 0;
    int n_atm = 0, n_mu = 0, M = 0, n_nu = 0, fs = 0, normalize = 0;
    int n_unk = 0, ns_total = 0, ns_max = 0;
    rt_options opt{};
    std::vector<int> ns, doff;
    std::vector<rt::AtmDesc> atm_h;
    std::vector<rt::BlockDesc> blk_h;
    int L = 8;                 // chunk length the tiles were built for
    int W = 4;                 // waves per sweep block the plan was made for
    int NB = 1;                // wave-batches per wave (per block: W * NB)
    int n_blocks = 0;
    int nblk_max = 0, nblk_max_tail = 0;  // most blocks of one slab, per plan
    long long n_pairs = 0, n_partial = 0;
    long long n_partial_main = 0;  // partial sums of the main plan's blocks
    // the tail plan over the same coefficient tiles (none when it would equal
    // the main plan); plan_tail selects it for the sweeps, their finalize pass
    // and the fused Arnoldi step, which all read the slab table it points to
    int n_blocks_tail = 0;
    bool plan_tail = false;

    // device copies of the problem
    double *d_tau = nullptr, *d_B = nullptr, *d_opac = nullptr, *d_phi = nullptr;
    double *d_mu_pos = nullptr, *d_w_pos = nullptr, *d_w_nu = nullptr;
    int *d_pt_atm = nullptr;
    rt::AtmDesc *d_atm = nullptr;
    rt::BlockDesc *d_blk = nullptr;
    rt::AtmDesc *d_atm_tail = nullptr;  // nblk, blk_first, part_off of the tail plan
    rt::BlockDesc *d_blk_tail = nullptr;
    rt::RayConst *d_rayc = nullptr;
    double *d_q = nullptr;        // per ray quadrature weight
    double *d_qt = nullptr;       // tile-ordered, zero-padded quadrature weights
    long long n_qt = 0;
    double2 *d_dirc = nullptr;    // per direction (T1, T1^2 + T2^2)
    double4 *d_Qs = nullptr;      // per slab quadrature moments (Q0, Q1, Q2)
    // step coefficients of the sweeps, by coefficient mode: (E, w) pairs or w
    // alone, in FP64 and FP32 (only those the handle's modes read are built)
    double2 *d_coef64 = nullptr;
    float2 *d_coef32 = nullptr;
    double *d_w64 = nullptr;
    float *d_w32 = nullptr;
    double2 *d_kt = nullptr;      // tile-ordered (kappa, 1 / kappa) per ray
    double *d_dtau = nullptr;     // tau_{k+1} - tau_k per depth point
    int cm64 = 0, cm32 = 0;       // coefficient modes of the FP64 and FP32 sweeps
    int plan_status = 0;          // stored launch plan: 0 none, 1 current, 2 other sources
    double *d_partial = nullptr;
    double *d_diag = nullptr, *d_dinv = nullptr, *d_b = nullptr;
    double *d_rpart = nullptr;    // ray-per-lane sweep: per-wavefront quadrature slots
    int *d_mu_idx = nullptr;      // per |mu| index m: caller's index of -mu (2m) and +mu (2m+1)
    double *d_fsig = nullptr;     // field formulation: J I, 2 values per depth point
    double *d_Rw = nullptr;       // redistribution: R(p, q) w_q per slab, [q][p]
    unsigned short *d_Rw_bf = nullptr;  // R w split in bf16 hi, lo: [2][slab][p][prd_nqp]
    int prd_nqp = 0;              // padded row length of the bf16 split (multiple of 32)
    double *d_prd_Jm = nullptr;   // per-|mu| quadrature stage (when not in LDS)
    double *d_prd_J = nullptr;    // monochromatic J, frequency-major [p][k][K]
    double *d_prd_diag = nullptr, *d_prd_dinv = nullptr;
    bool prd_ready = false;
    int prd_cached_nt = 0;        // threads of the cached-coefficient sweep, 0: the general sweep
    int prd_cached_nch = 0;       // its chunks per ray
    long long n_dense = 0;        // entries of the assembled A: sum over slabs of (2 ns)^2
    long long n_ew = 0;           // entries of the assembly coefficient table

    // dense route (allocated on first use)
    double2 *d_ew = nullptr;      // (E, w) per slab, interval and ray
    double *d_asm_dg = nullptr;   // node-diagonal moments per slice and direction
    double *d_asm_sc = nullptr;   // raw moments of ray slices after the first
    void *d_asm_task = nullptr;   // assembly task list
    int asm_tasks = 0, asm_rg = 0, asm_nw = 0, asm_cpm = 0, asm_slices = 0;
    double *d_A = nullptr;        // the handle's assembled A (SOR, SSOR)
    bool dense_ready = false;
    double *d_pz = nullptr;       // P^-1 v for the triangular preconditioners
    double *d_ones = nullptr;     // unit diagonal scaling of the Krylov updates
    double *d_LU = nullptr;       // LU factors of the assembled A
    int *d_piv = nullptr;         // their row exchanges
    int *d_sing = nullptr;        // per slab: a zero pivot was met
    int *d_lu_order = nullptr;    // slabs by decreasing size: the factorization's workgroup order
    bool lu_ready = false;

    // solver workspace (allocated on first use)
    int ws_restart = 0;
    double *d_V = nullptr;      // (restart + 1) x N Krylov basis
    double *d_H = nullptr;      // per slab (restart + 1) x restart Hessenberg
    double *d_cs = nullptr, *d_sn = nullptr, *d_g = nullptr;
    double *d_w = nullptr;      // operator output
    double *d_r = nullptr, *d_rh = nullptr, *d_p = nullptr, *d_v = nullptr, *d_s = nullptr,
           *d_t = nullptr;      // BiCGSTAB / refinement vectors
    double *d_cq = nullptr;     // CGS
    rt::KState *d_state = nullptr;
    int *d_active = nullptr;    // per slab: still iterating
    int *d_cycle = nullptr;     // per slab: GMRES cycle still running
    int *d_count = nullptr;     // reduction target for host checks
    int *h_count = nullptr;     // pinned host mirror
    int *h_seg_flag = nullptr;  // pinned: the segmented GMRES's end-of-cycle flag

    // workspace of the segmented GMRES (slot 0) and of the refinement around
    // it (slot 1), kept between calls and grown on demand
    void *seg_ws[2] = {nullptr, nullptr};
    size_t seg_ws_bytes[2] = {0, 0};

    // captured solver segments (one per distinct argument set), the stream
    // they are replayed on and the events that order it after the caller's
    struct Graph {
        std::vector<unsigned long long> key;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Graph> graphs;
    hipStream_t gstream = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
};

namespace rt {

// The slab table, block list and block count of the plan the sweeps use now.
inline const AtmDesc *plan_atm(const rt_handle *h) {
    return h->plan_tail ? h->d_atm_tail : h->d_atm;
}
inline const BlockDesc *plan_blk(const rt_handle *h) {
    return h->plan_tail ? h->d_blk_tail : h->d_blk;
}
inline int plan_blocks(const rt_handle *h) { return h->plan_tail ? h->n_blocks_tail : h->n_blocks; }
inline int plan_nblk_max(const rt_handle *h) {
    return h->plan_tail ? h->nblk_max_tail : h->nblk_max;
}

// sigma_out = A (scale .* sigma_in) for the slabs whose mask is set (all if
// mask is NULL): the sweep, then the finalize pass.  mode as in SweepArgs.
hipError_t apply_operator(rt_handle *h, const double *in, const double *scale, double *out,
                          const int *mask, bool fp32, int mode, hipStream_t s);
// sigma_out = A sigma_in in FP64 (rt_apply_op) with the per-block partial
// quadrature sums in `partial` (at least n_partial_main doubles) instead of
// the handle's buffer; main plan, no scaling, no mask.
hipError_t apply_operator_into(rt_handle *h, const double *in, double *out, double *partial,
                               hipStream_t s);
// The sweep of apply_operator (mode 0) alone: leaves the per-block quadrature
// sums in h->d_partial for a consumer that applies the scattering step itself.
hipError_t apply_sweep(rt_handle *h, const double *in, const double *scale, const int *mask,
                       bool fp32, hipStream_t s);

// The operator with the ray-per-lane FP64 sweep (formal solvers with a
// three-point stencil, rt_raysweep.hip): same contract as apply_operator.
hipError_t apply_ray_operator(rt_handle *h, const double *in, const double *scale, double *out,
                              const int *mask, int mode, hipStream_t s);
// The field as unknown (eq. crd_linear_system2, rt_field.hip): out = (Id -
// Lambda T J) in; b = Lambda T c + t; sigma = J I (+ c when with_c).
hipError_t apply_field_operator(rt_handle *h, const double *in, double *out, hipStream_t s);
hipError_t field_rhs(rt_handle *h, double *b, hipStream_t s);
hipError_t field_sigma(rt_handle *h, const double *I, double *sigma, int with_c, hipStream_t s);
// GMRES(restart) on the field system, unpreconditioned, batched over slabs
// (rt_fieldsolve.hip); b NULL: the handle's own Lambda T c + t.
int solve_field_gmres(rt_handle *h, const double *b, double *x, rt_solve_info *info,
                      hipStream_t s);
// The operator of a segmented solve: out = A (scale .* in), scale NULL for
// none (the right Jacobi scaling is applied by the operator's own kernels).
using SegOp = std::function<hipError_t(const double *in, const double *scale, double *out)>;
// The generic form: any block-diagonal operator with `per` entries per depth
// point, own_rhs filling b when b is NULL, optional right Jacobi scaling.
int solve_seg_gmres(rt_handle *h, const SegOp &op,
                    long long per, const double *b,
                    const std::function<hipError_t(double *)> &own_rhs, double *x,
                    const double *dinv, rt_solve_info *info, hipStream_t st);
// The same with an explicit tolerance and iteration limit (the inner solves
// of the refinement below).
int solve_seg_gmres_tol(rt_handle *h, const SegOp &op,
                        long long per, const double *b,
                        const std::function<hipError_t(double *)> &own_rhs, double *x,
                        const double *dinv, double rtol, int maxit, rt_solve_info *info,
                        hipStream_t st);
// FP64 iterative refinement: r = b - A x with op, d from GMRES(m) on op_lo to
// inner_rtol (or the looser tolerance kIrMargin allows), x += d, until every
// slab's ||r|| < rtol ||b|| (or maxit inner steps in total).
int solve_seg_refined(rt_handle *h, const SegOp &op, const SegOp &op_lo,
                      long long per, const double *b,
                      const std::function<hipError_t(double *)> &own_rhs, double *x,
                      const double *dinv, rt_solve_info *info, hipStream_t st);

// The frequency-redistribution variant (rt_prd.hip): out = A (scale .* in)
// (scale NULL: none), or the right-hand side when in is NULL; its Jacobi
// diagonal; workspace set-up.
hipError_t apply_prd_operator(const rt_handle *h, const double *in, double *out, hipStream_t s,
                              bool bf16x3 = false, const double *scale = nullptr);
hipError_t prd_diag(const rt_handle *h, double *diag, double *dinv, hipStream_t s);
int ensure_prd(rt_handle *h, hipStream_t s);
int solve_prd_gmres(rt_handle *h, const double *b, double *x, rt_solve_info *info,
                    hipStream_t s);
// Quadrature slots per slab of that sweep (two per wavefront of rays).
int ray_slots(const rt_handle *h);

// Destroy the handle's captured solver graphs.
void clear_graphs(rt_handle *h);

// Thread-local error message for rt_last_error.
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
}  // namespace rt
