/*
 * rt_ext.h -- additional entry points of the gfx950 library, beside rt.h.
 * Same conventions as rt.h (device FP64 vectors of length N, hipStream_t as
 * void*, return codes, rt_last_error).
 */
#ifndef RT_EXT_H
#define RT_EXT_H

#include "rt.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * sigma_out = A sigma_in with the formal-solver sweep and quadrature of
 * Algorithm 1 carried out in FP32 (step coefficients rounded from their FP64
 * values, FP32 recurrences and accumulators; input read and output written in
 * FP64).  This is the operator of the inner solves of RT_PREC_MIXED; its error
 * against rt_apply_op is of the order of the FP32 unit roundoff times the
 * number of steps along a ray.  In-place allowed, as for rt_apply_op.
 */
int rt_apply_op_fp32(rt_handle *h, const double *sigma_in, double *sigma_out, void *stream);

/*
 * For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * sigma_out = A sigma_in exactly as rt_apply_op computes it (same kernels,
 * same launch plan, same result bit for bit), with the sweep's per-workgroup
 * partial quadrature sums kept in a fixed device array of
 * RT_NOALLOC_MAX_PARTIAL doubles (32 MiB) that the library holds on every
 * GPU it runs on until the process ends, instead of the handle's buffer.
 * The call allocates nothing.  The handle's sweep must need at most
 * RT_NOALLOC_MAX_PARTIAL partial sums (the 512-slab batch of up to 512
 * depths, 16 directions and 101 frequencies needs about 2.4 million), else
 * RT_EINVAL; the DELO-parabolic solver is not supported (RT_EINVAL); the
 * handle's device must be current (RT_EINVAL).  Every call on one GPU uses
 * that GPU's one array: calls that overlap in time on one GPU (different
 * streams or handles) race and give wrong results.  Stream-ordered; in-place
 * allowed as for rt_apply_op.
 */
#define RT_NOALLOC_MAX_PARTIAL (4LL * 1024 * 1024)
int rt_apply_op_noalloc(rt_handle *h, const double *sigma_in, double *sigma_out, void *stream);

/*
 * Solve A x = b with the conjugate gradient squared method (Sect. 2.2;
 * Sonneveld), right-preconditioned by Jacobi: two products by A per step, none
 * by A^T.  Same contract as rt_solve_gmres (b NULL means the handle's own
 * right-hand side; x in: initial guess, out: solution; info host array of
 * n_atm entries or NULL).  iterations counts full steps; convergence is tested
 * on the recursively updated residual and relres is recomputed from x at the
 * end.  rho = 0, (r0, A P^-1 p) = 0 or a non-finite residual returns
 * RT_EBREAKDOWN for that slab with x at the last iterate.  Synchronizes the
 * stream before returning.
 */
int rt_solve_cgs(rt_handle *h, const double *b, double *x, rt_solve_info *info, void *stream);

/*
 * Describe the sweep plan: chunk length L, number of sweep workgroups, number
 * of stored coefficient pairs (tiles, including padding) and of ray-interval
 * pairs sum_slabs (ns - 1) (n_mu / 2) n_nu.  Any output pointer may be NULL.
 * Host only.
 */
int rt_plan_info(const rt_handle *h, int *chunk_L, int *n_blocks, long long *n_pairs,
                 long long *n_intervals);

/*
 * The sweep launch configuration of rt_apply_op (fp32 = 0) or
 * rt_apply_op_fp32 (fp32 != 0) on this handle: wavefronts per workgroup, and
 * 1 if the step coefficients of a wavefront's next ray batch are loaded while
 * the current one is swept, 0 if they are loaded on use.  Any output pointer
 * may be NULL.  Host only.
 */
int rt_sweep_config(const rt_handle *h, int fp32, int *waves, int *prefetch);

/*
 * Where the FP32 (fp32 != 0) or FP64 sweep of this handle takes its step
 * coefficients from, as resolved from options.coef_mode at setup: 0 = (E, w)
 * pairs streamed, 1 = w streamed and E derived, 2 = both computed in the
 * sweep.  Host only.
 */
int rt_sweep_coef_mode(const rt_handle *h, int fp32, int *mode);

/*
 * Stored launch plans (rt_options.autotune).  rt_tuned_plan_status: 0 = no
 * plan was stored for the handle's problem (or autotune was off), 1 = a plan
 * measured with the sweep sources this library was built from was applied,
 * 2 = a plan measured with other sources was applied (stale: re-tune).  rt_sweep_source_hash: the
 * hash of the sweep sources this library was built from.  rt_plan_key: the
 * key of problem p at precision (RT_PREC_*) on architecture arch (NULL: the
 * current device's, e.g. "gfx950"), written NUL-terminated into buf of
 * buflen bytes (RT_EINVAL if too short).  Host only.
 */
int rt_tuned_plan_status(const rt_handle *h);
/* The options the handle runs with: the caller's, with the stored plan's
 * fields filled in where options.autotune applied one (plan_file is returned
 * as NULL).  Host only. */
int rt_get_options(const rt_handle *h, rt_options *o);
const char *rt_sweep_source_hash(void);
int rt_plan_key(const rt_problem *p, int precision, const char *arch, char *buf, int buflen);

/*
 * Number of doubles of the assembled operator: the sum over slabs of
 * (2 ns)^2.  Host only.
 */
int rt_assembled_size(const rt_handle *h, long long *count);

/*
 * Assemble A = Id - J Lambda T explicitly (Sect. 3.3 builds A column by
 * column from Algorithm 1 applied to the unit vectors; Sect. 4.4 uses that a
 * point source gives zero intensity upwind of it).  A_out is a caller-owned
 * device array of rt_assembled_size doubles; slab s's (2 ns_s) x (2 ns_s)
 * block is stored row-major at offset sum_{t<s} (2 ns_t)^2, rows and columns
 * in the unknowns' order [s00(z_1), s20(z_1), s00(z_2), ...], so that
 * A_s x_s = (rt_apply_op(x))_s up to rounding.  The first call on a handle
 * also builds a coefficient table of sum_s (ns_s - 1) (n_mu / 2) n_nu (E, w)
 * pairs (16 bytes each) kept until rt_destroy, plus, when one workgroup
 * cannot hold a slab's rays, scratch of the size of A per extra ray slice.
 * Stream-ordered on `stream`; RT_ENOMEM if a workspace allocation fails.
 */
int rt_assemble(rt_handle *h, double *A_out, void *stream);

/*
 * Solve A x = b directly (the assembled route of Sect. 3.3 and 4.5): every
 * slab's A is assembled (rt_assemble) and factored with partial pivoting by
 * rows, PA = LU, on the first call; the factors are kept by the handle, so
 * later calls only substitute.  b NULL means the handle's own right-hand side;
 * x is output only.  info[i] (host, n_atm entries, or NULL) gets status RT_OK
 * (RT_EBREAKDOWN if a pivot was exactly zero), iterations 0, matvecs 1 and the
 * relative residual ||b - A x|| / ||b|| recomputed with the matrix-free FP64
 * operator.  Workspace: (2 ns)^2 doubles per slab for the factors, plus those
 * of rt_assemble.  Synchronizes the stream before returning.
 */
int rt_solve_lu(rt_handle *h, const double *b, double *x, rt_solve_info *info, void *stream);

/*
 * z = P^-1 v with the handle's preconditioner (options.precond, Sect. 2.3):
 * Jacobi as rt_precond_jacobi; SOR and SSOR by triangular solves with the
 * assembled A (built on the first call that needs it, see rt_assemble).
 * Device vectors of length N; z == v allowed.  Stream-ordered.
 */
int rt_precond_apply(rt_handle *h, const double *v, double *z, void *stream);

/*
 * The Stokes field as unknown (eq. crd_linear_system2): (Id - Lambda T J) I =
 * Lambda T c + t, whose solution gives sigma = J I + c.  A field vector holds,
 * per slab (slabs concatenated in ns order), I then Q at every depth, every mu
 * of the caller's mu array and every frequency:
 *   index  2 n_mu n_nu doff_s + ((st ns_s + k) n_mu + m) n_nu + p,  st = 0 (I), 1 (Q),
 * so that a depth's rays are contiguous.  J maps a field to xi [J00, W2 J20]
 * (eqs. J00/J02 with S00/S02), T the multipolar components to the source
 * functions, Lambda is the formal solution with zero incoming radiation and t
 * the transmitted field (I_bot entering at the bottom for mu > 0).
 * rt_field_size: the number of doubles of a field, 2 n_mu n_nu sum ns.
 * rt_apply_op_field: I_out = (Id - Lambda T J) I_in; device arrays that must
 *   not alias.  rt_get_rhs_field: b_field = Lambda T c + t.
 * rt_sigma_from_field: sigma (length N) = J I + c.
 * All FP64 and stream-ordered (the formal solver runs one lane per ray).
 */
int rt_field_size(const rt_handle *h, long long *count);
int rt_apply_op_field(rt_handle *h, const double *I_in, double *I_out, void *stream);
int rt_get_rhs_field(rt_handle *h, double *b_field, void *stream);
int rt_sigma_from_field(rt_handle *h, const double *I, double *sigma, void *stream);

/*
 * Solve the field system with unpreconditioned GMRES(options.restart)
 * (Sect. 2.1; Sect. 3.2 expects this larger, sparser system to suit Krylov
 * methods).  Each slab is its own system, tested on ||b - K I|| / ||b|| <
 * options.rtol within options.maxit Arnoldi steps.  b_field NULL means the
 * handle's own Lambda T c + t; I (device, rt_field_size doubles) holds the
 * initial guess and receives the solution; b_field and I must not alias.
 * info[i] (host, n_atm entries, or NULL): status (RT_OK or RT_ENOCONV),
 * Arnoldi steps, the batch's operator applications (an upper bound for the
 * slab) and the explicit relative residual.  Workspace of (restart + 2)
 * fields is allocated on the first call that needs it and kept by the handle
 * (grown when a later call needs more) until rt_destroy; RT_ENOMEM if it
 * does not fit.  Synchronizes the stream.
 */
int rt_solve_field_gmres(rt_handle *h, const double *b_field, double *I, rt_solve_info *info,
                         void *stream);

/*
 * Frequency redistribution (an extension of the paper's complete
 * redistribution, CRD, of Sect. 3.1: the emission at frequency p is
 * sum_q R(p, q) w_q J_q / phi_p instead of phi_p times the frequency-
 * integrated J).  The unknown is sigma^K(k, p) per depth and frequency,
 * laid out 2 n_nu doff_s + (k n_nu + p) 2 + K (K = 0: s00, 1: s20), and
 *   S_I = s00(k, p) + T1 s20(k, p),  S_Q = T2 s20(k, p);
 *   J^K_p(k) = the angle quadrature of eqs. J00/J02 at frequency p;
 *   (A sigma)^K(k, p) = sigma^K(k, p) - xi W_K sum_q R(p, q) w_q J^K_q(k) / phi_p,
 * W_0 = 1, W_2 = W2; b is the same contraction of the transmitted field plus
 * [eps B, 0].  R proportional to phi(p) phi(q) gives back CRD at every p.
 * rt_set_redistribution: R (host, n_atm x n_nu x n_nu, R[s][p][q] row-major;
 *   copied, finite) for the handle's slabs; enables the calls below (RT_EINVAL
 *   before).  rt_setup calls it itself when rt_problem.R is set.  The
 *   contraction runs on the FP64 matrix cores (and on the BF16 ones in the
 *   calls so named).
 * rt_prd_size: 2 n_nu sum ns doubles.
 * rt_apply_op_prd / rt_get_rhs_prd / rt_get_jacobi_diag_prd: A sigma, b,
 *   diag(A) (device arrays, stream-ordered).
 * rt_apply_op_prd_bf16x3: A sigma with the contraction on the BF16 matrix
 *   cores: R w and J are each split into bf16 hi + lo (about 16 significant
 *   bits), the products hi.hi, hi.lo and lo.hi are accumulated in FP32 and
 *   added in FP64; normwise error about 1e-5 of |sigma| + |xi J~ / phi|.
 *   Same arguments as rt_apply_op_prd.
 * rt_solve_prd_gmres: Jacobi-preconditioned (from the right) GMRES(restart)
 *   to options.rtol; b NULL means the handle's own b; x holds the initial
 *   guess and receives the solution; info as for rt_solve_gmres.  FP64:
 *   FP64 operator throughout.  MIXED: FP64 iterative refinement, r = b - A x
 *   with the FP64 operator, an inner GMRES on the BF16x3 operator to
 *   options.inner_rtol or the looser 0.5 rtol ||b|| (inner_maxit steps at
 *   most), x += d, until
 *   ||r|| < rtol ||b|| per slab; iterations counts the inner steps,
 *   outer_steps the refinement steps.  Synchronizes the stream.
 */
int rt_set_redistribution(rt_handle *h, const double *R);
int rt_prd_size(const rt_handle *h, long long *count);
int rt_apply_op_prd(rt_handle *h, const double *sigma_in, double *sigma_out, void *stream);
int rt_apply_op_prd_bf16x3(rt_handle *h, const double *sigma_in, double *sigma_out, void *stream);
int rt_get_rhs_prd(rt_handle *h, double *b, void *stream);
int rt_get_jacobi_diag_prd(rt_handle *h, double *d, void *stream);
int rt_solve_prd_gmres(rt_handle *h, const double *b, double *x, rt_solve_info *info,
                       void *stream);

/*
 * Run the validation of rt_setup on (p, o) without touching any device:
 * RT_OK or RT_EINVAL with the message in rt_last_error().  o may be NULL.
 */
int rt_validate(const rt_problem *p, const rt_options *o);

#ifdef __cplusplus
}
#endif
#endif /* RT_EXT_H */
