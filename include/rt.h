/*
 * rt.h -- C ABI of the MI355X (gfx950) library for the matrix-free operator
 *         A = Id - J Lambda T of a 1D two-level-atom scattering-polarization
 *         line (J_u = 1, J_l = 0, complete frequency redistribution, Stokes
 *         I and Q) and for the Jacobi-preconditioned Krylov solvers of
 *         A sigma = J t + c.
 *
 * Paper: Benedusi, Janett, Belluzzi & Krause, "Numerical solutions to linear
 * transfer problems of polarized radiation II. Krylov methods and matrix-free
 * implementation" (A&A).  Section, equation and algorithm labels below are the
 * paper's.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - sigma layout (Sect. 3.2, eq. matricial_form_1): for each slab, depth
 *    points top first, interleaved [s00(z1), s20(z1), s00(z2), s20(z2), ...];
 *    slabs concatenated in the order of rt_problem.ns.  Length
 *    N = 2 * sum(ns).  All vector arguments (sigma_in, sigma_out, v, z, b, x,
 *    d) are DEVICE pointers to FP64 arrays of length N, owned by the caller
 *    (hipMalloc or torch device tensors), contiguous.
 *  - "stream" is a hipStream_t passed as void* (NULL = the default stream).
 *    rt_apply_op, rt_precond_jacobi, rt_get_rhs and rt_get_jacobi_diag are
 *    stream-ordered and asynchronous.  The rt_solve_* calls run on the given
 *    stream and synchronize it before returning.
 *  - Return codes: RT_OK (0); negative for caller or system errors, with no
 *    effect on the outputs (RT_EINVAL, RT_ENOMEM, RT_EDEVICE); positive for
 *    numerical outcomes of a solve (RT_ENOCONV, RT_EBREAKDOWN), in which case
 *    x holds the last iterate.  For a batch of slabs the return value is the
 *    worst status over slabs and info[i] holds slab i's status.
 *    rt_last_error() returns a message for the calling thread's last non-zero
 *    return.
 *  - A handle may be used from one host thread at a time.  Calls on one
 *    handle must not overlap in time on different streams.
 */
#ifndef RT_H
#define RT_H

#ifdef __cplusplus
extern "C" {
#endif

#define RT_OK 0
#define RT_EINVAL (-1)
#define RT_ENOMEM (-2)
#define RT_EDEVICE (-3)
#define RT_ENOCONV 1
#define RT_EBREAKDOWN 2

/* Formal solvers (Sect. 4.1).  DELO-linear: exact integration of a linearly
 * interpolated source function along the ray.  Trapezoidal: Crank-Nicolson
 * step of the transfer equation in optical path (not one of the paper's
 * four solvers; provided for comparison).  Implicit Euler: the backward
 * difference I_k = (I_u + d S_k) / (1 + d), d the optical step (one of the
 * paper's four solvers, Sect. 4.1). */
#define RT_FS_DELO_LINEAR 0
#define RT_FS_TRAPEZOIDAL 1
#define RT_FS_IMPLICIT_EULER 2
/* DELO-parabolic (Sect. 4.1): the source interpolated by the parabola through
 * the upwind, current and downwind points of the ray, integrated exactly; the
 * last point of a ray takes the DELO-linear step.  Without dichroism, as
 * here, DELOPAR is the same step.  Its operator runs a ray-per-lane FP64
 * sweep (also in RT_PREC_MIXED); rt_assemble, rt_solve_lu and the SOR/SSOR
 * preconditioners are not available for it (RT_EINVAL). */
#define RT_FS_DELO_PARABOLIC 3

/* Arithmetic of the solves.  FP64: every step in FP64.  MIXED: an FP32
 * formal-solver sweep and quadrature inside an inner GMRES, with the outer
 * residual, the update of x, the step coefficients and the Hessenberg
 * least-squares problem in FP64 (iterative refinement). */
#define RT_PREC_FP64 0
#define RT_PREC_MIXED 1

/* Preconditioners (Sect. 2.3); see rt_options.precond. */
#define RT_PC_JACOBI 0
#define RT_PC_SOR 1
#define RT_PC_SSOR 2

/* Where the formal-solver sweep takes each ray-interval's step coefficients
 * from (rt_options.coef_mode).  Every formal solver here steps the deviation
 * D = I - S as D_k = E D_u + w (S_u - S_k) with w = (1 - E) / d, d the optical
 * step r_p |tau_k - tau_u| / |mu| (Sect. 4.1).
 *  RT_COEF_PAIRS      (E, w) per ray-interval, built at setup in FP64 and
 *                     FP32, streamed by every application (16 or 8 bytes);
 *  RT_COEF_STREAM_W   w alone streamed (8 or 4 bytes), E = 1 - w d derived
 *                     from d = kappa dtau, kappa = r_p / |mu| per ray and
 *                     dtau per interval;
 *  RT_COEF_RECOMPUTE  E and w both computed in the sweep from d (one
 *                     exponential per ray-interval for DELO-linear, one
 *                     reciprocal for the trapezoidal rule and implicit Euler);
 *  RT_COEF_RECOMPUTE_FP32  FP32 sweeps recompute, FP64 sweeps stream w;
 *  RT_COEF_AUTO       the library's choice (RT_COEF_STREAM_W).
 * Results agree to rounding between modes.  Setup builds only the tiles
 * the handle's modes stream. */
#define RT_COEF_AUTO 0
#define RT_COEF_PAIRS 1
#define RT_COEF_STREAM_W 2
#define RT_COEF_RECOMPUTE 3
#define RT_COEF_RECOMPUTE_FP32 4

/* Largest supported depth grid per slab, and largest GMRES restart length. */
#define RT_MAX_NS 2048
#define RT_MAX_RESTART 128

typedef struct rt_handle rt_handle;

/*
 * The discrete problem (Sect. 3.1-3.2, 4.1).  Host pointers; rt_setup copies
 * everything it needs, so the caller may free them afterwards.
 *
 *  n_atm            number of independent slabs (>= 1)
 *  ns[n_atm]        depth points per slab, 2 <= ns <= RT_MAX_NS
 *  tau[sum ns]      optical depths per slab, top first, strictly increasing,
 *                   finite (Sect. 4.1: the linearizing fixed grid)
 *  n_mu, mu, w_mu   direction cosines on [-1, 1] and their weights
 *                   (Gauss-Legendre in the paper).  Must be symmetric:
 *                   n_mu even, mu values pairwise -mu with equal weights, no
 *                   mu = 0, |mu| <= 1, weights > 0 summing to 2.
 *  n_nu, w_nu       frequency quadrature weights (trapezoidal in the paper)
 *  phi[n_atm*n_nu]  absorption profile at the frequency nodes (eqs. J00/J02)
 *  opac[n_atm*n_nu] opacity ratio r_p > 0: the optical-depth step of ray
 *                   (mu_m, nu_p) over an interval is r_p |dtau| / |mu_m|
 *  eps[n_atm]       thermalization parameter in [0, 1]; xi = 1 - eps
 *                   (eqs. S00/S02)
 *  W2[n_atm]        polarizability: sigma20 = xi W2 J20 (W2 = 1 is the
 *                   paper's J_u = 1, J_l = 0 atom)
 *  B[sum ns]        Planck function in the Wien limit (the paper's W = 1);
 *                   NULL means B = 1.  The constant term is c = [eps B, 0].
 *  I_bot[n_atm]     intensity entering at the bottom for mu > 0 (Sect. 3.1:
 *                   1); NULL means B at the deepest point
 *  formal_solver    RT_FS_DELO_LINEAR, RT_FS_TRAPEZOIDAL or RT_FS_IMPLICIT_EULER
 *  normalize_profile  nonzero: divide the spectral weights w_p phi_p by their
 *                   sum so scattering conserves photons on the truncated grid;
 *                   zero: use w_p phi_p as given (the paper's setting)
 *  R                NULL (complete redistribution), or the frequency
 *                   redistribution matrices [n_atm][n_nu][n_nu], R[s][p][q],
 *                   which rt_setup hands to rt_set_redistribution (rt_ext.h):
 *                   the same as calling it after setup
 */
typedef struct rt_problem {
    int n_atm;
    const int *ns;
    const double *tau;
    int n_mu;
    const double *mu;
    const double *w_mu;
    int n_nu;
    const double *w_nu;
    const double *phi;
    const double *opac;
    const double *eps;
    const double *W2;
    const double *B;
    const double *I_bot;
    int formal_solver;
    int normalize_profile;
    const double *R;
} rt_problem;

/*
 * Solver settings (Sect. 4.2).  rt_default_options fills the defaults shown.
 *  precision   RT_PREC_FP64 (default) or RT_PREC_MIXED
 *  restart     GMRES cycle length, 1..RT_MAX_RESTART (30)
 *  maxit       iteration limit per slab: Arnoldi steps for GMRES (over all
 *              restarts and, in MIXED mode, all inner solves), full steps
 *              for BiCGSTAB, updates for Richardson (10000)
 *  rtol        stop when ||b - A x||_2 / ||b||_2 < rtol, the unpreconditioned
 *              relative residual of Sect. 4.2, computed in FP64 (1e-10)
 *  inner_rtol  MIXED: each inner FP32 GMRES solve stops once its Arnoldi
 *              residual estimate falls below inner_rtol times its right-hand
 *              side r (3e-4), or below 0.5 rtol ||b|| where that is looser
 *              (the last refinement step: enough to bring the slab under
 *              rtol, with a factor 2 to spare) ...
 *  inner_maxit MIXED: ... or after this many Arnoldi steps (200)
 *  max_outer   MIXED: refinement steps limit (30)
 *  chunk       formal-solver sweep chunk length: 0 = choose automatically,
 *              else one of 4, 8, 16, 32
 *  wave_batches  ray batches each wavefront of the sweep handles in turn:
 *              0 = choose automatically, else 1..64.  When automatic, a
 *              GMRES cycle that starts with at most 128 slabs iterating
 *              sweeps with at most 8 per wavefront (more workgroups per
 *              slab); a fixed value holds for every cycle
 *  prefetch    step coefficients of the next ray batch loaded while the
 *              current one is swept: 0 = automatic, 1 = no, 2 or 3 = yes
 *              (yes is available for chunk lengths up to 8)
 *  check_every iterations between convergence checks read back by the host
 *              for BiCGSTAB and Richardson (16); GMRES checks once per cycle
 *  sweep_waves wavefronts per sweep workgroup: 0 = automatic, 4 or 8 (8 is
 *              available for chunk lengths up to 8)
 *  graphs      1 = the kernels of one GMRES cycle (of check_every BiCGSTAB or
 *              Richardson iterations) are captured once in a HIP graph and
 *              replayed, the host testing convergence between replays;
 *              0 = kernels launched one by one, GMRES also testing every
 *              check_every steps within a cycle (default: measured faster)
 *  precond     preconditioner of every solver (Sect. 2.3), with A = D + L + U
 *              split into its diagonal and strict lower and upper triangles
 *              in the unknowns' order:
 *              RT_PC_JACOBI (default)  P = D;
 *              RT_PC_SOR               P = omega^-1 D + U;
 *              RT_PC_SSOR              P = omega (2 - omega)^-1
 *                                          (omega^-1 D + U) D^-1 (omega^-1 D + L).
 *              SOR and SSOR need the assembled A (built on the device on the
 *              first solve, (2 ns)^2 doubles per slab, kept by the handle)
 *  omega       relaxation of SOR and SSOR, 0 < omega < 2 (1; the paper uses
 *              1.5 for Richardson, 1 for the Krylov methods)
 *  coef_mode   where the sweep takes its step coefficients from: one of the
 *              RT_COEF_* values above (RT_COEF_AUTO)
 *  autotune    1 = apply the launch plan stored for this problem's shape
 *              (chunk, sweep_waves, prefetch, wave_batches, coef_mode), for
 *              the fields left automatic (0); 0 = do not look (default).  A
 *              stored plan that fails validation for these options is not
 *              applied.  rt_tuned_plan_status reports what was found
 *  plan_file   the plan file autotune reads: NULL means the file named by the
 *              environment variable RT_TUNE_PLANS, else tuned_plans.txt in
 *              the directory of this library.  Text, one plan per line:
 *                key chunk sweep_waves prefetch wave_batches coef_mode source
 *              key as rt_plan_key writes it, source the rt_sweep_source_hash
 *              of the build it was measured with; '#' starts a comment line
 */
typedef struct rt_options {
    int precision;
    int restart;
    int maxit;
    double rtol;
    double inner_rtol;
    int inner_maxit;
    int max_outer;
    int chunk;
    int wave_batches;
    int prefetch;
    int check_every;
    int sweep_waves;
    int graphs;
    int precond;
    double omega;
    int coef_mode;
    int autotune;
    const char *plan_file;
} rt_options;

/* Per-slab outcome of a solve. */
typedef struct rt_solve_info {
    int status;         /* RT_OK, RT_ENOCONV or RT_EBREAKDOWN              */
    int iterations;     /* as counted for maxit                            */
    int matvecs;        /* applications of A (FP64 and FP32)               */
    int outer_steps;    /* MIXED: refinement steps; 0 otherwise            */
    double relres;      /* final ||b - A x|| / ||b||, FP64, recomputed     */
} rt_solve_info;

/* Fill *o with the defaults listed above. */
void rt_default_options(rt_options *o);

/*
 * Validate the problem (no device call happens before validation passes),
 * copy it to the current HIP device and precompute everything the operator
 * needs (Sect. 4.2 notes the action of P^-1 is precomputed):
 *   - per-interval step coefficients of every ray, in FP64 and FP32;
 *   - the quadrature weights of eqs. J00/J02 and the T^2_0 factors of
 *     eqs. sourceI/sourceQ;
 *   - the Jacobi preconditioner P = D = diag(A) (Sect. 2.3), as D^-1;
 *   - the right-hand side b = J t + c (eq. crd_linear_system).
 * On success *h owns all device memory until rt_destroy.  Synchronizes the
 * device before returning.
 * Errors: RT_EINVAL (bad shapes or values; message names the field),
 * RT_ENOMEM, RT_EDEVICE (no usable GPU or a HIP error).
 */
int rt_setup(rt_handle **h, const rt_problem *p, const rt_options *o);

/* Free every device and host resource of h (NULL is allowed). */
void rt_destroy(rt_handle *h);

/* Number of unknowns N = 2 * sum(ns) of the handle's problem. */
int rt_num_unknowns(const rt_handle *h);

/*
 * sigma_out = A sigma_in, A = Id - J Lambda T: Algorithm 1 of the paper,
 * S = T sigma_in (eqs. sourceI/sourceQ), then a formal solution along every
 * ray with zero incoming radiation (eqs. RTE_delo1/2), then the quadrature of
 * eqs. J00/J02 and sigma_out = sigma_in - xi [J00, W2 J20], FP64 throughout.
 * sigma_out may equal sigma_in (in-place); partial overlap is not allowed.
 * Errors: RT_EINVAL (NULL handle or vector), RT_EDEVICE (launch failure).
 */
int rt_apply_op(rt_handle *h, const double *sigma_in, double *sigma_out, void *stream);

/*
 * z = P^-1 v with the Jacobi preconditioner P = D = diag(A) (Sect. 2.3,
 * item 1), elementwise.  z may equal v.
 */
int rt_precond_jacobi(rt_handle *h, const double *v, double *z, void *stream);

/* Copy the right-hand side b = J t + c (eq. crd_linear_system) into b. */
int rt_get_rhs(rt_handle *h, double *b, void *stream);

/* Copy the diagonal D of A into d. */
int rt_get_jacobi_diag(rt_handle *h, double *d, void *stream);

/*
 * Solve A x = b with restarted GMRES (Sect. 2.1; Saad & Schultz), right-
 * preconditioned by Jacobi so the residual it minimizes and stops on is the
 * unpreconditioned one of Sect. 4.2.  Arnoldi runs on the device with
 * classical Gram-Schmidt applied twice (for at most 4 slabs of 1024 points or
 * more, with the second pass delayed by one step, so that the convergence
 * test of a step comes one operator application later); the Hessenberg
 * least-squares problem is solved with Givens rotations in FP64.  In MIXED
 * precision the solve is an FP64 iterative refinement around inner
 * FP32-sweep GMRES solves.
 *  b     right-hand side (device, N); NULL means the handle's own J t + c
 *  x     in: initial guess (the paper uses [1, 0, 1, 0, ...]); out: solution
 *  info  host array of n_atm entries, or NULL
 */
int rt_solve_gmres(rt_handle *h, const double *b, double *x, rt_solve_info *info, void *stream);

/* Same contract, BiCGSTAB (Sect. 2.2; van der Vorst), right-preconditioned by
 * Jacobi.  Breakdown (rho = 0 or (r0, v) = 0 or omega = 0, or a non-finite
 * residual) returns RT_EBREAKDOWN for that slab with x at the last iterate. */
int rt_solve_bicgstab(rt_handle *h, const double *b, double *x, rt_solve_info *info, void *stream);

/* Same contract, the stationary preconditioned Richardson iteration
 * x <- x + D^-1 (b - A x) of eq. rich_iteration (Jacobi).  A non-finite
 * residual returns RT_EBREAKDOWN. */
int rt_solve_richardson(rt_handle *h, const double *b, double *x, rt_solve_info *info, void *stream);

/* Message describing the calling thread's last non-zero return. */
const char *rt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RT_H */
