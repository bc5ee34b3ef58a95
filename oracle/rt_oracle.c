/*
 * rt_oracle.c -- plain, slow, FP64 CPU oracle for the matrix-free operator
 * A = Id - J Lambda T of the 1D two-level-atom scattering-polarization
 * problem (Benedusi, Janett, Belluzzi & Krause, "Krylov methods and
 * matrix-free implementation", Sect. 3) and for the solvers that call it.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the GPU library.
 *
 * The operator is its definition written out: A sigma = sigma - J Lambda T
 * sigma, three maps applied in turn and each coded on its own --
 *   T      the source functions of every direction from sigma
 *          (eqs. sourceI/sourceQ);
 *   Lambda the formal solution of the transfer equation along every ray
 *          (mu_m, nu_p) with zero incoming radiation (Sect. 3.1, 4.1),
 *          giving the whole Stokes field I, Q;
 *   J      the angle-frequency quadrature of eqs. (J00)/(J02) times the
 *          scattering factors of eqs. (S00)/(S02): xi [J00, W2 J20].
 * The right-hand side is b = J t + c with t the transmitted field.  The
 * field is materialized between the maps (no fusion, blocking or
 * reordering).  Built with -ffp-contract=off so every product and sum
 * rounds as written.
 *
 * Readings of the paper taken here (each also recorded in the design notes):
 *  - tau increases downward, tau[0] at the top; mu<0 rays travel downward
 *    (entering at the top), mu>0 rays travel upward (entering at the
 *    bottom) -- boundary conditions of Sect. 3.1.
 *  - the optical-depth step of ray (m,p) over the interval (u,k) is
 *    r_p |tau_k - tau_u| / |mu_m|, r_p an input opacity ratio.
 *  - polarizability W2 scales the emission of sigma^2_0 only:
 *    sigma^2_0 = xi W2 J^2_0 (W2 = 1 is the paper's atom, Sect. 3.1).
 *  - the frequency weights are w_p phi_p, renormalized to sum to one when
 *    `normalize` is set, so that scattering conserves photons on the
 *    truncated frequency grid.
 *  - Planck function B_k (the paper's W = 1) enters as c = [eps B_k, 0].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ns;               /* depth points                                  */
    const double *tau;    /* [ns] optical depth, top first, increasing      */
    int nmu;              /* direction nodes on [-1, 1]                     */
    const double *mu;     /* [nmu]                                          */
    const double *wmu;    /* [nmu] weights, sum 2                           */
    int nnu;              /* frequency nodes                                */
    const double *wnu;    /* [nnu] frequency quadrature weights             */
    const double *phi;    /* [nnu] absorption profile                       */
    const double *opac;   /* [nnu] opacity ratio r_p                        */
    double eps;           /* thermalization parameter, xi = 1 - eps         */
    double W2;            /* polarizability                                 */
    double Ibot;          /* incoming intensity at the bottom for mu > 0    */
    const double *B;      /* [ns] Planck function                           */
    int fs;               /* 0: DELO-linear, 1: trapezoidal, 2: impl. Euler */
    int normalize;        /* renormalize the frequency weights              */
} orc_slab;

/* ------------------------------------------------------------------------
 * Polarization tensor components for gamma = 0 (eqs. sourceI/sourceQ).
 * ---------------------------------------------------------------------- */
void orc_t20(double mu, double *t1, double *t2)
{
    *t1 = sqrt(2.0) * (3.0 * mu * mu - 1.0) / 4.0;
    *t2 = sqrt(2.0) * (3.0 * mu * mu - 3.0) / 4.0;
}

/* ------------------------------------------------------------------------
 * DELO-linear step coefficients (Sect. 4.1; no dichroism, so DELO reduces
 * to an exact integration of a linearly interpolated source function along
 * the ray).  With t the optical path from the upwind point (t = 0) to the
 * current point (t = d):
 *     I_k = E I_u + pu S_u + pk S_k,   E = exp(-d),
 *     pu  = int_0^d (1 - t/d) exp(-(d - t)) dt,
 *     pk  = int_0^d (t/d)     exp(-(d - t)) dt.
 * Closed forms: pu = (1 - (1 + d) E)/d, pk = (1 - E) - pu.  For small d the
 * closed forms cancel, so the Taylor series of the same integrals is used:
 *     pu = sum_{n>=2} (-1)^n (n-1) d^(n-1) / n!
 *     pk = sum_{n>=2} (-1)^n       d^(n-1) / n!
 * ---------------------------------------------------------------------- */
void orc_delo_linear(double d, double *E, double *pu, double *pk)
{
    if (d < 0.1) {
        double term = 1.0;   /* d^(n-1)/n! built incrementally; n = 1 */
        double su = 0.0, sk = 0.0;
        int n;
        for (n = 2; n <= 20; n++) {
            double sgn = (n % 2 == 0) ? 1.0 : -1.0;
            term = term * d / (double)n;        /* now d^(n-1)/n! */
            su += sgn * (double)(n - 1) * term;
            sk += sgn * term;
        }
        *E = exp(-d);
        *pu = su;
        *pk = sk;
    } else {
        double e = exp(-d);
        double w0 = -expm1(-d);
        double w1 = w0 - d * e;
        *E = e;
        *pu = w1 / d;
        *pk = w0 - *pu;
    }
}

/* ------------------------------------------------------------------------
 * Trapezoidal (Crank-Nicolson) step on dI/dt = S - I over one interval:
 *     I_k - I_u = (d/2) [(S_u - I_u) + (S_k - I_k)]
 *  => I_k = a I_u + b (S_u + S_k),  a = (1 - d/2)/(1 + d/2), b = (d/2)/(1 + d/2).
 * Not among the paper's formal solvers; used by the benchmark's second
 * configuration.
 * ---------------------------------------------------------------------- */
void orc_trapezoid(double d, double *a, double *b)
{
    double h = 0.5 * d;
    *a = (1.0 - h) / (1.0 + h);
    *b = h / (1.0 + h);
}

/* ------------------------------------------------------------------------
 * Implicit Euler step (one of the paper's formal solvers, Sect. 4.1): the
 * backward difference of dI/dt = S - I over one interval,
 *     (I_k - I_u) / d = S_k - I_k  =>  I_k = a I_u + b S_k,
 *     a = 1/(1 + d), b = d/(1 + d).
 * ---------------------------------------------------------------------- */
void orc_implicit_euler(double d, double *a, double *b)
{
    *a = 1.0 / (1.0 + d);
    *b = d / (1.0 + d);
}

/* ------------------------------------------------------------------------
 * DELO-parabolic step (Sect. 4.1 names it; the coefficients below are the
 * exact integrals for this problem, which has no dichroism, so DELOPAR --
 * which differs only in how it treats the dichroic term -- coincides with
 * it).  With t the optical path measured from the current point k back
 * towards the upwind point u (t = 0 at k, t = d at u, t = -dd at the
 * downwind point d), S is the parabola through (d, S_u), (0, S_k),
 * (-dd, S_d), and
 *     I_k = E I_u + int_0^d S(t) exp(-t) dt = E I_u + pu S_u + pk S_k + pd S_d.
 * With the moments w_n = int_0^d t^n exp(-t) dt of the Lagrange basis
 *     L_u = t (t + dd) / (d (d + dd)),
 *     L_k = (d - t)(t + dd) / (d dd),
 *     L_d = t (t - d) / (dd (d + dd)):
 *     pu = (w2 + dd w1) / (d (d + dd)),
 *     pk = ((d - dd) w1 + d dd w0 - w2) / (d dd),
 *     pd = (w2 - d w1) / (dd (d + dd)).
 * The moments are 1 - E, 1 - (1 + d) E, 2 - (d^2 + 2 d + 2) E, or below
 * d = 1 (where these cancel) their series
 *     w_n = sum_{m>=0} (-1)^m d^(m+n+1) / (m! (m+n+1)).
 * ---------------------------------------------------------------------- */
void orc_exp_moments(double d, double *w)
{
    int n, m;
    if (d < 1.0) {
        for (n = 0; n < 3; n++) {
            double term = 1.0, sum = 0.0;   /* term = d^m / m! */
            for (m = 0; m <= 30; m++) {
                double sgn = (m % 2 == 0) ? 1.0 : -1.0;
                sum += sgn * term * pow(d, (double)(n + 1)) / (double)(m + n + 1);
                term = term * d / (double)(m + 1);
            }
            w[n] = sum;
        }
    } else {
        double e = exp(-d);
        w[0] = -expm1(-d);
        w[1] = 1.0 - (1.0 + d) * e;
        w[2] = 2.0 - (d * d + 2.0 * d + 2.0) * e;
    }
}

void orc_delo_parabolic(double d, double dd, double *E, double *pu, double *pk, double *pd)
{
    double w[3];
    orc_exp_moments(d, w);
    *E = exp(-d);
    *pu = (w[2] + dd * w[1]) / (d * (d + dd));
    *pk = ((d - dd) * w[1] + d * dd * w[0] - w[2]) / (d * dd);
    *pd = (w[2] - d * w[1]) / (dd * (d + dd));
}

/* ------------------------------------------------------------------------
 * Formal solution along one ray (eqs. RTE_delo1/2 written in optical path
 * along the ray).  kappa = r_p / |mu|.  upward = 0: the ray enters at the
 * top (index 0) and moves to larger tau; upward = 1: it enters at the
 * bottom (index ns-1) and moves to smaller tau.  I[entry] = I_entry.
 * ---------------------------------------------------------------------- */
void orc_ray(int ns, const double *tau, double kappa, int upward, int fs,
             const double *S, double I_entry, double *I)
{
    int k;
    if (!upward) {
        I[0] = I_entry;
        for (k = 1; k < ns; k++) {
            int u = k - 1;
            double d = kappa * fabs(tau[k] - tau[u]);
            if (fs == 3 && k < ns - 1) {      /* parabola through u, k, k + 1 */
                double E, pu, pk, pd;
                orc_delo_parabolic(d, kappa * fabs(tau[k + 1] - tau[k]), &E, &pu, &pk, &pd);
                I[k] = E * I[u] + pu * S[u] + pk * S[k] + pd * S[k + 1];
            } else if (fs == 0 || fs == 3) {  /* DELO-parabolic's last point: linear */
                double E, pu, pk;
                orc_delo_linear(d, &E, &pu, &pk);
                I[k] = E * I[u] + pu * S[u] + pk * S[k];
            } else if (fs == 2) {
                double a, b;
                orc_implicit_euler(d, &a, &b);
                I[k] = a * I[u] + b * S[k];
            } else {
                double a, b;
                orc_trapezoid(d, &a, &b);
                I[k] = a * I[u] + b * (S[u] + S[k]);
            }
        }
    } else {
        I[ns - 1] = I_entry;
        for (k = ns - 2; k >= 0; k--) {
            int u = k + 1;
            double d = kappa * fabs(tau[k] - tau[u]);
            if (fs == 3 && k > 0) {           /* parabola through u, k, k - 1 */
                double E, pu, pk, pd;
                orc_delo_parabolic(d, kappa * fabs(tau[k] - tau[k - 1]), &E, &pu, &pk, &pd);
                I[k] = E * I[u] + pu * S[u] + pk * S[k] + pd * S[k - 1];
            } else if (fs == 0 || fs == 3) {
                double E, pu, pk;
                orc_delo_linear(d, &E, &pu, &pk);
                I[k] = E * I[u] + pu * S[u] + pk * S[k];
            } else if (fs == 2) {
                double a, b;
                orc_implicit_euler(d, &a, &b);
                I[k] = a * I[u] + b * S[k];
            } else {
                double a, b;
                orc_trapezoid(d, &a, &b);
                I[k] = a * I[u] + b * (S[u] + S[k]);
            }
        }
    }
}

/* ------------------------------------------------------------------------
 * Quadrature weights of eqs. (J00)/(J02): the angular integral
 * (1/2) int dmu over [-1, 1] with the given nodes, times the spectral
 * integral int dnu phi with weights w_p phi_p (renormalized if asked).
 * q[m * nnu + p].
 * ---------------------------------------------------------------------- */
void orc_weights(const orc_slab *s, double *q)
{
    int m, p;
    double norm = 1.0;
    if (s->normalize) {
        double sum = 0.0;
        for (p = 0; p < s->nnu; p++) sum += s->wnu[p] * s->phi[p];
        norm = sum;
    }
    for (m = 0; m < s->nmu; m++)
        for (p = 0; p < s->nnu; p++)
            q[m * s->nnu + p] = 0.5 * s->wmu[m] * (s->wnu[p] * s->phi[p] / norm);
}

/* ------------------------------------------------------------------------
 * The three maps of A = Id - J Lambda T (Sect. 3.2).  A field holds the
 * Stokes I and Q of every ray at every depth, index
 * ((st * nmu + m) * nnu + p) * ns + k, st = 0 for I, 1 for Q.
 *   field_J:          sig = xi [J00, W2 J20] of a field (eqs. J00/J02,
 *                     S00/S02);
 *   field_from_sigma: F = Lambda T sig, the formal solution of every ray
 *                     with the source functions of sig (eqs.
 *                     sourceI/sourceQ), plus the transmitted field t when
 *                     with_t is set (I_bot entering at the bottom for
 *                     mu > 0, nothing at the top, Q = 0).
 * The same maps give the formulation with the field as unknown (eq.
 * crd_linear_system2): (Id - Lambda T J) I = Lambda T c + t, sigma = J I + c.
 * ---------------------------------------------------------------------- */
static void field_J(const orc_slab *s, const double *q, const double *F, double *sig)
{
    int ns = s->ns, nmu = s->nmu, nnu = s->nnu, k, m, p;
    double xi = 1.0 - s->eps;
    for (k = 0; k < 2 * ns; k++) sig[k] = 0.0;
    for (m = 0; m < nmu; m++) {
        double t1, t2;
        orc_t20(s->mu[m], &t1, &t2);
        for (p = 0; p < nnu; p++) {
            const double *I = F + ((size_t)(0 * nmu + m) * nnu + p) * ns;
            const double *Q = F + ((size_t)(1 * nmu + m) * nnu + p) * ns;
            double w = q[m * nnu + p];
            for (k = 0; k < ns; k++) {
                sig[2 * k] += w * I[k];
                sig[2 * k + 1] += w * (t1 * I[k] + t2 * Q[k]);
            }
        }
    }
    for (k = 0; k < ns; k++) {
        sig[2 * k] *= xi;
        sig[2 * k + 1] *= xi * s->W2;
    }
}

/* F = Lambda T sig, plus the transmitted field t when with_t is set. */
static int field_from_sigma(const orc_slab *s, const double *sig, int with_t, double *F)
{
    int ns = s->ns, nmu = s->nmu, nnu = s->nnu, k, m, p;
    double *SI = (double *)malloc(sizeof(double) * ns);
    double *SQ = (double *)malloc(sizeof(double) * ns);
    if (!SI || !SQ) { free(SI); free(SQ); return -1; }
    for (m = 0; m < nmu; m++) {
        double t1, t2;
        int upward = s->mu[m] > 0.0;
        orc_t20(s->mu[m], &t1, &t2);
        for (k = 0; k < ns; k++) {
            SI[k] = sig[2 * k] + t1 * sig[2 * k + 1];
            SQ[k] = t2 * sig[2 * k + 1];
        }
        for (p = 0; p < nnu; p++) {
            double kappa = s->opac[p] / fabs(s->mu[m]);
            double inflow = (with_t && upward) ? s->Ibot : 0.0;
            orc_ray(ns, s->tau, kappa, upward, s->fs, SI, inflow,
                    F + ((size_t)(0 * nmu + m) * nnu + p) * ns);
            orc_ray(ns, s->tau, kappa, upward, s->fs, SQ, 0.0,
                    F + ((size_t)(1 * nmu + m) * nnu + p) * ns);
        }
    }
    free(SI); free(SQ);
    return 0;
}

/* A sigma = sigma - J Lambda T sigma, sigma interleaved
 * [s00(z1), s20(z1), s00(z2), ...] (Sect. 3.2). */
int orc_apply(const orc_slab *s, const double *sin, double *sout)
{
    size_t nf = (size_t)2 * s->ns * s->nmu * s->nnu;
    int i, rc = -1;
    double *F = (double *)malloc(sizeof(double) * nf);
    double *q = (double *)malloc(sizeof(double) * s->nmu * s->nnu);
    double *em = (double *)malloc(sizeof(double) * 2 * s->ns);
    if (F && q && em) {
        orc_weights(s, q);
        rc = field_from_sigma(s, sin, 0, F);
        if (rc == 0) {
            field_J(s, q, F, em);
            for (i = 0; i < 2 * s->ns; i++) sout[i] = sin[i] - em[i];
        }
    }
    free(F); free(q); free(em);
    return rc;
}

/* Iout = Iin - Lambda T J Iin. */
int orc_apply_I(const orc_slab *s, const double *Iin, double *Iout)
{
    size_t n = (size_t)2 * s->ns * s->nmu * s->nnu, i;
    double *q = (double *)malloc(sizeof(double) * s->nmu * s->nnu);
    double *sig = (double *)malloc(sizeof(double) * 2 * s->ns);
    double *F = (double *)malloc(sizeof(double) * n);
    int rc = -1;
    if (q && sig && F) {
        orc_weights(s, q);
        field_J(s, q, Iin, sig);
        rc = field_from_sigma(s, sig, 0, F);
        for (i = 0; i < n && rc == 0; i++) Iout[i] = Iin[i] - F[i];
    }
    free(q); free(sig); free(F);
    return rc;
}

/* bI = Lambda T c + t, c = [eps B, 0]. */
int orc_rhs_I(const orc_slab *s, double *bI)
{
    int k;
    double *c = (double *)malloc(sizeof(double) * 2 * s->ns);
    int rc;
    if (!c) return -1;
    for (k = 0; k < s->ns; k++) {
        c[2 * k] = s->eps * s->B[k];
        c[2 * k + 1] = 0.0;
    }
    rc = field_from_sigma(s, c, 1, bI);
    free(c);
    return rc;
}

/* sigma = J I + c. */
int orc_sigma_from_I(const orc_slab *s, const double *I, double *sigma)
{
    int k;
    double *q = (double *)malloc(sizeof(double) * s->nmu * s->nnu);
    if (!q) return -1;
    orc_weights(s, q);
    field_J(s, q, I, sigma);
    for (k = 0; k < s->ns; k++) sigma[2 * k] += s->eps * s->B[k];
    free(q);
    return 0;
}

/* ------------------------------------------------------------------------
 * Right-hand side b = J t + c (eq. crd_linear_system): t is the radiation
 * transmitted from the boundaries (S = 0, I = Ibot entering at the bottom
 * for mu > 0, I = 0 entering at the top, Q = 0 everywhere), c = [eps B, 0].
 * ---------------------------------------------------------------------- */
int orc_rhs(const orc_slab *s, double *b)
{
    size_t nf = (size_t)2 * s->ns * s->nmu * s->nnu;
    int k, rc = -1;
    double *zero = (double *)calloc((size_t)2 * s->ns, sizeof(double));
    double *F = (double *)malloc(sizeof(double) * nf);
    double *q = (double *)malloc(sizeof(double) * s->nmu * s->nnu);
    if (zero && F && q) {
        orc_weights(s, q);
        rc = field_from_sigma(s, zero, 1, F);
        if (rc == 0) {
            field_J(s, q, F, b);
            for (k = 0; k < s->ns; k++) b[2 * k] = b[2 * k] + s->eps * s->B[k];
        }
    }
    free(zero); free(F); free(q);
    return rc;
}

/* ------------------------------------------------------------------------
 * Diagonal entries of A by their definition: d_i = (A e_i)_i, one matvec
 * per requested index (column-by-column assembly, Sect. 3.3).
 * ---------------------------------------------------------------------- */
int orc_diag(const orc_slab *s, int nidx, const int *idx, double *d)
{
    int n = 2 * s->ns, j;
    double *e = (double *)calloc(n, sizeof(double));
    double *col = (double *)malloc(sizeof(double) * n);
    if (!e || !col) { free(e); free(col); return -1; }
    for (j = 0; j < nidx; j++) {
        int i = idx[j];
        e[i] = 1.0;
        orc_apply(s, e, col);
        d[j] = col[i];
        e[i] = 0.0;
    }
    free(e); free(col);
    return 0;
}

/* Column-by-column assembly of the full A (n x n, row-major). */
int orc_assemble(const orc_slab *s, double *A)
{
    int n = 2 * s->ns, i, j;
    double *e = (double *)calloc(n, sizeof(double));
    double *col = (double *)malloc(sizeof(double) * n);
    if (!e || !col) { free(e); free(col); return -1; }
    for (j = 0; j < n; j++) {
        e[j] = 1.0;
        orc_apply(s, e, col);
        for (i = 0; i < n; i++) A[i * n + j] = col[i];
        e[j] = 0.0;
    }
    free(e); free(col);
    return 0;
}

/* ------------------------------------------------------------------------
 * Solvers.  All are right-preconditioned by P^-1 (identity if pc is NULL),
 * so the residual they stop on is the unpreconditioned ||b - A x||_2 /
 * ||b||_2 of Sect. 4.2 (GMRES can also precondition from the left).
 *
 * Preconditioners of Sect. 2.3, with A = D + L + U split into its diagonal
 * and strictly lower and upper triangles (unknowns ordered as sigma, top
 * depth point first) and 0 < omega < 2:
 *   Jacobi  P = D;
 *   SOR     P = omega^-1 D + U;
 *   SSOR    P = omega (2 - omega)^-1 (omega^-1 D + U) D^-1 (omega^-1 D + L).
 * Sect. 2.3 prints SOR as omega^-1 D + L (or + U) and SSOR with the lower
 * factor first, and Sect. 4.2 names the upper-triangle variant; numbering
 * the depth points from the bottom turns the printed lower factor into the
 * upper one here.  These are the forms whose iteration counts equal the
 * paper's SOR and SSOR tables.
 *
 * Status: 0 converged, 1 iteration limit reached, 2 breakdown, -1 memory.
 * ---------------------------------------------------------------------- */
enum { ORC_PC_NONE = 0, ORC_PC_JACOBI = 1, ORC_PC_SOR = 2, ORC_PC_SSOR = 3 };

typedef struct {
    int kind;             /* ORC_PC_*                                        */
    const double *dinv;   /* Jacobi: [n] reciprocals of diag(A)              */
    const double *A;      /* SOR, SSOR: [n*n] assembled A, row-major         */
    double omega;         /* SOR, SSOR relaxation parameter                  */
} orc_prec;
static double dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    int i;
    for (i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

static double nrm2(int n, const double *a) { return sqrt(dot(n, a, a)); }

/* z = P^-1 v; z and v must not alias for SOR and SSOR. */
static void precond(int n, const orc_prec *pc, const double *v, double *z)
{
    int i, j;
    const double *A;
    double om;
    if (!pc || pc->kind == ORC_PC_NONE) {
        for (i = 0; i < n; i++) z[i] = v[i];
        return;
    }
    if (pc->kind == ORC_PC_JACOBI) {
        for (i = 0; i < n; i++) z[i] = pc->dinv[i] * v[i];
        return;
    }
    A = pc->A;
    om = pc->omega;
    /* (omega^-1 D + U) z = v, back substitution from the last unknown */
    for (i = n - 1; i >= 0; i--) {
        double sum = v[i];
        for (j = i + 1; j < n; j++) sum -= A[(size_t)i * n + j] * z[j];
        z[i] = sum / (A[(size_t)i * n + i] / om);
    }
    if (pc->kind != ORC_PC_SSOR) return;
    /* then multiply by D, solve (omega^-1 D + L) z' = D z forward, and scale */
    for (i = 0; i < n; i++) z[i] = A[(size_t)i * n + i] * z[i];
    for (i = 0; i < n; i++) {
        double sum = z[i];
        for (j = 0; j < i; j++) sum -= A[(size_t)i * n + j] * z[j];
        z[i] = sum / (A[(size_t)i * n + i] / om);
    }
    for (i = 0; i < n; i++) z[i] = z[i] * ((2.0 - om) / om);
}

static void residual(const orc_slab *s, const double *b, const double *x, double *r)
{
    int n = 2 * s->ns, i;
    orc_apply(s, x, r);
    for (i = 0; i < n; i++) r[i] = b[i] - r[i];
}

/*
 * GMRES(m) (Saad & Schultz 1986; Sect. 2.1): Arnoldi with modified
 * Gram-Schmidt builds an orthonormal basis of the Krylov space of A P^-1,
 * Givens rotations reduce the Hessenberg least-squares problem, and
 * x = x0 + P^-1 V y minimizes ||b - A x||_2.  After each cycle the residual
 * is recomputed explicitly and the method restarts from x.
 * restart <= 0 means no restart (cycle length = maxit).
 * iters counts Arnoldi steps; matvecs counts every application of A.
 * left != 0 selects left preconditioning instead: the basis spans the Krylov
 * space of P^-1 A, x = x0 + V y, and both the minimized quantity and the
 * stopping test use the preconditioned residual ||P^-1 (b - A x)|| relative
 * to ||P^-1 b||.  Without a preconditioner the two variants coincide.
 */
int orc_gmres(const orc_slab *s, const double *b, double *x, const orc_prec *pc,
              int restart, double tol, int maxit, int *iters, int *matvecs,
              double *relres, double *hist, int hist_len, int left)
{
    int n = 2 * s->ns;
    int m = (restart <= 0 || restart > maxit) ? maxit : restart;
    int total = 0, nmv = 0, status = 1, i, j, jj;
    double bnorm, beta;
    double *V = (double *)malloc(sizeof(double) * (size_t)n * (m + 1));
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * m);
    double *sn = (double *)malloc(sizeof(double) * m);
    double *g = (double *)malloc(sizeof(double) * (m + 1));
    double *y = (double *)malloc(sizeof(double) * m);
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    if (!V || !H || !cs || !sn || !g || !y || !r || !z || !w) { status = -1; goto done; }

    left = left && pc && pc->kind != ORC_PC_NONE;
    if (left) {
        precond(n, pc, b, z);
        bnorm = nrm2(n, z);
    } else {
        bnorm = nrm2(n, b);
    }
    if (bnorm == 0.0) {
        for (i = 0; i < n; i++) x[i] = 0.0;
        if (relres) *relres = 0.0;
        status = 0;
        goto done;
    }
    residual(s, b, x, r); nmv++;
    if (left) { precond(n, pc, r, z); memcpy(r, z, sizeof(double) * n); }
    beta = nrm2(n, r);
    if (hist && hist_len > 0) hist[0] = beta / bnorm;
    if (beta / bnorm < tol) { status = 0; goto done_res; }

    while (total < maxit) {
        for (i = 0; i < n; i++) V[i] = r[i] / beta;
        for (i = 0; i <= m; i++) g[i] = 0.0;
        g[0] = beta;
        memset(H, 0, sizeof(double) * (size_t)(m + 1) * m);
        jj = 0;
        for (j = 0; j < m && total < maxit; j++) {
            double hnext, resid, tmp, den;
            if (left) {
                orc_apply(s, V + (size_t)j * n, z); nmv++;
                precond(n, pc, z, w);
            } else {
                precond(n, pc, V + (size_t)j * n, z);
                orc_apply(s, z, w); nmv++;
            }
            total++;
            for (i = 0; i <= j; i++) {     /* modified Gram-Schmidt */
                int l;
                double h = dot(n, w, V + (size_t)i * n);
                H[i * m + j] = h;
                for (l = 0; l < n; l++) w[l] -= h * V[(size_t)i * n + l];
            }
            hnext = nrm2(n, w);
            H[(j + 1) * m + j] = hnext;
            for (i = 0; i < j; i++) {      /* previous rotations */
                tmp = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = tmp;
            }
            den = sqrt(H[j * m + j] * H[j * m + j] + hnext * hnext);
            cs[j] = H[j * m + j] / den;
            sn[j] = hnext / den;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            resid = fabs(g[j + 1]);
            if (hist && total < hist_len) hist[total] = resid / bnorm;
            jj = j + 1;
            if (hnext != 0.0) {
                for (i = 0; i < n; i++) V[(size_t)(j + 1) * n + i] = w[i] / hnext;
            }
            if (resid / bnorm < tol || hnext == 0.0) break;
        }
        /* back substitution H y = g, then x += P^-1 V y (left: x += V y) */
        for (i = jj - 1; i >= 0; i--) {
            double sum = g[i];
            int l;
            for (l = i + 1; l < jj; l++) sum -= H[i * m + l] * y[l];
            y[i] = sum / H[i * m + i];
        }
        for (i = 0; i < n; i++) w[i] = 0.0;
        for (j = 0; j < jj; j++)
            for (i = 0; i < n; i++) w[i] += y[j] * V[(size_t)j * n + i];
        if (left) memcpy(z, w, sizeof(double) * n);
        else precond(n, pc, w, z);
        for (i = 0; i < n; i++) x[i] += z[i];
        residual(s, b, x, r); nmv++;
        if (left) { precond(n, pc, r, z); memcpy(r, z, sizeof(double) * n); }
        beta = nrm2(n, r);
        if (beta / bnorm < tol) { status = 0; break; }
        if (beta == 0.0) { status = 0; break; }
    }
done_res:
    if (relres) *relres = nrm2(n, r) / bnorm;
done:
    if (iters) *iters = total;
    if (matvecs) *matvecs = nmv;
    free(V); free(H); free(cs); free(sn); free(g); free(y); free(r); free(z); free(w);
    return status;
}

/*
 * BiCGSTAB (van der Vorst 1992; Sect. 2.2), right-preconditioned.
 * iters counts full steps (two applications of A each); a step that
 * converges on its half-way residual s counts as a full step.
 */
int orc_bicgstab(const orc_slab *s, const double *b, double *x, const orc_prec *pc,
                 double tol, int maxit, int *iters, int *matvecs, double *relres)
{
    int n = 2 * s->ns, it, i, status = 1, nmv = 0;
    double bnorm = nrm2(n, b);
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    double *r = (double *)malloc(sizeof(double) * n);
    double *rh = (double *)malloc(sizeof(double) * n);
    double *p = (double *)calloc(n, sizeof(double));
    double *v = (double *)calloc(n, sizeof(double));
    double *ph = (double *)malloc(sizeof(double) * n);
    double *sv = (double *)malloc(sizeof(double) * n);
    double *sh = (double *)malloc(sizeof(double) * n);
    double *t = (double *)malloc(sizeof(double) * n);
    it = 0;
    if (!r || !rh || !p || !v || !ph || !sv || !sh || !t) { status = -1; goto done; }
    if (bnorm == 0.0) {
        for (i = 0; i < n; i++) x[i] = 0.0;
        if (relres) *relres = 0.0;
        status = 0;
        goto done;
    }
    residual(s, b, x, r); nmv++;
    if (nrm2(n, r) / bnorm < tol) { status = 0; goto done_res; }
    for (i = 0; i < n; i++) rh[i] = r[i];
    for (it = 1; it <= maxit; it++) {
        double rho = dot(n, rh, r), beta, rv, tt;
        if (rho == 0.0 || !isfinite(rho)) { status = 2; it--; break; }
        beta = (rho / rho_old) * (alpha / omega);
        for (i = 0; i < n; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        precond(n, pc, p, ph);
        orc_apply(s, ph, v); nmv++;
        rv = dot(n, rh, v);
        if (rv == 0.0 || !isfinite(rv)) { status = 2; it--; break; }
        alpha = rho / rv;
        for (i = 0; i < n; i++) sv[i] = r[i] - alpha * v[i];
        if (nrm2(n, sv) / bnorm < tol) {
            for (i = 0; i < n; i++) x[i] += alpha * ph[i];
            status = 0;
            break;
        }
        precond(n, pc, sv, sh);
        orc_apply(s, sh, t); nmv++;
        tt = dot(n, t, t);
        if (tt == 0.0) { status = 2; break; }
        omega = dot(n, t, sv) / tt;
        for (i = 0; i < n; i++) x[i] += alpha * ph[i] + omega * sh[i];
        for (i = 0; i < n; i++) r[i] = sv[i] - omega * t[i];
        if (nrm2(n, r) / bnorm < tol) { status = 0; break; }
        if (omega == 0.0 || !isfinite(omega)) { status = 2; break; }
        rho_old = rho;
    }
    if (it > maxit) it = maxit;
    residual(s, b, x, r); nmv++;
done_res:
    if (relres) *relres = nrm2(n, r) / bnorm;
done:
    if (iters) *iters = it;
    if (matvecs) *matvecs = nmv;
    free(r); free(rh); free(p); free(v); free(ph); free(sv); free(sh); free(t);
    return status;
}

/*
 * Conjugate gradient squared (Sonneveld 1989; Sect. 2.2), right-
 * preconditioned.  Each step squares the BCG residual polynomial with two
 * products by A and none by A^T:
 *   rho = (rh, r);  beta = rho / rho_old (first step: u = p = r)
 *   u = r + beta q;  p = u + beta (q + beta p)
 *   v = A P^-1 p;  alpha = rho / (rh, v);  q = u - alpha v
 *   x += alpha P^-1 (u + q);  r -= alpha A P^-1 (u + q).
 * iters counts full steps (two products each); convergence is tested on the
 * recursively updated residual after each step, and the returned relres is
 * recomputed from x.
 */
int orc_cgs(const orc_slab *s, const double *b, double *x, const orc_prec *pc,
            double tol, int maxit, int *iters, int *matvecs, double *relres)
{
    int n = 2 * s->ns, it, i, status = 1, nmv = 0;
    double bnorm = nrm2(n, b), rho_old = 1.0;
    double *r = (double *)malloc(sizeof(double) * n);
    double *rh = (double *)malloc(sizeof(double) * n);
    double *u = (double *)malloc(sizeof(double) * n);
    double *p = (double *)calloc(n, sizeof(double));
    double *q = (double *)calloc(n, sizeof(double));
    double *v = (double *)malloc(sizeof(double) * n);
    double *ph = (double *)malloc(sizeof(double) * n);
    double *uq = (double *)malloc(sizeof(double) * n);
    double *uh = (double *)malloc(sizeof(double) * n);
    it = 0;
    if (!r || !rh || !u || !p || !q || !v || !ph || !uq || !uh) { status = -1; goto done; }
    if (bnorm == 0.0) {
        for (i = 0; i < n; i++) x[i] = 0.0;
        if (relres) *relres = 0.0;
        status = 0;
        goto done;
    }
    residual(s, b, x, r); nmv++;
    if (nrm2(n, r) / bnorm < tol) { status = 0; goto done_res; }
    for (i = 0; i < n; i++) rh[i] = r[i];
    for (it = 1; it <= maxit; it++) {
        double rho = dot(n, rh, r), alpha, sig;
        if (rho == 0.0 || !isfinite(rho)) { status = 2; it--; break; }
        if (it == 1) {
            for (i = 0; i < n; i++) { u[i] = r[i]; p[i] = u[i]; }
        } else {
            double beta = rho / rho_old;
            for (i = 0; i < n; i++) {
                u[i] = r[i] + beta * q[i];
                p[i] = u[i] + beta * (q[i] + beta * p[i]);
            }
        }
        precond(n, pc, p, ph);
        orc_apply(s, ph, v); nmv++;
        sig = dot(n, rh, v);
        if (sig == 0.0 || !isfinite(sig)) { status = 2; it--; break; }
        alpha = rho / sig;
        for (i = 0; i < n; i++) {
            q[i] = u[i] - alpha * v[i];
            uq[i] = u[i] + q[i];
        }
        precond(n, pc, uq, uh);
        for (i = 0; i < n; i++) x[i] += alpha * uh[i];
        orc_apply(s, uh, v); nmv++;              /* v now holds A P^-1 (u + q) */
        for (i = 0; i < n; i++) r[i] -= alpha * v[i];
        if (nrm2(n, r) / bnorm < tol) { status = 0; break; }
        rho_old = rho;
    }
    if (it > maxit) it = maxit;
    residual(s, b, x, r); nmv++;
done_res:
    if (relres) *relres = nrm2(n, r) / bnorm;
done:
    if (iters) *iters = it;
    if (matvecs) *matvecs = nmv;
    free(r); free(rh); free(u); free(p); free(q); free(v); free(ph); free(uq); free(uh);
    return status;
}

/*
 * Preconditioned Richardson iteration x <- x + P^-1 (b - A x)
 * (eq. rich_iteration).  iters = number of updates applied when the
 * relative residual first drops below tol.
 */
int orc_richardson(const orc_slab *s, const double *b, double *x, const orc_prec *pc,
                   double tol, int maxit, int *iters, int *matvecs, double *relres)
{
    int n = 2 * s->ns, it, i, status = 1, nmv = 0;
    double bnorm = nrm2(n, b), rel = 0.0;
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    if (!r || !z) { free(r); free(z); return -1; }
    if (bnorm == 0.0) {
        for (i = 0; i < n; i++) x[i] = 0.0;
        if (iters) *iters = 0;
        if (matvecs) *matvecs = 0;
        if (relres) *relres = 0.0;
        free(r); free(z);
        return 0;
    }
    for (it = 0;; it++) {
        residual(s, b, x, r); nmv++;
        rel = nrm2(n, r) / bnorm;
        if (rel < tol) { status = 0; break; }
        if (!isfinite(rel)) { status = 2; break; }   /* diverged */
        if (it == maxit) { status = 1; break; }
        precond(n, pc, r, z);
        for (i = 0; i < n; i++) x[i] += z[i];
    }
    if (iters) *iters = it;
    if (matvecs) *matvecs = nmv;
    if (relres) *relres = rel;
    free(r); free(z);
    return status;
}
