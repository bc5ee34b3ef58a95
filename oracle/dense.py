"""Dense route to the same operator, for tiny grids (test infrastructure only).

An independent construction of the matrices of Sect. 3.2 of the paper:
  * T (eq. matricial_form_2) maps sigma to the source functions S_I, S_Q,
  * Lambda (eq. matricial_form_3) maps S to the Stokes field, one dense
    block per ray built as L^-1 M by a triangular solve (no recurrence),
  * J (eq. matricial_form_1) maps the field to xi [J00, W2 J20],
  * t is the transmitted field, c = [eps B, 0],
then A = Id - J Lambda T and b = J t + c (eq. crd_linear_system), solved by
LAPACK LU.  The alternative system (Id - Lambda T J) I = Lambda T c + t
(eq. crd_linear_system2) is also formed.

Only the per-interval step coefficients are taken from the oracle library
(they are pinned on their own against the integrals that define them); the
assembly order, the linear algebra and the quadrature here are separate code.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import oracle as O


def _ray_matrices(tau, kappa, upward, fs):
    """Lambda (ns x ns) for one ray and the transmitted profile for unit
    incoming intensity.  Points are ordered along the ray, L I = M S with
    L unit lower bidiagonal (-a on the sub-diagonal), M holding the
    coefficients of S_u (sub-diagonal), S_k (diagonal) and, for
    DELO-parabolic, S_d (super-diagonal); the entry row of M is zero (zero
    incoming radiation)."""
    ns = tau.shape[0]
    order = np.arange(ns)[::-1] if upward else np.arange(ns)
    t = tau[order]
    L = np.eye(ns)
    M = np.zeros((ns, ns))
    for j in range(1, ns):
        d = kappa * abs(t[j] - t[j - 1])
        if fs == 3 and j < ns - 1:
            # DELO-parabolic: a third coefficient, on the downwind source
            E, pu, pk, pd = O.delo_parabolic(d, kappa * abs(t[j + 1] - t[j]))
            a, cu, ck = E, pu, pk
            M[j, j + 1] = pd
        elif fs in (0, 3):
            E, pu, pk = O.delo_linear(d)
            a, cu, ck = E, pu, pk
        elif fs == 2:
            a, ck = O.implicit_euler(d)
            cu = 0.0
        else:
            a, b = O.trapezoid(d)
            cu = ck = b
        L[j, j - 1] = -a
        M[j, j - 1] = cu
        M[j, j] = ck
    Lam_ray = sla.solve_triangular(L, M, lower=True, unit_diagonal=True)
    e0 = np.zeros(ns)
    e0[0] = 1.0
    trans_ray = sla.solve_triangular(L, e0, lower=True, unit_diagonal=True)
    # back to depth order
    P = np.zeros((ns, ns))
    P[np.arange(ns), order] = 1.0           # P @ v_depth = v_ray
    Lam = P.T @ Lam_ray @ P
    trans = P.T @ trans_ray
    return Lam, trans


class Dense:
    """Explicit T, Lambda, J, t, c for one slab of ``prob``.

    Field ordering: index ((s * nmu + m) * nnu + p) * ns + k with s = 0 for
    I and s = 1 for Q.  Source ordering: (s * nmu + m) * ns + k.
    """

    def __init__(self, prob, i=0):
        ns = int(prob.ns[i])
        off = prob.offsets
        tau = prob.tau[off[i]:off[i + 1]]
        B = prob.B[off[i]:off[i + 1]]
        mu, wmu = prob.mu, prob.w_mu
        wnu, phi, opac = prob.w_nu, prob.phi[i], prob.opac[i]
        nmu, nnu = mu.shape[0], wnu.shape[0]
        eps, W2, Ibot = float(prob.eps[i]), float(prob.W2[i]), float(prob.I_bot[i])
        xi = 1.0 - eps
        fs = int(prob.formal_solver)
        self.ns, self.nmu, self.nnu = ns, nmu, nnu
        nsig, nsrc, nfld = 2 * ns, 2 * ns * nmu, 2 * ns * nmu * nnu

        # spectral weights of the J integrals
        wp = wnu * phi
        if prob.normalize_profile:
            wp = wp / wp.sum()
        t1 = np.sqrt(2.0) * (3.0 * mu ** 2 - 1.0) / 4.0
        t2 = np.sqrt(2.0) * (3.0 * mu ** 2 - 3.0) / 4.0

        # T: S_I(k,m) = s00_k + t1_m s20_k ; S_Q(k,m) = t2_m s20_k
        T = np.zeros((nsrc, nsig))
        for m in range(nmu):
            for k in range(ns):
                T[(0 * nmu + m) * ns + k, 2 * k] = 1.0
                T[(0 * nmu + m) * ns + k, 2 * k + 1] = t1[m]
                T[(1 * nmu + m) * ns + k, 2 * k + 1] = t2[m]

        # Lambda and t: block diagonal over (stokes, m, p)
        Lam = np.zeros((nfld, nsrc))
        tvec = np.zeros(nfld)
        for m in range(nmu):
            up = mu[m] > 0
            for p in range(nnu):
                Lr, tr = _ray_matrices(tau, opac[p] / abs(mu[m]), up, fs)
                for s in range(2):
                    r0 = ((s * nmu + m) * nnu + p) * ns
                    c0 = (s * nmu + m) * ns
                    Lam[r0:r0 + ns, c0:c0 + ns] = Lr
                if up:   # I enters at the bottom with Ibot; Q enters with 0
                    r0 = ((0 * nmu + m) * nnu + p) * ns
                    tvec[r0:r0 + ns] = Ibot * tr

        # J: sigma00 = xi sum_mp (w_m/2) wp_p I ; sigma20 = xi W2 sum (w_m/2) wp_p (t1 I + t2 Q)
        J = np.zeros((nsig, nfld))
        for m in range(nmu):
            for p in range(nnu):
                w = 0.5 * wmu[m] * wp[p]
                for k in range(ns):
                    iI = ((0 * nmu + m) * nnu + p) * ns + k
                    iQ = ((1 * nmu + m) * nnu + p) * ns + k
                    J[2 * k, iI] = xi * w
                    J[2 * k + 1, iI] = xi * W2 * w * t1[m]
                    J[2 * k + 1, iQ] = xi * W2 * w * t2[m]
        c = np.zeros(nsig)
        c[0::2] = eps * B

        self.T, self.Lam, self.J, self.t, self.c = T, Lam, J, tvec, c
        self.A = np.eye(nsig) - J @ Lam @ T
        self.b = J @ tvec + c

    def solve(self):
        """LAPACK LU solve of A sigma = b."""
        lu = sla.lu_factor(self.A)
        return sla.lu_solve(lu, self.b)

    def solve_I_formulation(self):
        """Solve (Id - Lambda T J) I = Lambda T c + t and map back by
        sigma = J I + c (eq. crd_linear_system2)."""
        n = self.Lam.shape[0]
        K = np.eye(n) - self.Lam @ self.T @ self.J
        rhs = self.Lam @ self.T @ self.c + self.t
        I = sla.lu_solve(sla.lu_factor(K), rhs)
        return self.J @ I + self.c, I


def redistribution_matrix_A(prob, R, i=0):
    """Explicit A of the redistribution variant on a tiny grid: unknowns
    (k * n_nu + p) * 2 + K, A = Id - C Jm Lambda T with T the per-frequency
    source map, Lambda the per-ray blocks of _ray_matrices, Jm the
    monochromatic angle quadrature and C the redistribution
    sum_p' R(p, p') w_p' (.) / phi_p with xi W_K."""
    ns = int(prob.ns[i])
    off = prob.offsets
    tau = prob.tau[off[i]:off[i + 1]]
    mu, wmu = prob.mu, prob.w_mu
    wnu, phi, opac = prob.w_nu, prob.phi[i], prob.opac[i]
    nmu, nnu = mu.shape[0], wnu.shape[0]
    xi, W2 = 1.0 - float(prob.eps[i]), float(prob.W2[i])
    t1 = np.sqrt(2.0) * (3.0 * mu ** 2 - 1.0) / 4.0
    t2 = np.sqrt(2.0) * (3.0 * mu ** 2 - 3.0) / 4.0
    nsig, nfld = 2 * ns * nnu, 2 * ns * nmu * nnu

    def sidx(k, p, K):
        return (k * nnu + p) * 2 + K

    def fidx(st, m, p, k):
        return ((st * nmu + m) * nnu + p) * ns + k

    T = np.zeros((nfld, nsig))   # sources, laid out like the field
    for m in range(nmu):
        for p in range(nnu):
            for k in range(ns):
                T[fidx(0, m, p, k), sidx(k, p, 0)] = 1.0
                T[fidx(0, m, p, k), sidx(k, p, 1)] = t1[m]
                T[fidx(1, m, p, k), sidx(k, p, 1)] = t2[m]
    Lam = np.zeros((nfld, nfld))
    for m in range(nmu):
        for p in range(nnu):
            Lr, _ = _ray_matrices(tau, opac[p] / abs(mu[m]), mu[m] > 0, int(prob.formal_solver))
            for st in range(2):
                r0 = fidx(st, m, p, 0)
                Lam[r0:r0 + ns, r0:r0 + ns] = Lr
    Jm = np.zeros((nsig, nfld))
    for m in range(nmu):
        for p in range(nnu):
            for k in range(ns):
                Jm[sidx(k, p, 0), fidx(0, m, p, k)] = 0.5 * wmu[m]
                Jm[sidx(k, p, 1), fidx(0, m, p, k)] = 0.5 * wmu[m] * t1[m]
                Jm[sidx(k, p, 1), fidx(1, m, p, k)] = 0.5 * wmu[m] * t2[m]
    Cm = np.zeros((nsig, nsig))
    for k in range(ns):
        for p in range(nnu):
            for q in range(nnu):
                Cm[sidx(k, p, 0), sidx(k, q, 0)] = xi * R[p, q] * wnu[q] / phi[p]
                Cm[sidx(k, p, 1), sidx(k, q, 1)] = xi * W2 * R[p, q] * wnu[q] / phi[p]
    return np.eye(nsig) - Cm @ Jm @ Lam @ T
