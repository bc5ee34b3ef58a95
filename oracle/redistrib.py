"""Oracle of the frequency-redistribution variant (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU leg may import
this module.  The unknown is sigma^K(k, p) per depth k and frequency p
(K = 0, 2), laid out per slab as index (k * n_nu + p) * 2 + K.  The operator
is the CRD one (A = Id - J Lambda T) with the frequency quadrature of J
replaced by the redistribution:

  S_I(k, m, p) = s0(k, p) + T1(mu_m) s2(k, p),   S_Q(k, m, p) = T2(mu_m) s2(k, p);
  I, Q = the formal solution along ray (m, p) with zero incoming radiation;
  J0_p(k) = sum_m (w_m / 2) I(k, m, p),  J2_p(k) = sum_m (w_m / 2) (T1 I + T2 Q)
      (the monochromatic angle quadrature of eqs. J00/J02);
  Jt^K(k, p) = sum_p' R(p, p') w_p' J^K_p'(k)       (the redistribution);
  (A sigma)^K(k, p) = sigma^K(k, p) - xi W_K Jt^K(k, p) / phi_p,  W_0 = 1, W_2 = W2.

With R(p, p') proportional to phi_p phi_p' (gamma = 0) this is the complete
redistribution operator of the CRD problem, replicated over frequency.
The right-hand side is the same contraction of the transmitted field plus
[eps B, 0].
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def _t20(mu):
    return np.sqrt(2.0) * (3.0 * mu * mu - 1.0) / 4.0, np.sqrt(2.0) * (3.0 * mu * mu - 3.0) / 4.0


def _mono_J(prob, i, s0, s2, with_inflow):
    """Monochromatic J0, J2 [ns, nnu] of the field with sources s0, s2 [ns, nnu]."""
    off = prob.offsets
    tau = np.ascontiguousarray(prob.tau[off[i]:off[i + 1]])
    ns, nnu = tau.shape[0], len(prob.w_nu)
    J0 = np.zeros((ns, nnu))
    J2 = np.zeros((ns, nnu))
    for m, mu in enumerate(prob.mu):
        t1, t2 = _t20(mu)
        up = mu > 0
        for p in range(nnu):
            kappa = prob.opac[i][p] / abs(mu)
            inflow = float(prob.I_bot[i]) if (with_inflow and up) else 0.0
            I = O.ray(tau, kappa, up, s0[:, p] + t1 * s2[:, p], I_entry=inflow,
                      fs=int(prob.formal_solver))
            Q = O.ray(tau, kappa, up, t2 * s2[:, p], I_entry=0.0, fs=int(prob.formal_solver))
            J0[:, p] += 0.5 * prob.w_mu[m] * I
            J2[:, p] += 0.5 * prob.w_mu[m] * (t1 * I + t2 * Q)
    return J0, J2


def _contract(prob, i, R, J):
    """Jt(k, p) = sum_p' R(p, p') w_p' J(k, p')."""
    return J @ (R * np.asarray(prob.w_nu)[None, :]).T


def apply(prob, R, sigma, i=0):
    """A sigma for slab i (sigma laid out (k * n_nu + p) * 2 + K)."""
    ns, nnu = int(prob.ns[i]), len(prob.w_nu)
    sg = np.asarray(sigma, dtype=np.float64).reshape(ns, nnu, 2)
    J0, J2 = _mono_J(prob, i, sg[:, :, 0], sg[:, :, 1], False)
    xi, W2 = 1.0 - float(prob.eps[i]), float(prob.W2[i])
    phi = np.asarray(prob.phi[i])
    out = np.empty_like(sg)
    out[:, :, 0] = sg[:, :, 0] - xi * _contract(prob, i, R, J0) / phi[None, :]
    out[:, :, 1] = sg[:, :, 1] - xi * W2 * _contract(prob, i, R, J2) / phi[None, :]
    return out.ravel()


def rhs(prob, R, i=0):
    """b = xi W_K (contraction of the transmitted field's J) / phi + [eps B, 0]."""
    ns, nnu = int(prob.ns[i]), len(prob.w_nu)
    z = np.zeros((ns, nnu))
    J0, J2 = _mono_J(prob, i, z, z, True)
    xi, W2 = 1.0 - float(prob.eps[i]), float(prob.W2[i])
    phi = np.asarray(prob.phi[i])
    off = prob.offsets
    B = np.asarray(prob.B[off[i]:off[i + 1]])
    out = np.empty((ns, nnu, 2))
    out[:, :, 0] = xi * _contract(prob, i, R, J0) / phi[None, :] + float(prob.eps[i]) * B[:, None]
    out[:, :, 1] = xi * W2 * _contract(prob, i, R, J2) / phi[None, :]
    return out.ravel()
