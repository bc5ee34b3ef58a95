"""Seeded synthetic inputs shaped like the paper's 1D benchmark problem.

This module builds *inputs only*: depth grids, angular and spectral
quadrature nodes and weights, the absorption profile and opacity ratios,
thermalization parameters and random test vectors.  It holds none of the
solver's arithmetic (no formal solver, no scattering step, no Krylov
method), so both the GPU path and the CPU oracle can be fed from it.

Problem statement followed (Sect. 3.1-3.2 and 4.1 of the paper):
  * depth grid: log-spaced optical depths, top first (Sect. 4.1);
  * directions: Gauss-Legendre nodes on mu in [-1, 1] (Sect. 4.1);
  * frequencies: equispaced reduced frequencies x with trapezoidal weights
    (Sect. 4.1);
  * absorption profile: Voigt profile with damping a (eqs. J00/J02);
  * thermalization eps, Planck function B (Wien limit W = 1), bottom
    boundary intensity (Sect. 3.1).

Two readings of the optical-depth scale are offered (the paper's grid is in
frequency-integrated optical depth, Sect. 4.1; the benchmark configurations
here quote line-centre optical depth):
  * ``"line_center"``  r_p = H(a, x_p) / H(a, 0);
  * ``"integrated"``   r_p = H(a, x_p) / sqrt(pi)  (= phi_p).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
from scipy.special import wofz

SEED_BASE = 211011873

FS_DELO_LINEAR = 0
FS_TRAPEZOIDAL = 1
FS_IMPLICIT_EULER = 2
FS_DELO_PARABOLIC = 3
_FS_NAMES = {"delo_linear": FS_DELO_LINEAR, "trapezoidal": FS_TRAPEZOIDAL,
             "implicit_euler": FS_IMPLICIT_EULER, "delo_parabolic": FS_DELO_PARABOLIC}


@dataclasses.dataclass
class Problem:
    """A batch of independent 1D slabs sharing the angular/spectral grids.

    Array layouts (all float64 unless noted, C-contiguous):
      ns        int32 [n_atm]       depth points per slab
      tau       [sum(ns)]           optical depths, top first, increasing
      mu, w_mu  [n_mu]              direction cosines on [-1,1] and weights
      x, w_nu   [n_nu]              reduced frequencies and weights
      phi       [n_atm, n_nu]       absorption profile at x (unnormalized)
      opac      [n_atm, n_nu]       opacity ratio r_p (optical-depth scale)
      eps, W2, I_bot  [n_atm]       thermalization, polarizability, bottom
                                    boundary intensity for mu > 0
      B         [sum(ns)]           Planck function (Wien limit)
    """

    ns: np.ndarray
    tau: np.ndarray
    mu: np.ndarray
    w_mu: np.ndarray
    x: np.ndarray
    w_nu: np.ndarray
    phi: np.ndarray
    opac: np.ndarray
    eps: np.ndarray
    W2: np.ndarray
    I_bot: np.ndarray
    B: np.ndarray
    formal_solver: int = FS_DELO_LINEAR
    normalize_profile: bool = True
    name: str = "custom"

    @property
    def n_atm(self) -> int:
        return int(self.ns.shape[0])

    @property
    def n_mu(self) -> int:
        return int(self.mu.shape[0])

    @property
    def n_nu(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_unknowns(self) -> int:
        return 2 * int(self.ns.sum())

    @property
    def offsets(self) -> np.ndarray:
        """Start of each slab in the depth-indexed arrays (tau, B)."""
        off = np.zeros(self.n_atm + 1, dtype=np.int64)
        off[1:] = np.cumsum(self.ns)
        return off

    @property
    def n_intervals(self) -> int:
        """Sum over slabs of (ns-1) * (n_mu/2) * n_nu."""
        return int(((self.ns.astype(np.int64) - 1) * (self.n_mu // 2) * self.n_nu).sum())

    def slab(self, i: int) -> "Problem":
        """The i-th slab as a one-slab problem (views copied)."""
        off = self.offsets
        s = slice(off[i], off[i + 1])
        return Problem(
            ns=self.ns[i:i + 1].copy(), tau=self.tau[s].copy(), mu=self.mu, w_mu=self.w_mu,
            x=self.x, w_nu=self.w_nu, phi=self.phi[i:i + 1].copy(), opac=self.opac[i:i + 1].copy(),
            eps=self.eps[i:i + 1].copy(), W2=self.W2[i:i + 1].copy(),
            I_bot=self.I_bot[i:i + 1].copy(), B=self.B[s].copy(),
            formal_solver=self.formal_solver, normalize_profile=self.normalize_profile,
            name=f"{self.name}[{i}]")

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------------------
# grids and profiles (inputs)
# ----------------------------------------------------------------------------

def voigt_H(a: float, x: np.ndarray) -> np.ndarray:
    """Voigt function H(a, x) = Re w(x + i a), w the Faddeeva function."""
    return np.real(wofz(np.asarray(x, dtype=np.float64) + 1j * a))


def gauss_legendre(n: int):
    mu, w = np.polynomial.legendre.leggauss(n)
    return mu.astype(np.float64), w.astype(np.float64)


def trapezoid_grid(n: int, xmax: float):
    x = np.linspace(-xmax, xmax, n)
    h = x[1] - x[0]
    w = np.full(n, h)
    w[0] = w[-1] = 0.5 * h
    return x, w


def log_tau(ns: int, tmin: float, tmax: float) -> np.ndarray:
    return np.logspace(math.log10(tmin), math.log10(tmax), ns)


def _profiles(a_list, x, scale: str):
    phi = np.empty((len(a_list), x.shape[0]))
    opac = np.empty_like(phi)
    for i, a in enumerate(a_list):
        H = voigt_H(a, x)
        phi[i] = H / math.sqrt(math.pi)
        if scale == "line_center":
            opac[i] = H / voigt_H(a, np.array([0.0]))[0]
        elif scale == "integrated":
            opac[i] = H / math.sqrt(math.pi)
        else:
            raise ValueError(scale)
    return phi, opac


def make_slabs(ns_list, tau_ranges, n_mu, n_nu, xmax, a_list, eps_list, W2_list,
               formal_solver="delo_linear", scale="line_center", normalize=True,
               B=1.0, I_bot=None, name="custom") -> Problem:
    mu, w_mu = gauss_legendre(n_mu)
    x, w_nu = trapezoid_grid(n_nu, xmax)
    phi, opac = _profiles(a_list, x, scale)
    ns = np.asarray(ns_list, dtype=np.int32)
    tau = np.concatenate([log_tau(int(n), lo, hi) for n, (lo, hi) in zip(ns, tau_ranges)])
    Bv = np.full(tau.shape[0], float(B))
    if I_bot is None:
        I_bot = np.full(ns.shape[0], float(B))
    fs = _FS_NAMES[formal_solver] if isinstance(formal_solver, str) else int(formal_solver)
    return Problem(ns=ns, tau=tau, mu=mu, w_mu=w_mu, x=x, w_nu=w_nu, phi=phi, opac=opac,
                   eps=np.asarray(eps_list, dtype=np.float64),
                   W2=np.asarray(W2_list, dtype=np.float64),
                   I_bot=np.asarray(I_bot, dtype=np.float64), B=Bv,
                   formal_solver=fs, normalize_profile=bool(normalize), name=name)


# ----------------------------------------------------------------------------
# the benchmark workloads
# ----------------------------------------------------------------------------

def config1(formal_solver="delo_linear") -> Problem:
    """FP64 tiny: Ns=40, tau in [1e-2, 1e4], 8 mu, 21 nu on [-5,5], a=1e-3, eps=1e-2, W2=0.5."""
    return make_slabs([40], [(1e-2, 1e4)], 8, 21, 5.0, [1e-3], [1e-2], [0.5],
                      formal_solver=formal_solver, name="c1_tiny_ns40")


def config1_subgrid(formal_solver="delo_linear") -> Problem:
    """The 10 x 4 x 5 sub-grid of the tiny case, for dense LU checks."""
    return make_slabs([10], [(1e-2, 1e4)], 4, 5, 5.0, [1e-3], [1e-2], [0.5],
                      formal_solver=formal_solver, name="c1_sub_10x4x5")


def config2(formal_solver="delo_linear") -> Problem:
    """Paper-shaped: Ns=200, tau in [1e-4, 1e8], 20 mu, 101 nu on [-10,10], a=1e-3, eps=1e-4, W2=0.5."""
    return make_slabs([200], [(1e-4, 1e8)], 20, 101, 10.0, [1e-3], [1e-4], [0.5],
                      formal_solver=formal_solver, name=f"c2_ns200_mu20_nu101_{formal_solver}")


def config3() -> Problem:
    """Single large slab: Ns=1024, tau in [1e-4,1e8], 32 mu, 201 nu, a ~ logU[1e-4,1e-2]."""
    rng = np.random.default_rng(SEED_BASE + 3)
    a = float(10 ** rng.uniform(-4, -2))
    return make_slabs([1024], [(1e-4, 1e8)], 32, 201, 10.0, [a], [1e-4], [0.5],
                      name="c3_ns1024_mu32_nu201")


def config4(n_slabs: int = 512) -> Problem:
    """Batched uneven slabs: Ns ~ U{64..512}, tau_max ~ logU[1e4,1e8], 16 mu, 101 nu,
    eps ~ logU[1e-6,1e-2], a ~ logU[1e-4,1e-2], W2 ~ U[0,0.7]."""
    rng = np.random.default_rng(SEED_BASE + 4)
    ns = rng.integers(64, 513, size=n_slabs)
    tmax = 10 ** rng.uniform(4, 8, size=n_slabs)
    eps = 10 ** rng.uniform(-6, -2, size=n_slabs)
    a = 10 ** rng.uniform(-4, -2, size=n_slabs)
    W2 = rng.uniform(0.0, 0.7, size=n_slabs)
    return make_slabs(list(ns), [(1e-4, t) for t in tmax], 16, 101, 10.0, list(a), list(eps),
                      list(W2), name=f"c4_batched{n_slabs}")


def paper_replica(ns: int, n_mu: int = 20, n_nu: int = 20, scale: str = "integrated",
                  normalize: bool = True) -> Problem:
    """The paper's own setup (Sect. 4.1-4.2): tau in [1e-5, 1e4], x in [-5, 5],
    a = 1e-3, eps = 1e-4, W = 1, w(2) = 1."""
    return make_slabs([ns], [(1e-5, 1e4)], n_mu, n_nu, 5.0, [1e-3], [1e-4], [1.0],
                      scale=scale, normalize=normalize, name=f"paper_ns{ns}_{n_mu}x{n_nu}")


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded U[-1, 1] test vector."""
    return np.random.default_rng(SEED_BASE + 1000 + seed).uniform(-1.0, 1.0, n)


def initial_guess(p: Problem) -> np.ndarray:
    """x0 = [1, 0, 1, 0, ...] (Sect. 4.2)."""
    x0 = np.zeros(p.n_unknowns)
    x0[0::2] = 1.0
    return x0


CONFIGS = {
    "c1": config1,
    "c2": config2,
    "c3": config3,
    "c4": config4,
}


# ----------------------------------------------------------------------------
# frequency redistribution (the benchmark's fifth configuration)
# ----------------------------------------------------------------------------

def redistribution_matrix(x, w_nu, phi, gamma):
    """Synthetic redistribution kernel R(x, x') = (1 - gamma) phi(x) phi(x') +
    gamma phi(x') exp(-(x - x')^2 / 2) / sqrt(2 pi), each column scaled so that
    sum_x w_x R(x, x') = phi(x') (the discrete form of int R dx = phi(x'))."""
    x = np.asarray(x, dtype=np.float64)
    w_nu = np.asarray(w_nu, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    g = np.exp(-0.5 * (x[:, None] - x[None, :]) ** 2) / math.sqrt(2.0 * math.pi)
    R = (1.0 - gamma) * np.outer(phi, phi) + gamma * phi[None, :] * g
    col = (w_nu[:, None] * R).sum(axis=0)
    return R * (phi / col)[None, :]


def config5(gamma: float = 0.5, ns: int = 256, n_mu: int = 32, n_nu: int = 256):
    """Redistribution: Ns=256, tau in [1e-4, 1e8], 32 mu, 256 nu on [-12, 12], a=1e-3,
    eps=1e-4, W2=0.5, R with gamma = 0.5.  Returns (problem, R)."""
    p = make_slabs([ns], [(1e-4, 1e8)], n_mu, n_nu, 12.0, [1e-3], [1e-4], [0.5],
                   name=f"c5_ns{ns}_mu{n_mu}_nu{n_nu}_gamma{gamma}")
    return p, redistribution_matrix(p.x, p.w_nu, p.phi[0], gamma)
