"""The synthetic workloads: pencil, interval (0, gamma], NEV, L and seeds.

* Q1 2D, m = 40 (n = 1600): gamma encloses the 20 smallest eigenvalues,
  L = 32, seed 1001, 8 upper-half-plane poles.
* Q1 3D, m = 64 (n = 262,144, 27-point stencils): gamma in the first gap at or
  after the 100th eigenvalue (the 97th..102nd eigenvalues form a 6-fold cluster,
  so NEV = 102), L = 160, seed 1002, 8 poles.
* Batched: 64 Q1 diffusion pencils with lognormal(0, 0.5) element
  coefficients, n in [5000, 60000], drawn from seed 1004.

For tensor-product Q1 pencils the eigenvalues are known in closed form:
lambda = sum_d lambda_1D(k_d), lambda_1D(k) = (6/h^2)(1 - cos t_k)/(2 + cos t_k),
t_k = k pi/(m+1); gamma is placed in the middle of the spectral gap.
"""

from __future__ import annotations

import itertools

import numpy as np

from .pencils import q1_kron_pencil, q1_diffusion_pencil, hex_elasticity_pencil
from .blocks import seeded_rng


def q1_eigenvalues_1d(m: int) -> np.ndarray:
    h = 1.0 / (m + 1)
    t = np.arange(1, m + 1) * np.pi / (m + 1)
    return (6.0 / h ** 2) * (1.0 - np.cos(t)) / (2.0 + np.cos(t))


def _q1_smallest(m: int, dim: int, count: int) -> np.ndarray:
    lam1 = q1_eigenvalues_1d(m)
    k = min(m, count + 2)
    vals = [sum(c) for c in itertools.product(lam1[:k], repeat=dim)]
    return np.sort(np.asarray(vals))


def q1_gamma_nev(m: int, dim: int, count: int, rel_gap: float = 1e-6):
    """(gamma, nev): the first spectral gap at or after ``count`` eigenvalues.

    Eigenvalues that agree to ``rel_gap`` relative are one cluster; gamma is the
    midpoint between the last eigenvalue of the cluster holding the count-th
    eigenvalue and the next distinct one.
    """
    lam = _q1_smallest(m, dim, count + 64)
    c = count
    while lam[c] - lam[c - 1] <= rel_gap * lam[c]:
        c += 1
    return 0.5 * (lam[c - 1] + lam[c]), c


def config_q1_2d():
    p = q1_kron_pencil(40, 2)
    gamma, nev = q1_gamma_nev(40, 2, 20)
    return dict(pencil=p, gamma=gamma, nev=nev, L=32, seed=1001, npoles=8,
                name="q1_2d_m40")


def config_q1_3d(m: int = 64, L: int = 160, count: int = 100):
    p = q1_kron_pencil(m, 3)
    gamma, nev = q1_gamma_nev(m, 3, count)
    return dict(pencil=p, gamma=gamma, nev=nev, L=L, seed=1002, npoles=8,
                name=f"q1_3d_m{m}")


def batched_pencils(count: int = 64, seed: int = 1004, nmin: int = 5000, nmax: int = 60000,
                    only=None):
    """Draw the uneven batch: per pencil (dim, m, kappa, target eigenvalue count c).

    The interval (0, gamma] for each pencil needs its eigenvalues and is chosen
    by the caller; this returns the pencils and the drawn counts only.  `only`
    (an iterable of indices) assembles just those pencils (the draws of the
    others are still made, so every pencil is the same in any selection).
    """
    rng = seeded_rng(seed)
    keep = None if only is None else set(int(i) for i in only)
    out = []
    for i in range(count):
        dim = 2 if rng.random() < 0.5 else 3
        nt = rng.uniform(nmin, nmax)
        m = int(round(nt ** (1.0 / dim)))
        kappa = np.exp(rng.normal(0.0, 0.5, size=(m + 1) ** dim))
        c = int(rng.integers(10, 61))
        if keep is not None and i not in keep:
            continue
        out.append(dict(pencil=q1_diffusion_pencil(m, dim, kappa), count=c, dim=dim, m=m,
                        L=int(np.ceil(1.5 * c)), seed=seed * 1000 + i, index=i))
    return out


def config_elasticity(ne: int = 32, sigma: float = 0.3, seed: int = 1005, count: int = 50,
                      L: int = 75):
    """Clamped trilinear-hex elasticity on ne^3 elements, Young's modulus per
    element lognormal(0, sigma) from ``seed`` (nu = 0.3, rho = 1).

    ne = 32, sigma = 0.3, seed 1005, 50 eigenvalues, L = 75: the
    differentiation workload (n = 104,544); ne = 48, sigma = 0.5, seed 1003,
    200 eigenvalues, L = 300: the large elasticity workload (n = 345,744).
    The interval end gamma needs the eigenvalues and comes from the caller.
    """
    rng = seeded_rng(seed)
    young = np.exp(rng.normal(0.0, sigma, ne ** 3))
    p = hex_elasticity_pencil(ne, young)
    return dict(pencil=p, young=young, count=count, L=L, seed=seed + 100, npoles=8,
                name=f"elasticity_{ne}")
