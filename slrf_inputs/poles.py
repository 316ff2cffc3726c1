"""Pole and weight tables for the rational filter of Eq. (3).

Poles and weights are *inputs* of Algorithms 1 and 2 (their REQUIRE lists
take sigma_1..sigma_N and w_1..w_N).  Only the N poles in the upper half plane
are returned; the other N are their complex conjugates with conjugate weights
(the conjugate-pole halving of Section 2).

Shifted-Laplace poles (Section 2.2): the paper places the poles on the rays
y = x(1 +/- alpha i) with alpha = 1 and a relaxation parameter beta = 0.01, and
defers the formula for the real parts and the weights to its companion paper,
which is not available here.  :func:`slrf_poles` is therefore a stated reading,
not the paper's formula:

* real parts x_j = gamma (j - 1/2) / N, j = 1..N, so sigma_j = x_j (1 + alpha i);
* weights from the linear least-squares fit (2N real unknowns) of
  Phi(t) = sum_j 2 Re(w_j / (t - sigma_j)) to the indicator of (0, gamma] at
  4000 uniform samples on (0, gamma] and 4000 log-spaced samples on
  [(1 + beta) gamma, 1000 gamma]; beta is read as the excluded transition band.

The design is scale invariant (sigma/gamma and w/gamma do not depend on
gamma), so it is computed for gamma = 1 and scaled.  Any pole/weight table gives
the same converged eigenpairs; the table only changes convergence speed.
"""

from __future__ import annotations

import numpy as np


def slrf_poles(gamma: float, npoles: int = 8, alpha: float = 1.0, beta: float = 0.01,
               nin: int = 4000, nout: int = 4000):
    """Upper-half-plane shifted-Laplace poles and least-squares weights.

    Returns (sigma, w): complex128 arrays of length ``npoles``.
    """
    if gamma <= 0:
        raise ValueError("gamma must be positive")
    N = int(npoles)
    x = (np.arange(1, N + 1) - 0.5) / N
    s = x * (1.0 + 1j * alpha)
    t_in = np.linspace(1.0 / nin, 1.0, nin)
    t_out = np.logspace(np.log10(1.0 + beta), 3.0, nout)
    t = np.concatenate([t_in, t_out])
    target = np.concatenate([np.ones(nin), np.zeros(nout)])
    # 2 Re((a + i b) / (t - s)) = 2 (a (t - x) - b y) / |t - s|^2
    d = t[:, None] - s[None, :]
    den = np.abs(d) ** 2
    cols_a = 2.0 * (t[:, None] - s.real[None, :]) / den
    cols_b = -2.0 * s.imag[None, :] / den
    G = np.concatenate([cols_a, cols_b], axis=1)
    coef, *_ = np.linalg.lstsq(G, target, rcond=None)
    w = coef[:N] + 1j * coef[N:]
    return (gamma * s).astype(np.complex128), (gamma * w).astype(np.complex128)


def quadrature_poles(gamma: float, npoles: int, rule: str = "midpoint"):
    """Contour-quadrature poles/weights on the circle through 0 and gamma.

    The circle has centre c = gamma/2 and radius r = gamma/2; with nodes
    z_k = c + r exp(i phi_k) in the upper half and quadrature weights omega_k in
    phi, the resolvent integral (1/(2 pi i)) \\oint dz / (z - t) becomes
    Phi(t) = sum_k w_k / (t - z_k) with w_k = -omega_k r exp(i phi_k) / (2 pi).
    ``rule`` is "midpoint" (equispaced phi), "gauss-legendre" (Gauss-Legendre
    nodes on each half circle) or "gauss-chebyshev" (Chebyshev nodes of the
    first kind on each half circle, weights (pi/N) sqrt(1 - x^2) so the rule
    integrates plain functions of x).  These are the comparison filters of the
    paper's Table 1; they are provided as data only.
    """
    N = int(npoles)
    c = r = 0.5 * gamma
    if rule == "midpoint":
        phi = np.pi * (2 * np.arange(1, N + 1) - 1) / (2 * N)
        omega = np.full(N, np.pi / N)
    elif rule == "gauss-legendre":
        xg, wg = np.polynomial.legendre.leggauss(N)
        phi = 0.5 * np.pi * (1.0 + xg)
        omega = 0.5 * np.pi * wg
    elif rule == "gauss-chebyshev":
        xc = np.cos(np.pi * (2 * np.arange(1, N + 1) - 1) / (2 * N))
        phi = 0.5 * np.pi * (1.0 + xc)
        omega = 0.5 * np.pi * (np.pi / N) * np.sqrt(1.0 - xc ** 2)
    else:
        raise ValueError(f"unknown rule {rule!r}")
    z = c + r * np.exp(1j * phi)
    w = -omega * r * np.exp(1j * phi) / (2 * np.pi)
    order = np.argsort(z.real)
    return z[order].astype(np.complex128), w[order].astype(np.complex128)
