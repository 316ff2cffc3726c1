"""Rational filter: Phi of Eq. (3), the shifted systems of Eq. (2), the filtered block.

Section 2: the filter is Phi(t) = sum_{j=1}^{2N} w_j / (t - sigma_j) with the
second half of the poles and weights the complex conjugates of the first half,
so for real t and a real block X it reduces to N complex solves,
U = sum_{j=1}^{N} 2 Re(w_j (A - sigma_j B)^{-1} B X)  (the sum-reduce step of
Algorithms 1 and 2).

Pins: (i) for a B-orthonormal eigenvector u with A u = lambda B u the filter is
exactly U = Phi(lambda) u (closed form for tensor-product Q1 pencils); (ii) the
halved sum equals the full sum over all 2N conjugate poles; (iii) on tiny
pencils U equals X_e Phi(Lambda) X_e^T B X from a dense eigendecomposition.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def filter_function(t, poles, weights):
    """Phi(t) = sum_j 2 Re(w_j / (t - sigma_j)) over the upper-half-plane poles (Eq. (3))."""
    t = np.asarray(t, dtype=np.float64)
    poles = np.asarray(poles, dtype=np.complex128)
    weights = np.asarray(weights, dtype=np.complex128)
    return np.sum(2.0 * np.real(weights[None, :] / (t.reshape(-1, 1) - poles[None, :])),
                  axis=1).reshape(t.shape)


def shifted_matrix(A, B, sigma) -> sp.csc_matrix:
    """A - sigma B in complex128 (the operator of Eq. (2))."""
    return (A.astype(np.complex128) - sigma * B.astype(np.complex128)).tocsc()


def shifted_solve_exact(A, B, sigma, F):
    """Y = (A - sigma B)^{-1} F by sparse LU (SuperLU, MMD on A^T + A)."""
    lu = spla.splu(shifted_matrix(A, B, sigma), permc_spec="MMD_AT_PLUS_A")
    F = np.asarray(F)
    return lu.solve(F.astype(np.complex128))


def apply_filter(A, B, poles, weights, X, solver=None):
    """U = sum_j 2 Re(w_j (A - sigma_j B)^{-1} B X) (Algorithm 1, sum-reduce step).

    ``solver(sigma, F, j)`` returns the complex solution block; default exact LU.
    Poles are accumulated in increasing j.
    """
    X = np.asarray(X, dtype=np.float64)
    F = B @ X
    U = np.zeros_like(X, dtype=np.float64)
    for j, (s, w) in enumerate(zip(poles, weights)):
        Y = shifted_solve_exact(A, B, s, F) if solver is None else solver(s, F, j)
        U += 2.0 * np.real(w * Y)
    return U


def apply_filter_full(A, B, poles, weights, X):
    """sum over all 2N poles, sigma_j and conj(sigma_j) with w_j and conj(w_j), no halving."""
    X = np.asarray(X, dtype=np.float64)
    F = (B @ X).astype(np.complex128)
    U = np.zeros(X.shape, dtype=np.complex128)
    for s, w in zip(poles, weights):
        U += w * shifted_solve_exact(A, B, s, F)
        U += np.conj(w) * shifted_solve_exact(A, B, np.conj(s), F)
    return U
