"""Rayleigh-Ritz, convergence test, Algorithms 1 and 2, dense reference.

* Rayleigh-Ritz (Algorithm 1, projected-problem step): solve
  (U^T A U) s = theta (U^T B U) s, theta ascending, v = U s.
* Residual (Section 3.2): r_k = (A - theta_k B) x_k / (theta_k ||x_k||_B);
  a pair is converged when ||r_k||_2 < 1e-8.
* Algorithm 1: filter, Rayleigh-Ritz, convergence check, V_{k+1} = all Ritz
  vectors; no explicit orthogonalisation.
* Algorithm 2: adds It_max-linear on the inner solves, B-orthogonalisation of U
  against the locked vectors X when n_conv > 0, locking with n_act = L - n_conv,
  and the warm start Y_init = v / (theta - sigma).

Readings (the paper is silent): only pairs with theta in (0, gamma] are locked
or reported; the run stops when NEV pairs have converged; Ritz vectors are
B-normalised; the B-orthogonalisation against X is done twice (classical
Gram-Schmidt, repeated once).

Pins: closed-form Q1 eigenvalues; dense ``scipy.linalg.eigh(A, B)`` on tiny
pencils; Rayleigh-Ritz on an exact invariant subspace returns the exact
eigenvalues with zero residual.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .filter import apply_filter
from .gcr import shifted_solve_gcr


def rayleigh_ritz(A, B, U):
    """Ritz values (ascending) and B-normalised Ritz vectors of span(U)."""
    U = np.asarray(U, dtype=np.float64)
    AU = A @ U
    BU = B @ U
    Ah = U.T @ AU
    Bh = U.T @ BU
    Ah = 0.5 * (Ah + Ah.T)
    Bh = 0.5 * (Bh + Bh.T)
    try:
        theta, S = sla.eigh(Ah, Bh)
    except np.linalg.LinAlgError:
        # U^T B U not numerically definite: B-orthonormalise first, dropping
        # directions whose B-Gram eigenvalue is below 1e-14 of the largest.
        mu, W = sla.eigh(Bh)
        keep = mu > 1e-14 * mu.max()
        T = W[:, keep] / np.sqrt(mu[keep])
        theta, S2 = sla.eigh(T.T @ Ah @ T)
        S = T @ S2
    V = U @ S
    return theta, V


def residual_norms(A, B, theta, V):
    """||(A - theta B) v||_2 / (theta ||v||_B) per column (Section 3.2)."""
    V = np.asarray(V, dtype=np.float64)
    AV = A @ V
    BV = B @ V
    R = AV - BV * theta[None, :]
    vb = np.sqrt(np.maximum(np.einsum("ij,ij->j", V, BV), 0.0))
    return np.linalg.norm(R, axis=0) / (np.abs(theta) * vb)


def dense_eigs(A, B):
    """All eigenpairs by dense LAPACK (brute force for tiny pencils)."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    Bd = B.toarray() if hasattr(B, "toarray") else np.asarray(B)
    return sla.eigh(Ad, Bd)


def smallest_eigs(A, B, k):
    """The k smallest eigenvalues of the SPD pencil (A, B), ascending.

    Shift-invert Lanczos about 0 (ARPACK through ``scipy.sparse.linalg.eigsh``
    with an LU of A): a library routine standing for the plain definition of
    the eigenvalues of Eq. (1) at sizes where a dense solve does not fit.
    """
    import scipy.sparse.linalg as spla

    n = A.shape[0]
    if n <= 400:
        return dense_eigs(A, B)[0][:k]
    vals = spla.eigsh(A.tocsc(), k=k, M=B.tocsc(), sigma=0.0, which="LM", tol=1e-13,
                      return_eigenvectors=False)
    return np.sort(vals)


def smallest_eigpairs(A, B, k):
    """The k smallest eigenpairs (ascending) with B-orthonormal eigenvectors.

    Same shift-invert Lanczos about 0 as ``smallest_eigs`` (dense LAPACK for
    n <= 400), returning the eigenvectors as well; the vectors are
    B-orthonormalised once more (eigenvectors of distinct eigenvalues are
    B-orthogonal, Eq. (1); inside a cluster any B-orthonormal basis of the
    invariant subspace is valid).
    """
    import scipy.sparse.linalg as spla

    n = A.shape[0]
    if n <= 400:
        lam, X = dense_eigs(A, B)
        return lam[:k], X[:, :k]
    lam, X = spla.eigsh(A.tocsc(), k=k, M=B.tocsc(), sigma=0.0, which="LM", tol=1e-13)
    o = np.argsort(lam)
    lam, X = lam[o], X[:, o]
    G = X.T @ (B @ X)
    L = np.linalg.cholesky(0.5 * (G + G.T))
    X = np.linalg.solve(L, X.T).T
    return lam, X


def _filter(A, B, poles, weights, V, inner, theta_warm=None):
    """Filtered block with exact (inner=None) or GCR inner solves.

    With GCR and a warm start the initial guess for column c and pole j is
    v_c / (theta_c - sigma_j) (Algorithm 2, warm start).
    """
    if inner is None:
        return apply_filter(A, B, poles, weights, V), None
    its_all = []

    def solver(s, F, j):
        X0 = None
        if theta_warm is not None:
            X0 = V.astype(np.complex128) / (theta_warm[None, :] - s)
        Y, its = shifted_solve_gcr(A, B, s, F, X0=X0, **inner)
        its_all.append(its)
        return Y

    U = apply_filter(A, B, poles, weights, V, solver=solver)
    return U, np.stack(its_all)


def solve_alg1(A, B, gamma, nev, V1, poles, weights, tol_eig=1e-8, max_outer=100,
               inner=None):
    """Algorithm 1.  Returns dict(theta, X, iters, resid)."""
    V = np.array(V1, dtype=np.float64)
    hist = []
    for k in range(1, max_outer + 1):
        U, _ = _filter(A, B, poles, weights, V, inner)
        theta, Vr = rayleigh_ritz(A, B, U)
        res = residual_norms(A, B, theta, Vr)
        conv = (theta > 0) & (theta <= gamma) & (res < tol_eig)
        hist.append(int(conv.sum()))
        if conv.sum() >= nev:
            idx = np.nonzero(conv)[0][:nev]
            return dict(theta=theta[idx], X=Vr[:, idx], iters=k, resid=res[idx], history=hist)
        V = Vr
    idx = np.nonzero(conv)[0]
    return dict(theta=theta[idx], X=Vr[:, idx], iters=max_outer, resid=res[idx], history=hist,
                converged=False)


def b_orthogonalize(B, X, U, passes=2):
    """U <- U - X (X^T B U), repeated ``passes`` times (X B-orthonormal)."""
    for _ in range(passes):
        U = U - X @ (X.T @ (B @ U))
    return U


def solve_alg2(A, B, gamma, nev, V1, poles, weights, tol_eig=1e-8, max_outer=100,
               inner=None, warm_start=True):
    """Algorithm 2 (Enhanced ParaSLRF).  ``inner`` = GCR options incl. maxit = It_max."""
    n, L = V1.shape
    V = np.array(V1, dtype=np.float64)
    Theta = np.zeros(0)
    X = np.zeros((n, 0))
    theta_warm = None
    hist = []
    for k in range(1, max_outer + 1):
        U, _ = _filter(A, B, poles, weights, V, inner,
                       theta_warm if (warm_start and inner is not None) else None)
        if X.shape[1] > 0:
            U = b_orthogonalize(B, X, U)
        theta, Vr = rayleigh_ritz(A, B, U)
        res = residual_norms(A, B, theta, Vr)
        conv = (theta > 0) & (theta <= gamma) & (res < tol_eig)
        Theta = np.concatenate([Theta, theta[conv]])
        X = np.concatenate([X, Vr[:, conv]], axis=1)
        hist.append(int(conv.sum()))
        nconv = X.shape[1]
        if nconv >= nev:
            order = np.argsort(Theta)
            return dict(theta=Theta[order], X=X[:, order], iters=k, history=hist)
        nact = L - nconv
        keep = np.nonzero(~conv)[0][:nact]
        V = Vr[:, keep]
        theta_warm = theta[keep]
    order = np.argsort(Theta)
    return dict(theta=Theta[order], X=X[:, order], iters=max_outer, history=hist,
                converged=False)
