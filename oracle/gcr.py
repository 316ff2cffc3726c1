"""Restarted right-preconditioned GCR with classical Gram-Schmidt (inner solver).

Section 3.2 names GCR (generalized conjugate residual) as the linear solver,
stops it when ||f - M u_k||_2 / ||f||_2 < tol (1e-10 in the paper) or after a
maximum number of iterations (10000), and Section 4 / Algorithm 2 caps the
iteration count at It_max-linear.  The paper does not spell out the GCR
variant; the reading used here (and by the GPU path):

* right preconditioning with an operator z = P^{-1} r, so the recursively
  updated residual is the true residual f - M x;
* each step: z = P^{-1} r, p = z, q = M z; the coefficients
  beta_i = <q_i, q> / <q_i, q_i> are all taken from the un-updated q (classical
  Gram-Schmidt) against the stored directions of the current cycle; then
  q <- q - sum beta_i q_i, p <- p - sum beta_i p_i,
  alpha = <q, r> / <q, q>, x <- x + alpha p, r <- r - alpha q;
* <a, b> = a^H b (conjugate-linear in the first argument);
* after ``restart`` stored directions the cycle restarts with x kept.

Pins: the iterate of step k minimises ||f - M x|| over x_0 + P^{-1} K_k
(brute force least squares over an explicit Krylov basis); without restart it
reaches the exact solution in at most n steps; a converged solve equals the LU
solution; and Proposition 4.1 (the Cayley system with zero start and the
shift-invert system with start v/(theta - sigma) produce iterates related by
y_k = (u_k - v)/(sigma - theta)).
"""

from __future__ import annotations

import numpy as np


def gcr(matvec, f, x0=None, precond=None, restart: int = 30, tol: float = 1e-10,
        maxit: int = 10000, record: bool = False):
    """Solve M x = f.  Returns (x, iterations, history).

    ``history`` is a list of the iterates after each step when ``record`` is
    set (used by the pins), else empty.  The convergence test is made before
    each step, so a start that already satisfies it takes 0 steps.
    """
    f = np.asarray(f, dtype=np.complex128)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.complex128)
    r = f - matvec(x) if x0 is not None else f.copy()
    fn = np.linalg.norm(f)
    hist = []
    P, Q, QQ = [], [], []
    its = 0
    while its < maxit:
        if fn == 0.0 or np.linalg.norm(r) <= tol * fn:
            break
        z = r.copy() if precond is None else precond(r)
        p = z
        q = matvec(z)
        beta = [np.vdot(qi, q) / qqi for qi, qqi in zip(Q, QQ)]
        for bi, pi, qi in zip(beta, P, Q):
            q = q - bi * qi
            p = p - bi * pi
        qq = np.vdot(q, q).real
        if qq == 0.0:
            break
        alpha = np.vdot(q, r) / qq
        x = x + alpha * p
        r = r - alpha * q
        its += 1
        if record:
            hist.append(x.copy())
        P.append(p)
        Q.append(q)
        QQ.append(qq)
        if len(P) == restart:
            P, Q, QQ = [], [], []
    return x, its, hist


def jacobi(A, B, sigma):
    """Point-Jacobi preconditioner z = r / diag(A - sigma B)."""
    d = A.diagonal().astype(np.complex128) - sigma * B.diagonal().astype(np.complex128)
    return lambda r: r / d


def shifted_solve_gcr(A, B, sigma, F, X0=None, restart=30, tol=1e-10, maxit=10000,
                      precond="jacobi"):
    """Column-by-column GCR solves of (A - sigma B) Y = F.  Returns (Y, iterations)."""
    M = (A.astype(np.complex128) - sigma * B.astype(np.complex128)).tocsr()
    pc = jacobi(A, B, sigma) if precond == "jacobi" else None
    F = np.asarray(F)
    Y = np.zeros(F.shape, dtype=np.complex128)
    its = np.zeros(F.shape[1], dtype=np.int64)
    for c in range(F.shape[1]):
        x0 = None if X0 is None else X0[:, c]
        Y[:, c], its[c], _ = gcr(lambda v: M @ v, F[:, c], x0, pc, restart, tol, maxit)
    return Y, its
