"""Eigenvalue sensitivities with respect to per-element parameters.

For a simple eigenpair (lambda, x) of A(theta) x = lambda B(theta) x with
x^T B x = 1, d lambda / d theta_e = x^T (dA/dtheta_e - lambda dB/dtheta_e) x
(differentiating the Rayleigh quotient).  With A = sum_e theta_e K_e and
B independent of theta (Young's modulus), dA/dtheta_e = K_e (the element
stiffness for unit modulus) and dB/dtheta_e = 0; with a density
parameterisation dB/dtheta_e = M_e.  For a loss L(lambda) with gradient
g_i = dL/dlambda_i the chain rule gives
dL/dtheta_e = sum_i g_i x_{i,e}^T (K_e - lambda_i M_e) x_{i,e},
x_{i,e} being the element's dofs of x_i (constrained dofs contribute zero).

Pins: Euler homogeneity (A linear in theta, B fixed: sum_e theta_e dlambda/dtheta_e
= lambda exactly), and central finite differences of dense eigenvalues.
"""

from __future__ import annotations

import numpy as np


def eig_grad(elem_dofs, dK, dM, X, lam, glam):
    """Per-element dL/dtheta_e by an explicit loop over elements.

    elem_dofs: [nelem, ndof_e] int, -1 for constrained dofs.
    dK, dM: [ndof_e, ndof_e] element derivative matrices (dM may be None).
    X: [n, k] B-normalised eigenvectors; lam, glam: [k].
    """
    X = np.asarray(X, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    glam = np.asarray(glam, dtype=np.float64)
    nelem = elem_dofs.shape[0]
    g = np.zeros(nelem)
    for e in range(nelem):
        d = elem_dofs[e]
        ok = d >= 0
        xe = np.zeros((d.shape[0], X.shape[1]))
        xe[ok] = X[d[ok]]
        kq = np.einsum("ai,ab,bi->i", xe, dK, xe)
        mq = np.einsum("ai,ab,bi->i", xe, dM, xe) if dM is not None else 0.0
        g[e] = np.sum(glam * (kq - lam * mq))
    return g
