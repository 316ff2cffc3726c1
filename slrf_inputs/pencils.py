"""Sparse FEM pencils (A = stiffness, B = mass) in CSR form.

Every generator returns a :class:`Pencil` whose A and B share one sparsity
pattern (identical ``indptr``/``indices``; entries that vanish in one matrix are
stored as explicit zeros), column indices sorted within each row, FP64 values
and int32 indices.  A shared pattern lets a single pass over the column indices
serve both matrices in the shifted operator A - sigma B of Eq. (2).

Generators:

* :func:`q1_kron_pencil` - tensor-product Q1 Laplace pencil on the unit square
  or cube with homogeneous Dirichlet conditions,
  A = K(x)M + M(x)K (2D) or K(x)M(x)M + M(x)K(x)M + M(x)M(x)K (3D), B = M(x)M(x)...,
  with 1D K = (1/h) tridiag(-1, 2, -1), M = (h/6) tridiag(1, 4, 1), h = 1/(m+1).
* :func:`q1_diffusion_pencil` - the same element family assembled element by
  element with a per-element coefficient kappa_e (consistent mass).
* :func:`hex_elasticity_pencil` - isotropic linear elasticity on a uniform
  trilinear hex mesh of the unit cube, clamped on the x = 0 face, 3 dofs/node,
  consistent mass, 2x2x2 Gauss quadrature (exact for both matrices on a cube).
"""

from __future__ import annotations

import dataclasses
import itertools
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Pencil:
    """A symmetric-definite pencil (A, B) on a shared CSR pattern."""

    indptr: np.ndarray  # int32 [n+1]
    indices: np.ndarray  # int32 [nnz], sorted per row
    a: np.ndarray  # float64 [nnz]
    b: np.ndarray  # float64 [nnz]
    name: str = ""
    # Optional element data (for the eigenvalue-gradient path):
    elem_dofs: Optional[np.ndarray] = None  # int32 [nelem, ndof_e]; -1 = constrained dof
    elem_param: Optional[np.ndarray] = None  # float64 [nelem]: the parameter theta_e
    ke_ref: Optional[np.ndarray] = None  # float64 [ndof_e, ndof_e]: dA/dtheta_e
    me_ref: Optional[np.ndarray] = None  # float64 [ndof_e, ndof_e]: element mass
    # Optional node coordinates (vector-valued pencils, node-major dofs):
    coords: Optional[np.ndarray] = None  # float64 [n_nodes, dofs per node]

    @property
    def n(self) -> int:
        return int(self.indptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    def A(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.a, self.indices, self.indptr), shape=(self.n, self.n))

    def B(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.b, self.indices, self.indptr), shape=(self.n, self.n))


def _assemble_shared(rows, cols, avals, bvals, n) -> tuple:
    """Sum duplicate (row, col) contributions for A and B onto one pattern.

    Explicit zeros are kept so that A and B share the pattern exactly.
    Returns (indptr, indices, a, b) with indices sorted inside each row.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = rows * n + cols
    uniq, inv = np.unique(key, return_inverse=True)
    a = np.bincount(inv, weights=avals, minlength=uniq.shape[0])
    b = np.bincount(inv, weights=bvals, minlength=uniq.shape[0])
    urow = uniq // n
    ucol = uniq % n
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, urow + 1, 1)
    indptr = np.cumsum(indptr)
    return (indptr.astype(np.int32), ucol.astype(np.int32), a.astype(np.float64),
            b.astype(np.float64))


# ---------------------------------------------------------------------------
# Tensor-product Q1 Laplace pencil (Kronecker form)
# ---------------------------------------------------------------------------

def q1_kron_pencil(m: int, dim: int) -> Pencil:
    """Q1 Laplace pencil on the unit square (dim=2) or cube (dim=3).

    m interior nodes per direction, h = 1/(m+1), lexicographic ordering with
    the first coordinate slowest (the ordering of numpy/scipy ``kron``).
    The pattern is the full 9-point (2D) or 27-point (3D) stencil of B; A is
    evaluated entry by entry on it (in 3D the face-neighbour entries of A are
    K M M + M K M + M M K = 0 up to rounding and are kept as stored entries).
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    h = 1.0 / (m + 1)
    k1 = {0: 2.0 / h, 1: -1.0 / h}
    m1 = {0: 4.0 * h / 6.0, 1: h / 6.0}
    n = m ** dim
    # Build the stencil pattern row by row, vectorised over all rows.
    coords = np.indices((m,) * dim).reshape(dim, -1).T  # [n, dim], row-major = kron order
    rows_l, cols_l, offs_l = [], [], []
    for off in itertools.product((-1, 0, 1), repeat=dim):
        nb = coords + np.asarray(off)
        ok = np.all((nb >= 0) & (nb < m), axis=1)
        r = np.nonzero(ok)[0]
        c = np.ravel_multi_index(nb[ok].T, (m,) * dim)
        rows_l.append(r)
        cols_l.append(c)
        offs_l.append(np.broadcast_to(np.abs(np.asarray(off)), (r.shape[0], dim)))
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l)
    offs = np.concatenate(offs_l)
    kk = np.where(offs == 0, k1[0], k1[1])  # [nnz, dim]
    mm = np.where(offs == 0, m1[0], m1[1])
    bvals = np.prod(mm, axis=1)
    avals = np.zeros_like(bvals)
    for d in range(dim):
        term = kk[:, d].copy()
        for e in range(dim):
            if e != d:
                term = term * mm[:, e]
        avals = avals + term
    indptr, indices, a, b = _assemble_shared(rows, cols, avals, bvals, n)
    return Pencil(indptr, indices, a, b, name=f"q1_kron_{dim}d_m{m}")


# ---------------------------------------------------------------------------
# Element-by-element Q1 diffusion pencil
# ---------------------------------------------------------------------------

def _q1_element_1d(h: float):
    k = (1.0 / h) * np.array([[1.0, -1.0], [-1.0, 1.0]])
    mm = (h / 6.0) * np.array([[2.0, 1.0], [1.0, 2.0]])
    return k, mm


def q1_element_matrices(h: float, dim: int):
    """Exact Q1 (bi/trilinear) element stiffness and mass on a cube of side h.

    Local node numbering is lexicographic over (0/1)^dim with the first
    coordinate slowest, matching ``np.kron`` of the 1D element matrices.
    """
    k, mm = _q1_element_1d(h)
    if dim == 2:
        ke = np.kron(k, mm) + np.kron(mm, k)
        me = np.kron(mm, mm)
    else:
        ke = (np.kron(k, np.kron(mm, mm)) + np.kron(mm, np.kron(k, mm))
              + np.kron(mm, np.kron(mm, k)))
        me = np.kron(mm, np.kron(mm, mm))
    return ke, me


def q1_diffusion_pencil(m: int, dim: int, kappa: Optional[np.ndarray] = None) -> Pencil:
    """Q1 diffusion pencil on the unit square/cube, Dirichlet on the boundary.

    (m+1)^dim elements, m^dim interior (free) nodes with the same ordering as
    :func:`q1_kron_pencil`; ``kappa`` holds one coefficient per element
    (lexicographic element order), default all ones (then A, B equal the
    Kronecker pencil up to rounding).
    """
    ne = m + 1
    h = 1.0 / ne
    nelem = ne ** dim
    if kappa is None:
        kappa = np.ones(nelem)
    kappa = np.asarray(kappa, dtype=np.float64)
    if kappa.shape != (nelem,):
        raise ValueError("kappa must have one entry per element")
    ke, me = q1_element_matrices(h, dim)
    ecoords = np.indices((ne,) * dim).reshape(dim, -1).T  # element lower corners
    local = np.array(list(itertools.product((0, 1), repeat=dim)))  # [2^dim, dim]
    gnode = ecoords[:, None, :] + local[None, :, :]  # grid node coords 0..m+1
    interior = np.all((gnode >= 1) & (gnode <= m), axis=2)
    dof = np.where(interior,
                   np.ravel_multi_index(np.clip(gnode - 1, 0, m - 1).transpose(2, 0, 1), (m,) * dim),
                   -1).astype(np.int64)  # [nelem, 2^dim]
    nl = local.shape[0]
    ri = np.repeat(dof, nl, axis=1)  # [nelem, nl*nl]
    ci = np.tile(dof, (1, nl))
    ok = (ri >= 0) & (ci >= 0)
    av = kappa[:, None] * ke.reshape(1, -1)
    bv = np.broadcast_to(me.reshape(1, -1), av.shape)
    indptr, indices, a, b = _assemble_shared(ri[ok], ci[ok], av[ok], bv[ok], m ** dim)
    p = Pencil(indptr, indices, a, b, name=f"q1_diff_{dim}d_m{m}")
    p.elem_dofs = dof.astype(np.int32)
    p.elem_param = kappa.copy()
    p.ke_ref = ke
    p.me_ref = me
    return p


# ---------------------------------------------------------------------------
# Trilinear hex linear elasticity
# ---------------------------------------------------------------------------

def hex_element_matrices(h: float, nu: float, rho: float = 1.0):
    """Stiffness (for Young's modulus 1) and consistent mass of a cube element.

    Trilinear shape functions on [0,h]^3, 8 nodes in lexicographic order over
    (0/1)^3 (x slowest), 24 dofs ordered node-major (3*node + component).
    Isotropic material, 2x2x2 Gauss quadrature.
    """
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    local = np.array(list(itertools.product((0, 1), repeat=3)), dtype=np.float64)
    g = 0.5 / np.sqrt(3.0)
    gp = [0.5 - g, 0.5 + g]
    ke = np.zeros((24, 24))
    me = np.zeros((24, 24))
    wq = (h ** 3) / 8.0
    for xi in itertools.product(gp, repeat=3):
        xi = np.asarray(xi)
        # shape functions on the unit cube and their gradients (physical: /h)
        N = np.prod(np.where(local == 1, xi, 1 - xi), axis=1)  # [8]
        dN = np.zeros((8, 3))
        for d in range(3):
            fac = np.where(local[:, d] == 1, 1.0, -1.0)
            other = np.prod(np.where(local == 1, xi, 1 - xi)[:, [e for e in range(3) if e != d]], axis=1)
            dN[:, d] = fac * other / h
        Bm = np.zeros((6, 24))
        for a in range(8):
            bx, by, bz = dN[a]
            Bm[0, 3 * a] = bx
            Bm[1, 3 * a + 1] = by
            Bm[2, 3 * a + 2] = bz
            Bm[3, 3 * a] = by
            Bm[3, 3 * a + 1] = bx
            Bm[4, 3 * a + 1] = bz
            Bm[4, 3 * a + 2] = by
            Bm[5, 3 * a] = bz
            Bm[5, 3 * a + 2] = bx
        ke += wq * Bm.T @ D @ Bm
        Nm = np.zeros((3, 24))
        for a in range(8):
            Nm[0, 3 * a] = Nm[1, 3 * a + 1] = Nm[2, 3 * a + 2] = N[a]
        me += wq * rho * Nm.T @ Nm
    return 0.5 * (ke + ke.T), 0.5 * (me + me.T)


def hex_elasticity_pencil(ne: int, young: np.ndarray, nu: float = 0.3, rho: float = 1.0,
                          clamp: bool = True) -> Pencil:
    """Linear elasticity pencil on a uniform ne^3 hex mesh of the unit cube.

    ``young`` holds one Young's modulus per element (lexicographic element
    order, x slowest).  With ``clamp`` the nodes on the x = 0 face are fixed.
    Free nodes are ordered lexicographically (x slowest) and dofs node-major,
    so n = 3 * ne * (ne+1)^2 when clamped.
    """
    h = 1.0 / ne
    nelem = ne ** 3
    young = np.asarray(young, dtype=np.float64)
    if young.shape != (nelem,):
        raise ValueError("young must have one entry per element")
    ke, me = hex_element_matrices(h, nu, rho)
    nn = ne + 1
    gx = np.arange(nn)
    free = np.ones((nn, nn, nn), dtype=bool)
    if clamp:
        free[0, :, :] = False
    node_id = -np.ones((nn, nn, nn), dtype=np.int64)
    node_id[free] = np.arange(int(free.sum()))
    ecoords = np.indices((ne,) * 3).reshape(3, -1).T
    local = np.array(list(itertools.product((0, 1), repeat=3)))
    gnode = ecoords[:, None, :] + local[None, :, :]  # [nelem, 8, 3]
    nid = node_id[gnode[..., 0], gnode[..., 1], gnode[..., 2]]  # [nelem, 8]
    dof = np.where(nid[..., None] >= 0, 3 * nid[..., None] + np.arange(3), -1).reshape(nelem, 24)
    del gx
    nfree = int(free.sum()) * 3
    ri = np.repeat(dof, 24, axis=1)
    ci = np.tile(dof, (1, 24))
    ok = (ri >= 0) & (ci >= 0)
    av = young[:, None] * ke.reshape(1, -1)
    # The mass couples only equal components; it is stored on the stiffness
    # pattern (explicit zeros) so that A and B share one pattern.
    bv = np.broadcast_to(me.reshape(1, -1), av.shape)
    indptr, indices, a, b = _assemble_shared(ri[ok], ci[ok], av[ok], bv[ok], nfree)
    p = Pencil(indptr, indices, a, b, name=f"hex_elast_{ne}")
    p.coords = np.indices((nn,) * 3).reshape(3, -1).T[free.reshape(-1)] * h
    p.elem_dofs = dof.astype(np.int32)
    p.elem_param = young.copy()
    p.ke_ref = ke
    p.me_ref = me
    return p
