"""Input generators: FEM pencils, element matrices, poles, start blocks (CPU)."""

import numpy as np
import pytest
import scipy.linalg as sla

import slrf_inputs as si


def _check_pattern(p):
    n = p.n
    assert p.indptr.dtype == np.int32 and p.indices.dtype == np.int32
    assert p.indptr[0] == 0 and p.indptr[-1] == p.nnz
    for r in range(0, n, max(1, n // 50)):
        c = p.indices[p.indptr[r]:p.indptr[r + 1]]
        assert np.all(np.diff(c) > 0)
    A, B = p.A(), p.B()
    assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
    assert abs(B - B.T).max() <= 1e-12 * abs(B).max()


@pytest.mark.parametrize("dim,m", [(2, 7), (3, 5)])
def test_diffusion_unit_coefficient_equals_kronecker(dim, m):
    pk = si.q1_kron_pencil(m, dim)
    pd = si.q1_diffusion_pencil(m, dim)
    assert np.array_equal(pk.indptr, pd.indptr) and np.array_equal(pk.indices, pd.indices)
    assert np.max(np.abs(pk.a - pd.a)) <= 1e-13 * np.max(np.abs(pk.a))
    assert np.max(np.abs(pk.b - pd.b)) <= 1e-13 * np.max(np.abs(pk.b))
    _check_pattern(pk)
    _check_pattern(pd)


def test_kron_matches_scipy_kron():
    m = 6
    h = 1.0 / (m + 1)
    e = np.ones(m)
    import scipy.sparse as sp
    K = sp.diags([-e[1:], 2 * e, -e[1:]], [-1, 0, 1]) / h
    M = sp.diags([e[1:], 4 * e, e[1:]], [-1, 0, 1]) * (h / 6)
    A = sp.kron(K, sp.kron(M, M)) + sp.kron(M, sp.kron(K, M)) + sp.kron(M, sp.kron(M, K))
    B = sp.kron(M, sp.kron(M, M))
    p = si.q1_kron_pencil(m, 3)
    assert abs(p.A() - A).max() < 1e-14
    assert abs(p.B() - B).max() < 1e-14
    assert p.nnz == (3 * m - 2) ** 3


def test_hex_element_invariants():
    h = 0.25
    ke, me = si.hex_element_matrices(h, 0.3, rho=2.0)
    # rigid-body modes: 3 translations + 3 rotations span the null space
    w = np.linalg.eigvalsh(ke)
    assert np.sum(np.abs(w) < 1e-10 * w.max()) == 6
    assert np.all(w > -1e-10 * w.max())
    # consistent mass: total mass rho*h^3 per displacement component
    for c in range(3):
        assert np.isclose(me[c::3, c::3].sum(), 2.0 * h ** 3, rtol=1e-13)
        for d in range(3):
            if d != c:
                assert np.all(me[c::3, d::3] == 0)
    # a linear displacement field u = (x, 0, 0) has strain energy E*vol/... > 0
    # and a rotation field has zero energy
    local = np.array([[a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1)], float) * h
    rot = np.zeros(24)
    rot[0::3] = -local[:, 1]
    rot[1::3] = local[:, 0]
    assert abs(rot @ ke @ rot) < 1e-12 * np.abs(ke).max()


def test_hex_pencil_unclamped_rigid_body_and_size():
    ne = 2
    p = si.hex_elasticity_pencil(ne, np.ones(ne ** 3), clamp=False)
    w = sla.eigvalsh(p.A().toarray())
    assert np.sum(np.abs(w) < 1e-9 * w.max()) == 6
    pc = si.hex_elasticity_pencil(3, np.ones(27), clamp=True)
    assert pc.n == 3 * 3 * 4 * 4
    _check_pattern(pc)
    assert np.all(np.linalg.eigvalsh(pc.A().toarray()) > 0)


def test_pole_design_properties():
    s1, w1 = si.slrf_poles(1.0)
    s2, w2 = si.slrf_poles(250.0)
    assert np.allclose(s2, 250.0 * s1, rtol=1e-14)
    assert np.allclose(w2, 250.0 * w1, rtol=1e-9)
    assert np.all(s1.imag > 0) and np.allclose(s1.imag, s1.real)
    t_in = np.linspace(0.02, 1.0, 50)
    t_out = np.logspace(np.log10(1.05), 3, 50)
    phi = lambda t: np.sum(2 * np.real(w1[None] / (t[:, None] - s1[None])), axis=1)  # noqa: E731
    assert np.all(phi(t_in) > 0.7)
    assert np.all(np.abs(phi(t_out)) < 0.7)
    assert np.abs(phi(np.array([20.0]))) < 0.1


def test_start_block_seeded():
    a = si.start_block(100, 7, 5)
    b = si.start_block(100, 7, 5)
    assert a.flags.f_contiguous and a.shape == (100, 7)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, si.start_block(100, 7, 6))


def test_config_gammas():
    c1 = si.config_q1_2d()
    assert c1["nev"] == 20 and abs(c1["gamma"] - 328.6492) < 1e-3
    g, nev = si.q1_gamma_nev(64, 3, 100)
    assert nev == 102 and abs(g - 421.0642) < 1e-3


def test_quadrature_filters_midpoint_closed_form_and_shape():
    gamma = 10.0
    t = np.array([0.3, 2.0, 5.0, 9.0, 11.0, 20.0, 100.0])
    z, w = si.quadrature_poles(gamma, 8, "midpoint")
    phi = np.array([np.sum(2 * np.real(w / (x - z))) for x in t])
    s = (t - gamma / 2) / (gamma / 2)
    # equispaced midpoint nodes on the circle: Phi = 1 / (1 + s^(2N)) exactly
    assert np.allclose(phi, 1.0 / (1.0 + s ** 16), rtol=1e-12, atol=1e-14)
    for rule in ("gauss-legendre", "gauss-chebyshev"):
        z, w = si.quadrature_poles(gamma, 8, rule)
        assert np.all(z.imag > 0) and np.allclose(np.abs(z - gamma / 2), gamma / 2)
        phi = np.array([np.sum(2 * np.real(w / (x - z))) for x in (2.0, 5.0, 8.0, 30.0, 200.0)])
        assert np.all(np.abs(phi[:3] - 1) < 0.02) and np.all(np.abs(phi[3:]) < 0.01)
