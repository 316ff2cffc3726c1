"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test ties an oracle function to something other than itself: closed-form
Q1 eigenvalues, dense LAPACK brute force, the minimal-residual property of GCR
checked by explicit least squares, Proposition 4.1, conjugate-pole symmetry,
Euler homogeneity of the eigenvalue gradient and finite differences.
"""

import itertools

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
import slrf_inputs as si


def closed_form_1d(m):
    """Eigenvalues of the 1D Q1 pencil ((1/h)tridiag(-1,2,-1), (h/6)tridiag(1,4,1))."""
    h = 1.0 / (m + 1)
    t = np.arange(1, m + 1) * np.pi / (m + 1)
    return (6.0 / h ** 2) * (1 - np.cos(t)) / (2 + np.cos(t))


def sine_vector(m, ks):
    """Tensor product of sin(i k pi/(m+1)), first coordinate slowest."""
    v = np.ones(1)
    for k in ks:
        v = np.kron(v, np.sin(np.arange(1, m + 1) * k * np.pi / (m + 1)))
    return v


def phi_closed(t, poles, weights):
    # Eq. (3) with conjugate halving: sum_j 2 Re(w_j / (t - sigma_j))
    return sum(2 * np.real(w / (t - s)) for s, w in zip(poles, weights))


# ----------------------------------------------------------------------------
# Filter (Eq. (2)-(3), Algorithm 1 sum-reduce)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("dim,m", [(2, 20), (3, 9)])
def test_filter_on_sine_eigenvectors(dim, m):
    p = si.q1_kron_pencil(m, dim)
    A, B = p.A(), p.B()
    lam1 = closed_form_1d(m)
    gamma = 2.5 * dim * lam1[0]
    poles, weights = si.slrf_poles(gamma)
    ks = [(1,) * dim, (2,) + (1,) * (dim - 1), (3, 2) + (1,) * (dim - 2), (m,) * dim]
    X = np.stack([sine_vector(m, k) for k in ks], axis=1)
    lam = np.array([sum(lam1[np.array(k) - 1]) for k in ks])
    U = oracle.filter.apply_filter(A, B, poles, weights, X)
    expect = X * phi_closed(lam, poles, weights)[None, :]
    assert np.max(np.abs(U - expect)) <= 1e-10 * np.max(np.abs(X))


def test_filter_function_matches_one_by_one_pencils():
    poles, weights = si.slrf_poles(3.0)
    t = np.array([0.1, 0.7, 2.9, 3.1, 8.0, 100.0])
    A = sp.diags(t).tocsr()
    B = sp.identity(t.size, format="csr")
    U = oracle.filter.apply_filter(A, B, poles, weights, np.eye(t.size))
    assert np.allclose(np.diag(U), oracle.filter.filter_function(t, poles, weights), rtol=1e-12,
                       atol=1e-12)


def test_conjugate_halving_equals_full_sum():
    p = si.q1_kron_pencil(8, 2)
    A, B = p.A(), p.B()
    poles, weights = si.slrf_poles(300.0)
    X = si.start_block(p.n, 5, 7)
    U = oracle.filter.apply_filter(A, B, poles, weights, X)
    Ufull = oracle.filter.apply_filter_full(A, B, poles, weights, X)
    scale = np.max(np.abs(U))
    assert np.max(np.abs(Ufull.imag)) <= 1e-11 * scale
    assert np.max(np.abs(Ufull.real - U)) <= 1e-11 * scale


def test_filter_equals_eigendecomposition_form():
    p = si.q1_diffusion_pencil(4, 3, kappa=np.exp(np.random.default_rng(3).normal(0, 0.5, 125)))
    A, B = p.A(), p.B()
    lam, Xe = sla.eigh(A.toarray(), B.toarray())
    poles, weights = si.slrf_poles(lam[6] * 1.01)
    X = si.start_block(p.n, 4, 9)
    U = oracle.filter.apply_filter(A, B, poles, weights, X)
    expect = Xe @ (phi_closed(lam, poles, weights)[:, None] * (Xe.T @ (B @ X)))
    assert np.max(np.abs(U - expect)) <= 1e-10 * np.max(np.abs(expect))


# ----------------------------------------------------------------------------
# GCR (Section 3.2 inner solver)
# ----------------------------------------------------------------------------

def _small_system(n=40, seed=0):
    p = si.q1_diffusion_pencil(int(round(n ** 0.5)), 2,
                               kappa=np.exp(np.random.default_rng(seed).normal(0, .5, (int(round(n ** 0.5)) + 1) ** 2)))
    A, B = p.A(), p.B()
    sigma = 40.0 * (1 + 1j)
    M = (A - sigma * B).astype(np.complex128).tocsr()
    f = (B @ si.start_block(p.n, 1, seed + 1)[:, 0]).astype(np.complex128)
    return A, B, sigma, M, f


def test_gcr_iterates_minimise_residual_over_krylov_space():
    A, B, sigma, M, f = _small_system(36, 1)
    pc = oracle.gcr.jacobi(A, B, sigma)
    x0 = 0.1 * np.ones(f.shape, dtype=np.complex128)
    _, _, hist = oracle.gcr.gcr(lambda v: M @ v, f, x0, pc, restart=50, tol=0, maxit=7,
                                record=True)
    Md = M.toarray()
    r0 = f - Md @ x0
    dinv = np.diag(pc(np.ones(f.shape, dtype=np.complex128)))
    op = Md @ dinv  # M P^{-1}
    for k in range(1, 8):
        # Krylov basis of (M P^{-1}) from r0, orthonormalised for conditioning
        K = np.empty((f.size, k), dtype=np.complex128)
        v = r0 / np.linalg.norm(r0)
        for i in range(k):
            K[:, i] = v
            v = op @ v
            v -= K[:, :i + 1] @ (K[:, :i + 1].conj().T @ v)
            v /= np.linalg.norm(v)
        y, *_ = np.linalg.lstsq(op @ K, r0, rcond=None)
        xk = x0 + dinv @ (K @ y)
        assert np.linalg.norm(hist[k - 1] - xk) <= 1e-9 * np.linalg.norm(xk)


def test_gcr_restart_semantics():
    A, B, sigma, M, f = _small_system(36, 2)
    pc = oracle.gcr.jacobi(A, B, sigma)
    _, _, hist = oracle.gcr.gcr(lambda v: M @ v, f, None, pc, restart=3, tol=0, maxit=5,
                                record=True)
    # after a restart at step 3 the method is GCR started from x_3
    _, _, h2 = oracle.gcr.gcr(lambda v: M @ v, f, hist[2], pc, restart=3, tol=0, maxit=2,
                              record=True)
    assert np.linalg.norm(hist[4] - h2[1]) <= 1e-12 * np.linalg.norm(hist[4])


def test_gcr_finite_termination_and_lu_agreement():
    A, B, sigma, M, f = _small_system(25, 3)
    n = f.size
    x, its, _ = oracle.gcr.gcr(lambda v: M @ v, f, None, oracle.gcr.jacobi(A, B, sigma),
                               restart=n + 1, tol=0, maxit=n)
    xs = np.linalg.solve(M.toarray(), f)
    assert its == n
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    y, its2 = oracle.gcr.shifted_solve_gcr(A, B, sigma, f[:, None].real, tol=1e-12, restart=10)
    ylu = oracle.filter.shifted_solve_exact(A, B, sigma, f[:, None].real)
    assert np.linalg.norm(y - ylu) <= 1e-9 * np.linalg.norm(ylu)


def test_proposition_4_1_cayley_equals_warm_started_shift_invert():
    A, B, sigma, M, _ = _small_system(49, 4)
    v = si.start_block(A.shape[0], 1, 11)[:, 0]
    theta = 55.0
    pc = oracle.gcr.jacobi(A, B, sigma)
    Cayley_rhs = (A @ v - theta * (B @ v)).astype(np.complex128)
    SI_rhs = (B @ v).astype(np.complex128)
    y0 = v.astype(np.complex128) / (theta - sigma)
    # (i) initial residuals: r_SI = r_C / (sigma - theta)
    r_si = SI_rhs - M @ y0
    assert np.linalg.norm(r_si - Cayley_rhs / (sigma - theta)) <= 1e-13 * np.linalg.norm(r_si)
    # (ii) same Krylov spaces, hence iterates y_k = (u_k - v)/(sigma - theta)
    _, _, hu = oracle.gcr.gcr(lambda z: M @ z, Cayley_rhs, None, pc, restart=30, tol=0, maxit=8,
                              record=True)
    _, _, hy = oracle.gcr.gcr(lambda z: M @ z, SI_rhs, y0, pc, restart=30, tol=0, maxit=8,
                              record=True)
    for uk, yk in zip(hu, hy):
        assert np.linalg.norm(yk - (uk - v) / (sigma - theta)) <= 1e-10 * np.linalg.norm(yk)


# ----------------------------------------------------------------------------
# Rayleigh-Ritz, Algorithms 1 and 2
# ----------------------------------------------------------------------------

def test_rayleigh_ritz_on_invariant_subspace():
    m = 12
    p = si.q1_kron_pencil(m, 2)
    A, B = p.A(), p.B()
    lam1 = closed_form_1d(m)
    ks = [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1)]
    Xe = np.stack([sine_vector(m, k) for k in ks], axis=1)
    lam = np.array([lam1[a - 1] + lam1[b - 1] for a, b in ks])
    G = np.random.default_rng(0).standard_normal((5, 5))
    theta, V = oracle.eig.rayleigh_ritz(A, B, Xe @ G)
    assert np.allclose(theta, np.sort(lam), rtol=1e-12)
    res = oracle.eig.residual_norms(A, B, theta, V)
    assert res.max() < 1e-11
    assert np.allclose(V.T @ (B @ V), np.eye(5), atol=1e-12)


def test_alg1_config_q1_2d_closed_form():
    c = si.config_q1_2d()
    p = c["pencil"]
    poles, weights = si.slrf_poles(c["gamma"], c["npoles"])
    V1 = si.start_block(p.n, c["L"], c["seed"])
    r = oracle.eig.solve_alg1(p.A(), p.B(), c["gamma"], c["nev"], V1, poles, weights)
    lam1 = closed_form_1d(40)
    ex = np.sort((lam1[:, None] + lam1[None, :]).ravel())[:c["nev"]]
    assert r["theta"].shape == (20,)
    assert np.max(np.abs(r["theta"] - ex) / ex) < 1e-10
    assert r["resid"].max() < 1e-8


def test_alg2_truncated_inner_solves_closed_form():
    m = 16
    p = si.q1_kron_pencil(m, 2)
    lam1 = closed_form_1d(m)
    ex = np.sort((lam1[:, None] + lam1[None, :]).ravel())
    nev = 8
    gamma = 0.5 * (ex[nev - 1] + ex[nev])
    poles, weights = si.slrf_poles(gamma)
    V1 = si.start_block(p.n, 12, 5)
    r = oracle.eig.solve_alg2(p.A(), p.B(), gamma, nev, V1, poles, weights,
                              inner=dict(restart=30, tol=1e-10, maxit=13))
    assert np.max(np.abs(r["theta"] - ex[:nev]) / ex[:nev]) < 1e-10


@pytest.mark.parametrize("kind", ["q1_3d", "elasticity"])
def test_alg1_brute_force_dense(kind):
    if kind == "q1_3d":
        p = si.q1_diffusion_pencil(6, 3, kappa=np.exp(np.random.default_rng(1).normal(0, .5, 343)))
    else:
        p = si.hex_elasticity_pencil(2, np.exp(np.random.default_rng(2).normal(0, .5, 8)))
    A, B = p.A(), p.B()
    lam, _ = oracle.eig.dense_eigs(A, B)
    nev = 10
    gamma = 0.5 * (lam[nev - 1] + lam[nev])
    poles, weights = si.slrf_poles(gamma)
    V1 = si.start_block(p.n, 16, 3)
    r = oracle.eig.solve_alg1(A, B, gamma, nev, V1, poles, weights)
    assert np.max(np.abs(r["theta"] - lam[:nev]) / lam[:nev]) < 1e-10


# ----------------------------------------------------------------------------
# Eigenvalue gradient
# ----------------------------------------------------------------------------

def _tiny_elastic(seed=0, ne=2):
    E = np.exp(np.random.default_rng(seed).normal(0, .3, ne ** 3))
    return si.hex_elasticity_pencil(ne, E), E


def test_gradient_euler_homogeneity_and_fd():
    p, E = _tiny_elastic(0)
    lam, X = oracle.eig.dense_eigs(p.A(), p.B())
    k = 5
    glam = np.zeros(k)
    glam[2] = 1.0
    g = oracle.grad.eig_grad(p.elem_dofs, p.ke_ref, None, X[:, :k], lam[:k], glam)
    assert np.isclose(np.sum(E * g), lam[2], rtol=1e-10)
    # central finite differences on every element (relative step 1e-6)
    gl_all = np.ones(k)
    gsum = oracle.grad.eig_grad(p.elem_dofs, p.ke_ref, None, X[:, :k], lam[:k], gl_all)
    for e in range(E.size):
        d = 1e-6 * E[e]
        Ep, Em = E.copy(), E.copy()
        Ep[e] += d
        Em[e] -= d
        lp = sla.eigh(si.hex_elasticity_pencil(2, Ep).A().toarray(), p.B().toarray(), eigvals_only=True)
        lm = sla.eigh(si.hex_elasticity_pencil(2, Em).A().toarray(), p.B().toarray(), eigvals_only=True)
        fd = (lp[:k].sum() - lm[:k].sum()) / (2 * d)
        assert np.isclose(gsum[e], fd, rtol=1e-5)


def test_gradient_density_homogeneity():
    # B = sum_e rho_e M_e with A fixed: sum_e rho_e dlambda/drho_e = -lambda
    p, _ = _tiny_elastic(1)
    lam, X = oracle.eig.dense_eigs(p.A(), p.B())
    glam = np.array([0.0, 1.0, 0.0])
    g = oracle.grad.eig_grad(p.elem_dofs, np.zeros_like(p.ke_ref), p.me_ref, X[:, :3], lam[:3], glam)
    assert np.isclose(np.sum(g), -lam[1], rtol=1e-10)


def test_sine_vector_helper_is_eigenvector():
    m = 7
    p = si.q1_kron_pencil(m, 3)
    lam1 = closed_form_1d(m)
    for ks in itertools.islice(itertools.product(range(1, m + 1), repeat=3), 0, 343, 37):
        v = sine_vector(m, ks)
        lam = sum(lam1[np.array(ks) - 1])
        assert np.linalg.norm(p.A() @ v - lam * (p.B() @ v)) <= 1e-11 * lam * np.linalg.norm(p.B() @ v)


def test_smallest_eigs_closed_form_and_dense():
    # eigsh path (n > 400) against the closed-form 2D Q1 spectrum
    m = 40
    lam1 = closed_form_1d(m)
    lam2 = np.sort((lam1[:, None] + lam1[None, :]).ravel())
    p = si.q1_kron_pencil(m, 2)
    got = oracle.eig.smallest_eigs(p.A(), p.B(), 25)
    assert np.allclose(got, lam2[:25], rtol=1e-10, atol=0)
    # eigsh path against dense LAPACK on a variable-coefficient 3D pencil (n = 729)
    kappa = np.exp(np.random.default_rng(5).normal(0, 0.5, 10 ** 3))
    q = si.q1_diffusion_pencil(9, 3, kappa)
    dense = oracle.eig.dense_eigs(q.A(), q.B())[0]
    assert np.allclose(oracle.eig.smallest_eigs(q.A(), q.B(), 30), dense[:30], rtol=1e-10)


# ----------------------------------------------------------------------------
# Residual of Section 3.2 and the Jacobi preconditioner, on hand-worked cases
# ----------------------------------------------------------------------------

def test_residual_norm_normaliser_hand_worked():
    """r = (A - theta B) x / (theta ||x||_B) (Section 3.2) for a non-eigenvector.

    A = diag(2, 5), B = diag(1, 2), x = (1, 1), theta = 3 by hand:
    (A - 3B) x = (-1, -1), ||.||_2 = sqrt(2); ||x||_B = sqrt(1 + 2) = sqrt(3);
    so ||r|| = sqrt(2) / (3 sqrt(3)) = 0.272165526975909.  Dropping theta gives
    0.8165, the Euclidean norm of x instead of the B-norm 0.3333: both fail.
    """
    A = sp.diags([2.0, 5.0]).tocsr()
    B = sp.diags([1.0, 2.0]).tocsr()
    x = np.array([[1.0], [1.0]])
    r = oracle.eig.residual_norms(A, B, np.array([3.0]), x)
    assert abs(r[0] - 0.272165526975909) <= 1e-15
    # theta < 0 and a second column: A = [[4, 1], [1, 3]], B = I, x = (1, 0),
    # theta = -2: (A + 2I) x = (6, 1), norm sqrt(37); |theta| ||x||_B = 2
    A2 = sp.csr_matrix(np.array([[4.0, 1.0], [1.0, 3.0]]))
    X2 = np.array([[1.0, 1.0], [0.0, 1.0]])
    r2 = oracle.eig.residual_norms(A2, sp.identity(2, format="csr"), np.array([-2.0, 1.0]), X2)
    # column 2: theta = 1, (A - I)(1, 1) = (4, 3), norm 5; ||x||_B = sqrt(2)
    assert abs(r2[0] - np.sqrt(37.0) / 2.0) <= 1e-14
    assert abs(r2[1] - 5.0 / np.sqrt(2.0)) <= 1e-14


def test_jacobi_uses_the_shifted_diagonal_hand_worked():
    """z = r / diag(A - sigma B): A = [[2, 1], [1, 4]], B = I, sigma = 1 + i.

    diag(A - sigma B) = (1 - i, 3 - i); r = (1, 1) gives by hand
    z = (1 / (1 - i), 1 / (3 - i)) = (0.5 + 0.5i, 0.3 + 0.1i); the off-diagonal
    entries of A take no part.
    """
    A = sp.csr_matrix(np.array([[2.0, 1.0], [1.0, 4.0]]))
    pc = oracle.gcr.jacobi(A, sp.identity(2, format="csr"), 1.0 + 1.0j)
    z = pc(np.array([1.0 + 0j, 1.0 + 0j]))
    assert np.allclose(z, [0.5 + 0.5j, 0.3 + 0.1j], rtol=0, atol=1e-15)
    # B enters through its diagonal: B = diag(2, 0.5), sigma = 2i:
    # diag = (2 - 4i, 4 - i); r = (2 - 4i, 0) -> z = (1, 0)
    pc2 = oracle.gcr.jacobi(A, sp.diags([2.0, 0.5]).tocsr(), 2.0j)
    z2 = pc2(np.array([2.0 - 4.0j, 0.0]))
    assert np.allclose(z2, [1.0, 0.0], rtol=0, atol=1e-15)


def test_jacobi_gcr_solves_a_diagonal_pencil_in_one_step():
    """With a diagonal pencil the Jacobi-preconditioned operator is the identity,
    so right-preconditioned GCR reaches the exact solution y_i = f_i /
    (a_i - sigma b_i) in exactly one step (any other diagonal would need more)."""
    a = np.array([1.0, 3.0, 7.0, 20.0])
    b = np.array([0.5, 1.0, 2.0, 1.5])
    sigma = 2.0 + 1.5j
    A, B = sp.diags(a).tocsr(), sp.diags(b).tocsr()
    f = np.array([1.0, -2.0, 0.5, 4.0]).reshape(-1, 1)
    Y, its = oracle.gcr.shifted_solve_gcr(A, B, sigma, f, restart=30, tol=1e-14)
    assert its[0] == 1
    assert np.allclose(Y[:, 0], f[:, 0] / (a - sigma * b), rtol=1e-14, atol=0)


def test_smallest_eigpairs_against_closed_form_and_definition():
    """Eigenpairs of the 3D Q1 pencil (m = 9, n = 729 > 400: the Lanczos path):
    eigenvalues equal the closed form, the vectors are B-orthonormal and each
    satisfies A x = lambda B x (Eq. (1)) to rounding."""
    p = si.q1_kron_pencil(9, 3)
    A, B = p.A(), p.B()
    lam, X = oracle.eig.smallest_eigpairs(A, B, 12)
    l1 = closed_form_1d(9)
    ex = np.sort((l1[:, None, None] + l1[None, :, None] + l1[None, None, :]).ravel())[:12]
    assert np.max(np.abs(lam - ex) / ex) <= 1e-11
    assert np.max(np.abs(X.T @ (B @ X) - np.eye(12))) <= 1e-11
    R = A @ X - (B @ X) * lam[None, :]
    assert np.max(np.linalg.norm(R, axis=0) / lam) <= 1e-8
