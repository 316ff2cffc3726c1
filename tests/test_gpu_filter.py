"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances:
* shifted SpMM: elementwise |q - q_ref| <= 32 eps (|A| + |sigma||B|) |z|
  (a sum of <= 27 products per entry, eps of the sweep precision);
* converged solves: every system's FP64 relative residual <= tol (verified on
  the CPU with scipy from the returned solution), and the filtered block within
  sum_j 2|w_j| ||(A - sigma_j B)^{-1}|| tol ||f|| of the exact-LU oracle, with
  ||(A - sigma B)^{-1}||_2 <= 1 / (lambda_min(B) Im sigma) for SPD A, B;
* truncated GCR iterates (It_max-linear): equal to the oracle's GCR iterates up
  to rounding (1e-10 relative in FP64).
"""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2510_17334_amd as P
import slrf_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(x).T), device="cuda").t()


def _host(t):
    return t.detach().cpu().numpy()


def _handle(p, gamma, poles, weights, **opt):
    return P.Handle.from_pencil(p, gamma, poles, weights, P.default_options(**opt))


def _q1_lambda_min_B(m, dim):
    h = 1.0 / (m + 1)
    return ((h / 6.0) * (4.0 + 2.0 * np.cos(m * np.pi / (m + 1)))) ** dim


def _filter_bound(F, poles, weights, tol, lmin_b):
    fn = np.linalg.norm(F, axis=0)
    amp = np.sum(2 * np.abs(weights) / np.imag(poles))
    return 1.01 * tol * fn * amp / lmin_b


@pytest.fixture(scope="module")
def cfg1():
    c = si.config_q1_2d()
    poles, weights = si.slrf_poles(c["gamma"], c["npoles"])
    c["poles"], c["weights"] = poles, weights
    c["V1"] = si.start_block(c["pencil"].n, c["L"], c["seed"])
    return c


# ----------------------------------------------------------------------------
# shifted SpMM (a3)
# ----------------------------------------------------------------------------
SPMM_VARIANTS = [0, 1, 2, 3, 4, 5, 6, 7]  # auto, row-group, CSR-LDS u8, direct, u16, u32, halo,
# wave-uniform row groups


@pytest.mark.parametrize("variant", SPMM_VARIANTS)
@pytest.mark.parametrize("prec", [P.SLRF_PREC_FP64, P.SLRF_PREC_MIXED])
@pytest.mark.parametrize("which", ["q1_2d_m40", "diff_3d_m12"])
def test_shifted_spmm_parity(prec, which, variant):
    if which == "q1_2d_m40":
        p = si.q1_kron_pencil(40, 2)
    else:  # n = 2197: a ragged last slice of 5 rows
        p = si.q1_diffusion_pencil(12, 3, np.exp(np.random.default_rng(2).normal(0, .5, 13 ** 3)))
    poles, weights = si.slrf_poles(300.0)
    h = _handle(p, 300.0, poles, weights, spmm_variant=variant)
    nsys = 37
    rng = np.random.default_rng(7)
    Zh = rng.standard_normal((p.n, nsys)) + 1j * rng.standard_normal((p.n, nsys))
    pidx = np.arange(nsys) % len(poles)
    dt = torch.complex128 if prec == P.SLRF_PREC_FP64 else torch.complex64
    Zt = P.slrf.to_panels(torch.as_tensor(Zh, device="cuda").to(dt), p.n)
    Q = P.slrf.from_panels(h.slrf_shifted_spmm(Zt, pidx, prec), p.n, nsys)
    Qh = _host(Q).astype(np.complex128)
    Zr = _host(P.slrf.from_panels(Zt, p.n, nsys)).astype(np.complex128)  # rounded input
    order = h.slrf_get_row_order()  # panel vectors use the library's row order
    assert np.array_equal(np.sort(order), np.arange(p.n))
    A, B = p.A()[order][:, order], p.B()[order][:, order]
    absA, absB = abs(A), abs(B)
    eps = np.finfo(np.float64 if prec == P.SLRF_PREC_FP64 else np.float32).eps
    for s in range(nsys):
        sg = poles[pidx[s]]
        ref = A @ Zr[:, s] - sg * (B @ Zr[:, s])
        scale = absA @ np.abs(Zr[:, s]) + abs(sg) * (absB @ np.abs(Zr[:, s]))
        assert np.all(np.abs(Qh[:, s] - ref) <= 32 * eps * scale + 1e-300), s
    h.close()


@pytest.mark.parametrize("prec", [P.SLRF_PREC_FP64, P.SLRF_PREC_MIXED])
def test_shifted_spmm_full_size_sampled(prec):
    """The benchmark's sweep (n = 262,144, 1280 systems, 8 poles, the autotuned
    kernel) on sampled rows and systems against the row-by-row product."""
    c = si.config_q1_3d()
    p = c["pencil"]
    poles, weights = si.slrf_poles(c["gamma"], 8)
    h = _handle(p, c["gamma"], poles, weights)
    nsys = 1280
    pidx = np.arange(nsys) % 8
    dt = torch.complex128 if prec == P.SLRF_PREC_FP64 else torch.complex64
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    Zt = torch.randn((nsys // 16, p.n, 16), dtype=dt, device="cuda", generator=g)
    Q = h.slrf_shifted_spmm(Zt, pidx, prec)
    order = h.slrf_get_row_order()
    inv = np.empty_like(order)
    inv[order] = np.arange(p.n)
    rng = np.random.default_rng(12)
    rows = np.concatenate([[0, 1, p.n - 1], rng.choice(p.n, 997, replace=False)])
    systems = np.concatenate([[0, 15, 16, nsys - 1], rng.choice(nsys, 28, replace=False)])
    A, B = p.A().tocsr(), p.B().tocsr()
    eps = np.finfo(np.float64 if prec == P.SLRF_PREC_FP64 else np.float32).eps
    sys_t = torch.as_tensor(systems, device="cuda")
    Zs = _host(Zt[sys_t // 16, :, sys_t % 16]).astype(np.complex128)  # [systems, n]
    Qs = _host(Q[sys_t // 16, :, sys_t % 16]).astype(np.complex128)
    sg = poles[pidx[systems]]
    for i in rows:
        lo, hi = A.indptr[order[i]], A.indptr[order[i] + 1]
        cols = inv[A.indices[lo:hi]]
        a, b = A.data[lo:hi], B.data[lo:hi]
        z = Zs[:, cols]
        q = Qs[:, i]
        ref = z @ a - sg * (z @ b)
        scale = np.abs(z) @ np.abs(a) + np.abs(sg) * (np.abs(z) @ np.abs(b))
        assert np.all(np.abs(q - ref) <= 32 * eps * scale + 1e-300), i
    h.close()


@pytest.mark.parametrize("prec", [P.SLRF_PREC_FP64, P.SLRF_PREC_MIXED])
def test_shifted_spmm_full_size_sine_closed_form(prec):
    """Closed form at full size (n = 262,144): for a sine product u,
    (A - sigma B) u = (lambda_u - sigma) mu_u u with mu_u the B eigenvalue."""
    m = 64
    c = si.config_q1_3d()
    p = c["pencil"]
    poles, weights = si.slrf_poles(c["gamma"], 8)
    h = _handle(p, c["gamma"], poles, weights)
    h1d = 1.0 / (m + 1)
    t = np.arange(1, m + 1) * np.pi / (m + 1)
    lam1 = (6.0 / h1d ** 2) * (1 - np.cos(t)) / (2 + np.cos(t))
    mu1 = (h1d / 6.0) * (4 + 2 * np.cos(t))
    ks = [(1, 1, 1), (2, 1, 3), (5, 4, 1), (64, 64, 64), (33, 7, 50), (1, 64, 2)]
    # sin(j k pi / (m + 1)) with the argument reduced exactly (integer j k mod
    # 2 (m + 1)): high modes are then eigenvectors to rounding
    sv = lambda k: np.sin(((np.arange(1, m + 1) * k) % (2 * (m + 1))) * np.pi / (m + 1))
    U = np.stack([np.kron(sv(a), np.kron(sv(b), sv(cc))) for a, b, cc in ks], axis=1)
    lam = np.array([lam1[a - 1] + lam1[b - 1] + lam1[cc - 1] for a, b, cc in ks])
    mu = np.array([mu1[a - 1] * mu1[b - 1] * mu1[cc - 1] for a, b, cc in ks])
    order = h.slrf_get_row_order()
    nv, npole = len(ks), len(poles)
    nsys = nv * npole
    pidx = np.arange(nsys) % npole
    vidx = np.arange(nsys) // npole
    Zh = U[order][:, vidx].astype(np.complex128)
    dt = torch.complex128 if prec == P.SLRF_PREC_FP64 else torch.complex64
    Zt = P.slrf.to_panels(torch.as_tensor(Zh, device="cuda").to(dt), p.n)
    Q = _host(P.slrf.from_panels(h.slrf_shifted_spmm(Zt, pidx, prec), p.n, nsys))
    sg = poles[pidx]
    ref = Zh * ((lam[vidx] - sg) * mu[vidx])[None, :]
    A, B = abs(p.A()[order][:, order]), abs(p.B()[order][:, order])
    scale = A @ np.abs(Zh) + np.abs(sg)[None, :] * (B @ np.abs(Zh))
    eps = np.finfo(np.float64 if prec == P.SLRF_PREC_FP64 else np.float32).eps
    # the input is rounded to the sweep precision first in the mixed form
    assert np.all(np.abs(Q.astype(np.complex128) - ref) <= 64 * eps * scale + 1e-300)
    h.close()


# ----------------------------------------------------------------------------
# converged filter (a1-a7): residual certification and oracle parity
# ----------------------------------------------------------------------------
def _single_pole_solution(p, gamma, sigma, X, **opt):
    """Y = (A - sigma B)^{-1} B X from two one-pole filters (w = 1/2 and w = -i/2)."""
    outs = []
    for w in (0.5, -0.5j):
        h = _handle(p, gamma, np.array([sigma]), np.array([w]), **opt)
        U, st = h.slrf_filter(_dev(X))
        outs.append(_host(U))
        h.close()
    return outs[0] + 1j * outs[1], st


@pytest.mark.parametrize("pcnd", [P.SLRF_PC_JACOBI, P.SLRF_PC_AMG])
@pytest.mark.parametrize("prec", [P.SLRF_PREC_FP64, P.SLRF_PREC_MIXED])
def test_single_pole_solves_meet_tolerance(cfg1, prec, pcnd):
    p = cfg1["pencil"]
    A, B = p.A(), p.B()
    X = cfg1["V1"][:, :12]
    F = B @ X
    tol = 1e-10
    for j in (0, 3, 7):
        sigma = cfg1["poles"][j]
        Y, st = _single_pole_solution(p, cfg1["gamma"], sigma, X, precision=prec, tol_lin=tol,
                                      precond=pcnd)
        M = (A - sigma * B).tocsr()
        rel = np.linalg.norm(F - M @ Y, axis=0) / np.linalg.norm(F, axis=0)
        assert rel.max() <= 1.01 * tol, (j, rel.max())
        assert st["converged"] == 12 and st["capped"] == 0
        Ylu = oracle.filter.shifted_solve_exact(A, B, sigma, F)
        err = oracle.filter.shifted_solve_exact(A, B, sigma, F - M @ Y)
        assert np.linalg.norm(Y + err - Ylu) <= 1e-9 * np.linalg.norm(Ylu)


@pytest.mark.parametrize("variant", [0, 6, 7])
@pytest.mark.parametrize("pcnd", [P.SLRF_PC_JACOBI, P.SLRF_PC_AMG])
@pytest.mark.parametrize("prec", [P.SLRF_PREC_FP64, P.SLRF_PREC_MIXED])
def test_filter_matches_exact_lu_oracle(cfg1, prec, pcnd, variant):
    p = cfg1["pencil"]
    tol = 1e-10
    h = _handle(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"], precision=prec, tol_lin=tol,
                precond=pcnd, spmm_variant=variant)
    X = cfg1["V1"]
    U, st = h.slrf_filter(_dev(X))
    Uo = oracle.filter.apply_filter(p.A(), p.B(), cfg1["poles"], cfg1["weights"], X)
    bound = _filter_bound(p.B() @ X, cfg1["poles"], cfg1["weights"], tol, _q1_lambda_min_B(40, 2))
    err = np.linalg.norm(_host(U) - Uo, axis=0)
    assert np.all(err <= bound), (err / bound).max()
    assert st["converged"] == 8 * X.shape[1] and st["max_rel_resid"] <= tol
    h.close()


@pytest.mark.parametrize("variant", [0, 6, 7])
def test_filter_bitwise_deterministic_and_pool_independent(cfg1, variant):
    p = cfg1["pencil"]
    X = _dev(cfg1["V1"][:, :10])
    h = _handle(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"], spmm_variant=variant)
    U1, _ = h.slrf_filter(X)
    U2, _ = h.slrf_filter(X)
    assert torch.equal(U1, U2)
    h.close()
    # a pool of only 16 resident systems streams the 80 systems through it;
    # every system's arithmetic is independent of its slot, so U is identical
    h = _handle(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"], max_slots=16,
                spmm_variant=variant)
    U3, st = h.slrf_filter(X)
    assert torch.equal(U1, U3)
    h.close()


def test_filter_edge_columns(cfg1):
    p = cfg1["pencil"]
    X = cfg1["V1"][:, :3].copy()
    X[:, 1] = 0.0  # zero right-hand side: y = 0 exactly
    h = _handle(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"])
    U, st = h.slrf_filter(_dev(X), want_sys_iters=True)
    Uh = _host(U)
    assert np.all(Uh[:, 1] == 0.0)
    assert np.all(st["sys_iters"][8:16] == 0)
    # one column
    U1, _ = h.slrf_filter(_dev(X[:, :1]))
    Uo = oracle.filter.apply_filter(p.A(), p.B(), cfg1["poles"], cfg1["weights"], X[:, :1])
    assert np.linalg.norm(_host(U1) - Uo) <= 1e-6 * np.linalg.norm(Uo)
    # ncols = 0 is rejected before any device access
    assert P.lib().slrf_filter(h._h, 0, None, None, None, None) == 1
    h.close()


def test_filter_sine_eigenvectors_full_3d_size():
    """Config at full size (n = 262,144): U = Phi(lambda) x for sine eigenvectors."""
    m = 64
    c = si.config_q1_3d()
    p = c["pencil"]
    poles, weights = si.slrf_poles(c["gamma"], 8)
    h1d = 1.0 / (m + 1)
    t = np.arange(1, m + 1) * np.pi / (m + 1)
    lam1 = (6.0 / h1d ** 2) * (1 - np.cos(t)) / (2 + np.cos(t))
    ks = [(1, 1, 1), (1, 1, 2), (2, 1, 1), (3, 2, 1), (2, 2, 2), (4, 4, 4), (3, 3, 1), (6, 1, 1)]
    X = np.stack([np.kron(np.sin(np.arange(1, m + 1) * a * np.pi / (m + 1)),
                          np.kron(np.sin(np.arange(1, m + 1) * b * np.pi / (m + 1)),
                                  np.sin(np.arange(1, m + 1) * cc * np.pi / (m + 1))))
                  for a, b, cc in ks], axis=1)
    lam = np.array([lam1[a - 1] + lam1[b - 1] + lam1[cc - 1] for a, b, cc in ks])
    phi = np.sum(2 * np.real(weights[None, :] / (lam[:, None] - poles[None, :])), axis=1)
    tol = 1e-10
    for prec, pcnd in ((P.SLRF_PREC_MIXED, P.SLRF_PC_JACOBI), (P.SLRF_PREC_FP64, P.SLRF_PC_JACOBI),
                       (P.SLRF_PREC_MIXED, P.SLRF_PC_AMG)):
        h = _handle(p, c["gamma"], poles, weights, precision=prec, tol_lin=tol, precond=pcnd)
        U, st = h.slrf_filter(_dev(X))
        err = np.linalg.norm(_host(U) - X * phi[None, :], axis=0)
        bound = _filter_bound(p.B() @ X, poles, weights, tol, _q1_lambda_min_B(m, 3))
        assert np.all(err <= bound), (prec, (err / bound).max())
        assert st["converged"] == 8 * len(ks)
        h.close()


def _sine_block_3d(m, ks):
    """Sine products and their closed-form eigenvalues on the m^3 Q1 pencil."""
    h1d = 1.0 / (m + 1)
    t = np.arange(1, m + 1) * np.pi / (m + 1)
    lam1 = (6.0 / h1d ** 2) * (1 - np.cos(t)) / (2 + np.cos(t))
    # sin(j k pi / (m + 1)) with the argument reduced exactly: high modes stay
    # eigenvectors to rounding
    sv = lambda k: np.sin(((np.arange(1, m + 1) * k) % (2 * (m + 1))) * np.pi / (m + 1))
    X = np.stack([np.kron(sv(a), np.kron(sv(b), sv(cc))) for a, b, cc in ks], axis=1)
    lam = np.array([lam1[a - 1] + lam1[b - 1] + lam1[cc - 1] for a, b, cc in ks])
    return X, lam


@pytest.mark.parametrize("prec", [P.SLRF_PREC_MIXED, P.SLRF_PREC_FP64])
def test_filter_sine_full_size_benchmark_options(prec):
    """The benchmark's filter exactly as it runs (n = 262,144, 8 poles, AMG V-cycle
    with a coarsest level of at least 512, GCR(4), tol_lin 1e-8, cold start,
    autotuned sweep): in the mixed form this is the path whose cycles keep the
    Gram-Schmidt basis in complex bfloat16.  Per column U = Phi(lambda) u
    (closed form, Eq. (3)) within the bound the residual tolerance implies;
    modes inside (0, gamma], at the cluster by gamma, just above it and at the
    top of the spectrum.  The same with the default hierarchy (125 coarse
    dofs), which needs over a quarter more inner iterations."""
    m = 64
    c = si.config_q1_3d()
    p = c["pencil"]
    poles, weights = si.slrf_poles(c["gamma"], 8)
    ks = [(1, 1, 1), (2, 1, 1), (3, 2, 1), (4, 3, 1), (5, 1, 1), (4, 3, 2), (6, 1, 1),
          (64, 64, 64), (33, 7, 50), (1, 64, 2)]
    X, lam = _sine_block_3d(m, ks)
    phi = np.sum(2 * np.real(weights[None, :] / (lam[:, None] - poles[None, :])), axis=1)
    tol = 1e-8
    bound = _filter_bound(p.B() @ X, poles, weights, tol, _q1_lambda_min_B(m, 3))
    iters = {}
    for cmin in (512, 0):
        h = _handle(p, c["gamma"], poles, weights, precision=prec, tol_lin=tol,
                    precond=P.SLRF_PC_AMG, restart=4, amg_coarse_min=cmin)
        U, st = h.slrf_filter(_dev(X))
        h.close()
        assert st["basis_bf16"] == (1 if prec == P.SLRF_PREC_MIXED else 0)
        assert st["converged"] == 8 * len(ks) and st["max_rel_resid"] <= tol
        err = np.linalg.norm(_host(U) - X * phi[None, :], axis=0)
        assert np.all(err <= bound), (prec, cmin, (err / bound).max())
        iters[cmin] = st["total_iters"]
    assert iters[0] > 1.25 * iters[512], iters


@pytest.mark.parametrize("prec", [P.SLRF_PREC_MIXED, P.SLRF_PREC_FP64])
def test_filter_lu_oracle_benchmark_options(cfg1, prec):
    """The benchmark's filter options (AMG, GCR(4), tol_lin 1e-8, halo sweep) on the
    2D configuration against the exact-LU oracle, column by column, with every
    system's FP64 residual recomputed on the host from the single-pole solves."""
    p = cfg1["pencil"]
    tol = 1e-8
    opt = dict(precision=prec, tol_lin=tol, precond=P.SLRF_PC_AMG, restart=4, spmm_variant=6,
               amg_coarse_min=512)
    h = _handle(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"], **opt)
    X = cfg1["V1"]
    U, st = h.slrf_filter(_dev(X))
    h.close()
    assert st["basis_bf16"] == (1 if prec == P.SLRF_PREC_MIXED else 0)
    Uo = oracle.filter.apply_filter(p.A(), p.B(), cfg1["poles"], cfg1["weights"], X)
    bound = _filter_bound(p.B() @ X, cfg1["poles"], cfg1["weights"], tol, _q1_lambda_min_B(40, 2))
    err = np.linalg.norm(_host(U) - Uo, axis=0)
    assert np.all(err <= bound), (err / bound).max()
    assert st["converged"] == 8 * X.shape[1] and st["max_rel_resid"] <= tol
    A, B = p.A(), p.B()
    F = B @ X[:, :6]
    for j in (0, 4, 7):
        Y, sj = _single_pole_solution(p, cfg1["gamma"], cfg1["poles"][j], X[:, :6], **opt)
        M = (A - cfg1["poles"][j] * B).tocsr()
        rel = np.linalg.norm(F - M @ Y, axis=0) / np.linalg.norm(F, axis=0)
        assert rel.max() <= 1.01 * tol, (j, rel.max())


# ----------------------------------------------------------------------------
# truncated GCR (It_max-linear) and warm start (Algorithm 2, Proposition 4.1)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("restart", [30, 3])
def test_truncated_warm_started_gcr_matches_oracle_iterates(cfg1, restart):
    p = cfg1["pencil"]
    A, B = p.A(), p.B()
    X = cfg1["V1"][:, :4]
    theta = np.array([40.0, 120.0, 310.0, 500.0])
    itmax = 7
    for j in (1, 6):
        sigma = cfg1["poles"][j]
        outs = []
        for w in (0.5, -0.5j):
            h = _handle(p, cfg1["gamma"], np.array([sigma]), np.array([w]), it_max_lin=itmax,
                        restart=restart)
            U, st = h.slrf_filter(_dev(X), theta_warm=theta)
            outs.append(_host(U))
            h.close()
        Y = outs[0] + 1j * outs[1]
        M = (A - sigma * B).tocsr()
        pc = oracle.gcr.jacobi(A, B, sigma)
        for col in range(4):
            x0 = X[:, col].astype(np.complex128) / (theta[col] - sigma)
            yo, its, _ = oracle.gcr.gcr(lambda v: M @ v, B @ X[:, col], x0, pc, restart=restart,
                                        tol=1e-10, maxit=itmax)
            assert its == itmax
            assert np.linalg.norm(Y[:, col] - yo) <= 1e-10 * np.linalg.norm(yo), (j, col)


def test_warm_start_converges_to_same_filter(cfg1):
    p = cfg1["pencil"]
    X = cfg1["V1"][:, :8]
    theta = np.linspace(30.0, 600.0, 8)
    h = _handle(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"])
    U0, s0 = h.slrf_filter(_dev(X))
    U1, s1 = h.slrf_filter(_dev(X), theta_warm=theta)
    bound = _filter_bound(p.B() @ X, cfg1["poles"], cfg1["weights"], 1e-10, _q1_lambda_min_B(40, 2))
    assert np.all(np.linalg.norm(_host(U0) - _host(U1), axis=0) <= 2 * bound)
    h.close()


# ----------------------------------------------------------------------------
# Rayleigh-Ritz (a9-a12) and full solves (Algorithms 1 and 2)
# ----------------------------------------------------------------------------
def test_rayleigh_ritz_matches_oracle(cfg1):
    p = cfg1["pencil"]
    A, B = p.A(), p.B()
    U = oracle.filter.apply_filter(A, B, cfg1["poles"], cfg1["weights"], cfg1["V1"])
    th_o, V_o = oracle.eig.rayleigh_ritz(A, B, U)
    res_o = oracle.eig.residual_norms(A, B, th_o, V_o)
    h = _handle(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"])
    V, th, res = h.slrf_rayleigh_ritz(_dev(U))
    th, res, V = _host(th), _host(res), _host(V)
    assert np.max(np.abs(th - th_o) / np.abs(th_o)) <= 1e-11
    big = res_o > 1e-9
    assert np.allclose(res[big], res_o[big], rtol=1e-5)
    assert np.all(res[~big] < 1e-8)
    assert np.max(np.abs(V.T @ (B @ V) - np.eye(V.shape[1]))) <= 1e-10
    h.close()


def test_rayleigh_ritz_with_locked_vectors(cfg1):
    p = cfg1["pencil"]
    A, B = p.A(), p.B()
    lam, Xe = oracle.eig.dense_eigs(A, B)
    Xl = Xe[:, :5]
    U = cfg1["V1"][:, :12]
    Ub = oracle.eig.b_orthogonalize(B, Xl, U)
    th_o, _ = oracle.eig.rayleigh_ritz(A, B, Ub)
    h = _handle(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"])
    V, th, res = h.slrf_rayleigh_ritz(_dev(U), Xlocked=_dev(Xl))
    V = _host(V)
    assert np.max(np.abs(Xl.T @ (B @ V))) <= 1e-11
    assert np.max(np.abs(_host(th) - th_o) / np.abs(th_o)) <= 1e-10
    h.close()


def _closed_q1_2d(m, k):
    h = 1.0 / (m + 1)
    t = np.arange(1, m + 1) * np.pi / (m + 1)
    l1 = (6.0 / h ** 2) * (1 - np.cos(t)) / (2 + np.cos(t))
    return np.sort((l1[:, None] + l1[None, :]).ravel())[:k]


@pytest.mark.parametrize("mode", ["alg1_fp64", "alg2_fp64", "alg1_mixed", "alg2_mixed",
                                  "alg1_mixed_amg", "alg2_fp64_amg"])
def test_solve_config_q1_2d_closed_form(cfg1, mode):
    p = cfg1["pencil"]
    opt = dict(tol_lin=1e-10)
    if mode.endswith("_amg"):
        opt.update(precond=P.SLRF_PC_AMG)
        mode = mode[:-4]
    if mode.startswith("alg2"):
        opt.update(lock=1, warm_start=1, it_max_lin=13)
    if mode.endswith("mixed"):
        opt.update(precision=P.SLRF_PREC_MIXED)
    h = _handle(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"], **opt)
    th, X, nconv, st = h.slrf_solve(cfg1["nev"], _dev(cfg1["V1"]))
    ex = _closed_q1_2d(40, cfg1["nev"])
    assert nconv == cfg1["nev"]
    tol = 1e-10 if mode.endswith("fp64") else 1e-8
    assert np.max(np.abs(_host(th) - ex) / ex) <= tol, mode
    Xh = _host(X)
    res = oracle.eig.residual_norms(p.A(), p.B(), _host(th), Xh)
    assert res.max() < 1e-8
    h.close()


@pytest.mark.parametrize("prec", [P.SLRF_PREC_FP64, P.SLRF_PREC_MIXED])
def test_solve_q1_3d_m64_full_size_closed_form(prec):
    """The benchmark pencil at full size (n = 262,144, L = 160, 8 poles): Algorithm 2
    (locking, warm start; AMG-GCR(8); inner tolerance 1e-10) finds all 102
    eigenvalues of (0, gamma] (a 6-fold cluster at the boundary of the 100th)
    within 1e-10 (FP64) / 1e-8 (mixed) relative of the closed form, with
    sampled Ritz residuals recomputed on the host."""
    c = si.config_q1_3d()
    p, gamma, nev = c["pencil"], c["gamma"], c["nev"]
    poles, weights = si.slrf_poles(gamma)
    h = _handle(p, gamma, poles, weights, precision=prec, precond=P.SLRF_PC_AMG, restart=8,
                tol_lin=1e-10, lock=1, warm_start=1)
    th, X, nconv, st = h.slrf_solve(nev, _dev(si.start_block(p.n, c["L"], c["seed"])))
    h.close()
    assert nconv == nev
    h1 = 1.0 / 65
    t = np.arange(1, 13) * np.pi / 65
    lam1 = (6.0 / h1 ** 2) * (1 - np.cos(t)) / (2 + np.cos(t))  # 12 smallest 1D eigenvalues
    ex = np.sort((lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]).ravel())
    ex = ex[:nev]
    tol = 1e-10 if prec == P.SLRF_PREC_FP64 else 1e-8
    assert np.max(np.abs(_host(th) - ex) / ex) <= tol
    # Ritz residuals of 6 sampled pairs (first, cluster, last), recomputed in FP64
    idx = np.array([0, 1, 50, 97, 100, nev - 1])
    Xh = _host(X[:, idx])
    res = oracle.eig.residual_norms(p.A(), p.B(), _host(th)[idx], Xh)
    assert res.max() < 1e-8


@pytest.mark.parametrize("pcnd", [P.SLRF_PC_JACOBI, P.SLRF_PC_AMG])
def test_solve_3d_diffusion_vs_dense_lapack(pcnd):
    p = si.q1_diffusion_pencil(8, 3, np.exp(np.random.default_rng(4).normal(0, .5, 9 ** 3)))
    lam, _ = oracle.eig.dense_eigs(p.A(), p.B())
    nev = 12
    gamma = 0.5 * (lam[nev - 1] + lam[nev])
    poles, weights = si.slrf_poles(gamma)
    h = _handle(p, gamma, poles, weights, lock=1, warm_start=1, precond=pcnd)
    th, X, nconv, st = h.slrf_solve(nev, _dev(si.start_block(p.n, 18, 9)))
    assert nconv == nev
    assert np.max(np.abs(_host(th) - lam[:nev]) / lam[:nev]) <= 1e-10
    h.close()


# ----------------------------------------------------------------------------
# argument validation through the ABI
# ----------------------------------------------------------------------------
def test_setup_rejects_malformed_input():
    p = si.q1_kron_pencil(6, 2)
    poles, weights = si.slrf_poles(100.0)
    bad = p.indices.copy()
    bad[[1, 2]] = bad[[2, 1]]  # unsorted row
    with pytest.raises(P.SlrfError) as e:
        P.Handle(p.indptr, bad, p.a, p.b, 100.0, poles, weights)
    assert e.value.status == 1
    with pytest.raises(P.SlrfError) as e:
        P.Handle(p.indptr, p.indices, p.a, p.b, 100.0, np.conj(poles), weights)
    assert e.value.status == 1
    with pytest.raises(P.SlrfError) as e:
        P.Handle(p.indptr, p.indices, p.a, p.b, -1.0, poles, weights)
    assert e.value.status == 1


@pytest.mark.parametrize("prec", [P.SLRF_PREC_FP64, P.SLRF_PREC_MIXED])
def test_amg_elasticity_single_pole_residuals(prec):
    """AMG on a 3-dof elasticity pencil (aggregation of coupled dofs): every solve certified."""
    p = si.hex_elasticity_pencil(6, np.exp(np.random.default_rng(8).normal(0, .5, 216)))
    A, B = p.A(), p.B()
    lam = oracle.eig.dense_eigs(A, B)[0]
    gamma = 0.5 * (lam[9] + lam[10])
    poles, _ = si.slrf_poles(gamma)
    X = si.start_block(p.n, 5, 21)
    F = B @ X
    for j in (0, 7):
        Y, st = _single_pole_solution(p, gamma, poles[j], X, precision=prec, tol_lin=1e-10,
                                      precond=P.SLRF_PC_AMG)
        M = (A - poles[j] * B).tocsr()
        rel = np.linalg.norm(F - M @ Y, axis=0) / np.linalg.norm(F, axis=0)
        assert rel.max() <= 1.01e-10 and st["converged"] == 5


# ----------------------------------------------------------------------------
# caller-owned workspace
# ----------------------------------------------------------------------------
def test_workspace_minimum_streams_and_undersized_is_refused(cfg1):
    """The handle's device memory is the caller's workspace: at the minimum size
    (one panel of 16 resident systems) the filter streams its 256 systems and
    returns exactly the block of a full-size workspace; a workspace too small
    for the pencil data fails setup, and one that holds the pencil but not a
    call's buffers fails that call, both with SLRF_E_NOMEM."""
    p = cfg1["pencil"]
    X = _dev(cfg1["V1"])
    opt = dict(precision=P.SLRF_PREC_MIXED, precond=P.SLRF_PC_AMG, restart=5, tol_lin=1e-9)
    h = P.Handle.from_pencil(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"],
                             P.default_options(**opt), max_cols=32)
    full, mn = h.workspace_sizes(32)
    assert h.workspace.numel() == full and mn < full
    U1, st1 = h.slrf_filter(X)
    one_col_min = h.workspace_sizes(1)[1]
    h.close()
    h = P.Handle.from_pencil(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"],
                             P.default_options(**opt), workspace_bytes=mn)
    U2, st2 = h.slrf_filter(X)
    assert torch.equal(U1, U2) and st2["converged"] == st1["converged"] == 256
    h.close()
    with pytest.raises(P.SlrfError) as e:
        P.Handle.from_pencil(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"],
                             P.default_options(**opt), workspace_bytes=64 * 1024)
    assert e.value.status == 2
    h = P.Handle.from_pencil(p, cfg1["gamma"], cfg1["poles"], cfg1["weights"],
                             P.default_options(**opt), workspace_bytes=one_col_min)
    U3, _ = h.slrf_filter(X[:, :1])
    assert torch.equal(U3[:, 0], U1[:, 0])
    with pytest.raises(P.SlrfError) as e:
        h.slrf_filter(X)
    assert e.value.status == 2 and "workspace" in str(e.value)
    h.close()


@pytest.mark.parametrize("prec", [P.SLRF_PREC_FP64, P.SLRF_PREC_MIXED])
def test_real_spmm_halo_and_csr_forms_agree_bitwise(prec):
    """The right-hand sides F = B X come from the halo-tile real SpMM for an even
    column count and from the CSR kernel for an odd one; both sum each row in
    CSR order.  A system's arithmetic does not depend on its slot, so the first
    seven columns of a filtered 8-column block equal the 7-column filter bit
    for bit; warm-started filters (E = A X - theta B X on the same paths) too."""
    p = si.q1_diffusion_pencil(24, 3, np.exp(np.random.default_rng(21).normal(0, .5, 25 ** 3)))
    gamma = 60.0
    poles, weights = si.slrf_poles(gamma)
    X = si.start_block(p.n, 8, 2101)
    h = _handle(p, gamma, poles, weights, precision=prec, precond=P.SLRF_PC_AMG, restart=5,
                tol_lin=1e-9)
    U8, st8 = h.slrf_filter(_dev(X))
    U7, st7 = h.slrf_filter(_dev(X[:, :7]))
    assert st8["converged"] == 64 and st7["converged"] == 56
    assert torch.equal(U8[:, :7], U7)
    theta = np.linspace(5.0, 40.0, 8)
    W8, _ = h.slrf_filter(_dev(X), theta_warm=theta)
    W7, _ = h.slrf_filter(_dev(X[:, :7]), theta_warm=theta[:7])
    assert torch.equal(W8[:, :7], W7)
    h.close()
