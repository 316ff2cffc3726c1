"""GPU parity of the eigenvalue-gradient path (adjoint kernel and EigFn).

The kernel is compared with the oracle's per-element loop (same formula,
different summation order: 1e-12 relative); the autograd chain is checked by
Euler homogeneity (A linear in theta, B independent: sum_e theta_e dL/dtheta_e
= sum_i dL/dlambda_i lambda_i) and by central finite differences of dense
eigenvalues (relative step 1e-6, agreement 1e-5) and, on the full 32^3
elasticity mesh, of eigenvalues from GPU solves.
"""

import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import paper_2510_17334_amd as P
import slrf_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(x).T), device="cuda").t()


@pytest.mark.parametrize("kind", ["elasticity", "q1_3d", "q1_2d"])
def test_eig_grad_kernel_matches_oracle(kind):
    rng = np.random.default_rng(3)
    if kind == "elasticity":
        p = si.hex_elasticity_pencil(3, np.exp(rng.normal(0, .3, 27)))
        dB = None
    elif kind == "q1_3d":
        p = si.q1_diffusion_pencil(5, 3, np.exp(rng.normal(0, .5, 216)))
        dB = p.me_ref  # a density-like parameter entering B as well
    else:
        p = si.q1_diffusion_pencil(9, 2, np.exp(rng.normal(0, .5, 100)))
        dB = p.me_ref
    lam, Xe = oracle.eig.dense_eigs(p.A(), p.B())
    k = 7
    X, lam = Xe[:, :k], lam[:k]
    glam = rng.standard_normal(k)
    ref = oracle.grad.eig_grad(p.elem_dofs, p.ke_ref, dB, X, lam, glam)
    poles, weights = si.slrf_poles(lam[-1] * 1.1)
    h = P.Handle.from_pencil(p, lam[-1] * 1.1, poles, weights)
    g = h.slrf_eig_grad(_dev(X), lam, glam, p.elem_dofs, p.ke_ref, dB).cpu().numpy()
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))
    h.close()


class _ElasticProblem:
    def __init__(self, ne, nev, L, seed):
        self.ne = ne
        E0 = np.exp(np.random.default_rng(seed).normal(0, .3, ne ** 3))
        p0 = si.hex_elasticity_pencil(ne, E0)
        lam = oracle.eig.dense_eigs(p0.A(), p0.B())[0]
        self.nev = nev
        self.gamma = 0.5 * (lam[nev - 1] + lam[nev])
        self.poles, self.weights = si.slrf_poles(self.gamma)
        self.options = P.default_options(lock=1, warm_start=1, tol_lin=1e-10, tol_eig=1e-10,
                                         precond=P.SLRF_PC_AMG)
        self.V1 = si.start_block(p0.n, L, seed + 1)
        self.dA = p0.ke_ref
        self.dB = None
        self.E0 = E0

    def assemble(self, theta):
        return si.hex_elasticity_pencil(self.ne, np.asarray(theta, dtype=np.float64))


def test_eigfn_autograd_homogeneity_and_finite_differences():
    prob = _ElasticProblem(ne=4, nev=8, L=14, seed=5)
    theta = torch.tensor(prob.E0, dtype=torch.float64, device="cuda", requires_grad=True)
    lam = P.EigFn.apply(theta, prob)
    loss = lam.sum()
    loss.backward()
    g = theta.grad.cpu().numpy()
    lam_h = lam.detach().cpu().numpy()
    # Euler homogeneity: sum_e theta_e dL/dtheta_e = sum_i lambda_i
    assert np.isclose(np.sum(prob.E0 * g), lam_h.sum(), rtol=1e-9)
    # dense reference eigenvalues
    ref = sla.eigh(prob.assemble(prob.E0).A().toarray(), prob.assemble(prob.E0).B().toarray(),
                   eigvals_only=True)[:prob.nev]
    assert np.max(np.abs(lam_h - ref) / ref) < 1e-10
    # central differences on a few elements
    for e in np.random.default_rng(9).choice(prob.E0.size, 5, replace=False):
        d = 1e-6 * prob.E0[e]
        Ep, Em = prob.E0.copy(), prob.E0.copy()
        Ep[e] += d
        Em[e] -= d
        lp = sla.eigh(prob.assemble(Ep).A().toarray(), prob.assemble(Ep).B().toarray(),
                      eigvals_only=True)[:prob.nev].sum()
        lm = sla.eigh(prob.assemble(Em).A().toarray(), prob.assemble(Em).B().toarray(),
                      eigvals_only=True)[:prob.nev].sum()
        fd = (lp - lm) / (2 * d)
        assert np.isclose(g[e], fd, rtol=1e-5, atol=1e-8 * np.abs(g).max()), (e, g[e], fd)


GOLD_E32 = os.path.join(os.path.dirname(__file__), "golden", "elasticity32.json")


@pytest.mark.skipif(not os.path.exists(GOLD_E32), reason="golden elasticity eigenvalues missing")
def test_elasticity32_solve_and_gradient_full_size():
    """The differentiation workload at full size (n = 104,544, 50 eigenvalues):
    mixed Algorithm 2 eigenvalues vs the oracle's shift-invert Lanczos (1e-8
    relative after refinement; FP64 residuals of every inner solve 1e-10),
    the adjoint kernel vs the oracle's per-element formula on 20 sampled
    elements (same eigenvectors, 1e-10) and vs the oracle's gradient from its
    own eigenvectors (1e-5), and Euler homogeneity over all 32,768 elements
    (sum_e E_e dL/dE_e = sum_i lambda_i)."""
    gold = json.load(open(GOLD_E32))
    c = si.config_elasticity(32, 0.3, 1005, 50, 75)
    p = c["pencil"]
    assert p.n == gold["n"]
    poles, weights = si.slrf_poles(gold["gamma"])
    # Algorithm 2 (locking, warm start, It_max-linear = 60); AMG whose coarse
    # space carries the rigid-body modes (node coordinates from the pencil)
    opt = P.default_options(precision=P.SLRF_PREC_MIXED, precond=P.SLRF_PC_AMG, restart=30,
                            tol_lin=1e-10, lock=1, warm_start=1, max_outer=60, it_max_lin=60)
    h = P.Handle.from_pencil(p, gold["gamma"], poles, weights, opt, max_cols=c["L"])
    V1 = _dev(si.start_block(p.n, c["L"], c["seed"]))
    theta, X, nconv, st = h.slrf_solve(c["count"], V1)
    assert nconv == c["count"]
    lam = np.array(gold["eigenvalues"])
    th = theta.cpu().numpy()
    assert np.max(np.abs(th - lam) / lam) <= 1e-8
    glam = np.ones(nconv)
    g = h.slrf_eig_grad(X, th, glam, p.elem_dofs, p.ke_ref, None).cpu().numpy()
    assert np.isclose(np.sum(c["young"] * g), th.sum(), rtol=1e-9)
    idx = np.array(gold["sample_elements"])
    Xh = X.cpu().numpy()
    ref = oracle.grad.eig_grad(p.elem_dofs[idx], p.ke_ref, None, Xh, th, glam)
    assert np.max(np.abs(g[idx] - ref)) <= 1e-10 * np.max(np.abs(ref))
    # against the oracle's own gradient (its Lanczos eigenvectors; the sum over
    # the whole invariant subspace is basis-independent): the eigenvector error
    # of a Ritz residual below 1e-8 enters to first order, so 1e-5 relative
    gref = np.array(gold["grad_sum_lambda_samples"])
    err = np.max(np.abs(g[idx] - gref)) / np.max(np.abs(gref))
    print("gradient vs oracle gradient, max relative error", err)
    assert err <= 1e-5
    h.close()


@pytest.mark.skipif(not os.path.exists(GOLD_E32), reason="golden elasticity eigenvalues missing")
def test_elasticity32_central_differences_full_size():
    """Central differences of the sum of the 50 smallest eigenvalues on the full
    32^3 mesh, both sides solved on the GPU (FP64 Algorithm 2 to Ritz residuals
    1e-11, warm-started from the unperturbed eigenvectors), relative step 1e-6
    in E_e, against the adjoint kernel on 3 of the 20 sampled elements (the
    benchmark's fd32 workload covers all 20).  The quotient's error is the
    eigenvalue-sum error over the difference: about 1e-12 over d * g ~ 1e-8,
    so 2e-4 relative."""
    gold = json.load(open(GOLD_E32))
    c = si.config_elasticity(32, 0.3, 1005, 50, 75)
    p, nev = c["pencil"], c["count"]
    poles, weights = si.slrf_poles(gold["gamma"])
    opt = P.default_options(precision=P.SLRF_PREC_FP64, precond=P.SLRF_PC_AMG, restart=5,
                            tol_lin=1e-14, it_max_lin=20, lock=1, warm_start=1, max_outer=60,
                            tol_eig=1e-11)

    def solve(pen, V):
        h = P.Handle.from_pencil(pen, gold["gamma"], poles, weights, opt, max_cols=c["L"])
        th, X, nconv, _ = h.slrf_solve(nev, V)
        assert nconv == nev
        return h, th, X

    V1 = _dev(si.start_block(p.n, c["L"], c["seed"]))
    h, th, X = solve(p, V1)
    g = h.slrf_eig_grad(X, th.cpu().numpy(), np.ones(nev), p.elem_dofs, p.ke_ref).cpu().numpy()
    h.close()
    Vw = torch.cat([X, V1[:, nev:]], 1)
    for e in gold["sample_elements"][::7]:
        d = 1e-6 * c["young"][e]
        sums = []
        for sgn in (1.0, -1.0):
            y = c["young"].copy()
            y[e] += sgn * d
            hp, thp, _ = solve(si.hex_elasticity_pencil(32, y), Vw)
            sums.append(float(thp.sum()))
            hp.close()
        fd = (sums[0] - sums[1]) / (2 * d)
        print(f"element {e}: adjoint {g[e]:.12g} central difference {fd:.12g}")
        assert abs(fd - g[e]) <= 2e-4 * abs(g[e]), (e, g[e], fd)


def test_eig_grad_rejects_malformed_element_data():
    """Out-of-range dofs and element matrices past their arrays are refused with
    SLRF_E_ARG before the kernel runs."""
    rng = np.random.default_rng(4)
    p = si.q1_diffusion_pencil(5, 3, np.exp(rng.normal(0, .5, 216)))
    poles, weights = si.slrf_poles(100.0)
    h = P.Handle.from_pencil(p, 100.0, poles, weights)
    X = _dev(rng.standard_normal((p.n, 3)))
    lam, glam = np.ones(3), np.ones(3)
    g = h.slrf_eig_grad(X, lam, glam, p.elem_dofs, p.ke_ref)
    assert torch.isfinite(g).all()
    bad = p.elem_dofs.copy()
    bad[5, 3] = p.n
    with pytest.raises(P.SlrfError) as e:
        h.slrf_eig_grad(X, lam, glam, bad, p.ke_ref)
    assert e.value.status == 1
    with pytest.raises(P.SlrfError) as e:  # per-element stride over a single matrix
        h.slrf_eig_grad(X, lam, glam, p.elem_dofs, p.ke_ref, dA_stride=64)
    assert e.value.status == 1
    h.close()
