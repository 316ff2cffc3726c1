"""Batched entry points (many uneven pencils at once) through the C ABI.

* slrf_filter_batch returns, for every pencil, exactly (bitwise) the block the
  single slrf_filter call returns: each handle's arithmetic is independent of
  what runs beside it on other streams.
* slrf_solve_batch (Algorithm 2: locking, warm start; inner tolerance 1e-10 as
  in Section 3.2) on the 64-pencil uneven batch (Q1 diffusion, lognormal
  coefficients, n in [5000, 60000], 10-60 eigenvalues each) finds every
  eigenvalue of each interval (0, gamma] within 1e-8 relative of the oracle's
  shift-invert Lanczos values (tests/golden/batch64_q1_diffusion.json, written
  by the script beside it from oracle/ only).
"""

import json
import os

import numpy as np
import pytest

import paper_2510_17334_amd as P
import slrf_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batch64_q1_diffusion.json")


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(x).T), device="cuda").t()


def _small_batch():
    rng = np.random.default_rng(11)
    specs = [(2, 20), (3, 9), (2, 33), (3, 13), (2, 41)]
    out = []
    for dim, m in specs:
        kappa = np.exp(rng.normal(0, 0.5, (m + 1) ** dim))
        out.append(si.q1_diffusion_pencil(m, dim, kappa))
    return out


@pytest.mark.parametrize("prec", [P.SLRF_PREC_FP64, P.SLRF_PREC_MIXED])
def test_filter_batch_equals_single_calls(prec):
    pencils = _small_batch()
    hs, Xs = [], []
    for i, p in enumerate(pencils):
        gamma = 50.0 + 10 * i
        poles, weights = si.slrf_poles(gamma)
        opt = P.default_options(precision=prec, precond=P.SLRF_PC_AMG, restart=8, tol_lin=1e-9)
        hs.append(P.Handle.from_pencil(p, gamma, poles, weights, opt, stream=torch.cuda.Stream()))
        Xs.append(_dev(si.start_block(p.n, 6 + 3 * i, 300 + i)))
    torch.cuda.synchronize()
    out = P.slrf_filter_batch(hs, Xs, nthreads=4)
    for h, X, (U, st) in zip(hs, Xs, out):
        U1, st1 = h.slrf_filter(X)
        assert torch.equal(U, U1)
        assert st["converged"] == st1["converged"] == st["nsystems"]
        assert st["total_iters"] == st1["total_iters"]
    for h in hs:
        h.close()


def test_filter_batch_rejects_duplicate_handles():
    p = _small_batch()[0]
    poles, weights = si.slrf_poles(50.0)
    h = P.Handle.from_pencil(p, 50.0, poles, weights, P.default_options())
    X = _dev(si.start_block(p.n, 4, 1))
    with pytest.raises(P.SlrfError):
        P.slrf_filter_batch([h, h], [X, X])
    h.close()


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden batch eigenvalues not generated")
def test_solve_batch_64_uneven_pencils_match_oracle():
    gold = json.load(open(GOLDEN))["pencils"]
    draws = si.batched_pencils(64, seed=1004)
    hs, V1s, nevs = [], [], []
    for d, g in zip(draws, gold):
        p = d["pencil"]
        assert p.n == g["n"] and d["count"] == g["count"]
        poles, weights = si.slrf_poles(g["gamma"])
        opt = P.default_options(precision=P.SLRF_PREC_MIXED, precond=P.SLRF_PC_AMG, restart=8,
                                tol_lin=1e-10, lock=1, warm_start=1, max_outer=60)
        hs.append(P.Handle.from_pencil(p, g["gamma"], poles, weights, opt,
                                       stream=torch.cuda.Stream()))
        V1s.append(_dev(si.start_block(p.n, d["L"], d["seed"])))
        nevs.append(d["count"])
    torch.cuda.synchronize()
    out = P.slrf_solve_batch(hs, nevs, V1s, nthreads=8)
    worst = 0.0
    for (theta, X, nconv, st), g in zip(out, gold):
        lam = np.array(g["eigenvalues"])
        assert nconv == g["count"], (g["index"], nconv, g["count"])
        th = np.sort(theta.cpu().numpy())
        rel = np.abs(th - lam) / lam
        worst = max(worst, rel.max())
        assert rel.max() <= 1e-8, (g["index"], rel.max())
    print("worst relative eigenvalue error", worst)
    for h in hs:
        h.close()


def test_filter_batch_benchmark_options_coarse_floor():
    """Four pencils of the 64-pencil batch with the batch benchmark's options
    (mixed, AMG with a coarse-level floor of 128, GCR(4), tol_lin 1e-8): three
    of the hierarchies end in dense levels of 1728, 625 and 729 unknowns
    instead of 27 to 81 (the fourth already ends in 343), every system
    converges to its FP64 residual, the batched call equals the single calls
    bit for bit, and the floor cuts the inner iterations against the default
    hierarchy."""
    gold = json.load(open(GOLDEN))["pencils"]
    idx = [5, 40, 3, 19]
    draws = si.batched_pencils(64, seed=1004, only=idx)
    iters = {}
    for cmin in (128, 0):
        hs, Xs = [], []
        for d in draws:
            g = gold[d["index"]]
            poles, weights = si.slrf_poles(g["gamma"])
            opt = P.default_options(precision=P.SLRF_PREC_MIXED, precond=P.SLRF_PC_AMG,
                                    restart=4, tol_lin=1e-8, amg_coarse_min=cmin)
            hs.append(P.Handle.from_pencil(d["pencil"], g["gamma"], poles, weights, opt,
                                           stream=torch.cuda.Stream(), max_cols=d["L"]))
            Xs.append(_dev(si.start_block(d["pencil"].n, d["L"], d["seed"])))
        torch.cuda.synchronize()
        out = P.slrf_filter_batch(hs, Xs, nthreads=4)
        total = 0
        for h, X, (U, st) in zip(hs, Xs, out):
            assert st["converged"] == st["nsystems"] and st["max_rel_resid"] <= 1e-8
            total += st["total_iters"]
            if cmin:
                U1, st1 = h.slrf_filter(X)
                assert torch.equal(U, U1) and st["total_iters"] == st1["total_iters"]
        iters[cmin] = total
        for h in hs:
            h.close()
    assert iters[0] > 1.15 * iters[128], iters
