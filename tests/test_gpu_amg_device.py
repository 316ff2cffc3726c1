"""The device-built AMG hierarchy (options.amg_setup = SLRF_AMG_DEVICE).

The aggregation and the tentative prolongators run on the host; each level's
products (rho(D^-1 A), A T, the smoothed prolongator and its transpose, A P,
B P and the Galerkin products) run on the GPU in the host code's order, with
every product rounded before it is added.  The hierarchy therefore equals the
host build's, and so does everything computed with it: the filtered block and
the iteration counts of a filter call are compared bit for bit."""

import numpy as np
import pytest

import paper_2510_17334_amd as P
import slrf_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(x).T), device="cuda").t()


def _pencil(which):
    rng = np.random.default_rng(11)
    if which == "q1_3d":
        m = 24
        return si.q1_diffusion_pencil(m, 3, np.exp(rng.normal(0, .5, (m + 1) ** 3))), 60.0
    ne = 10
    return si.hex_elasticity_pencil(ne, np.exp(rng.normal(0, .3, ne ** 3))), 5.0


@pytest.mark.parametrize("which,prec,cmin", [("q1_3d", P.SLRF_PREC_MIXED, 0),
                                             ("q1_3d", P.SLRF_PREC_FP64, 0),
                                             ("q1_3d", P.SLRF_PREC_MIXED, 512),
                                             ("elasticity", P.SLRF_PREC_FP64, 0)])
def test_device_amg_setup_equals_host_build(which, prec, cmin):
    p, gamma = _pencil(which)
    poles, weights = si.slrf_poles(gamma)
    X = _dev(np.random.default_rng(5).standard_normal((p.n, 16)))
    out = {}
    for where in (P.SLRF_AMG_HOST, P.SLRF_AMG_DEVICE):
        opt = P.default_options(precision=prec, precond=P.SLRF_PC_AMG, restart=5, tol_lin=1e-9,
                                amg_setup=where, amg_coarse_min=cmin)
        h = P.Handle.from_pencil(p, gamma, poles, weights, opt, max_cols=16)
        U, st = h.slrf_filter(X)
        out[where] = (U, st, h.workspace_sizes(16))
        h.close()
    (U0, st0, ws0), (U1, st1, ws1) = out[P.SLRF_AMG_HOST], out[P.SLRF_AMG_DEVICE]
    assert st0["converged"] == st1["converged"] == 128
    assert st0["total_iters"] == st1["total_iters"]
    assert torch.equal(U0, U1)
    # (the device build's workspace estimate bounds the hierarchy it has not seen)
    assert ws1[0] >= ws0[0] and ws1[1] >= ws0[1]


def test_device_amg_setup_in_the_minimum_workspace():
    """slrf_workspace_size's bound holds: at the device build's reported minimum
    the hierarchy is built (its products in the workspace above the pencil) and
    the filter streams its systems to the block of a full-size workspace; a
    64 KiB workspace is refused with SLRF_E_NOMEM."""
    p, gamma = _pencil("elasticity")
    poles, weights = si.slrf_poles(gamma)
    X = _dev(np.random.default_rng(6).standard_normal((p.n, 16)))
    dev = P.default_options(precision=P.SLRF_PREC_MIXED, precond=P.SLRF_PC_AMG, restart=5,
                            tol_lin=1e-9, amg_setup=P.SLRF_AMG_DEVICE)
    h = P.Handle.from_pencil(p, gamma, poles, weights, dev, max_cols=16)
    U1, st1 = h.slrf_filter(X)
    mn = h.workspace_sizes(16)[1]
    h.close()
    h = P.Handle.from_pencil(p, gamma, poles, weights, dev, workspace_bytes=mn)
    U2, st2 = h.slrf_filter(X)
    h.close()
    assert torch.equal(U1, U2) and st1["converged"] == st2["converged"] == 128
    with pytest.raises(P.SlrfError) as e:
        P.Handle.from_pencil(p, gamma, poles, weights, dev, workspace_bytes=64 * 1024)
    assert e.value.status == 2
