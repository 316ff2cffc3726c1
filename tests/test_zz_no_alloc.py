"""The allocation-free sweep entry point against the ordinary one, through the C ABI.

slrf_shifted_spmm_noalloc keeps its pole table in a fixed per-GPU library array
instead of library workspace; it must give exactly the Q of slrf_shifted_spmm
(the same kernel on the same table), also when a call follows a larger one
whose table entries are still in the array.
"""

import ctypes as C

import numpy as np
import pytest

import paper_2510_17334_amd as P
import slrf_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _sweep(h, fn, Z, pidx, prec):
    Q = torch.full_like(Z, float("nan"))
    pole = np.ascontiguousarray(pidx, dtype=np.int32)
    args = [h._h, len(pole), pole.ctypes.data_as(C.POINTER(C.c_int32)), prec, Z.data_ptr(),
            Q.data_ptr()]
    if fn == "slrf_shifted_spmm":
        args.append(None)
    st = getattr(P.lib(), fn)(*args)
    assert st == 0, P.lib().slrf_last_error(h._h).decode()
    return Q


@pytest.mark.parametrize("prec", [P.SLRF_PREC_FP64, P.SLRF_PREC_MIXED])
def test_noalloc_sweep_equals_allocating_sweep(prec):
    p = si.q1_diffusion_pencil(12, 3, np.exp(np.random.default_rng(2).normal(0, .5, 13 ** 3)))
    poles, weights = si.slrf_poles(300.0)
    h = P.Handle.from_pencil(p, 300.0, poles, weights, P.default_options())
    dt = torch.complex128 if prec == P.SLRF_PREC_FP64 else torch.complex64
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    # first call: 203 systems (13 panels, ragged); second: 37 systems (3 panels)
    for nsys, seed in ((203, 1), (37, 2)):
        npad = (nsys + 15) // 16 * 16
        Z = torch.randn((npad // 16, p.n, 16), dtype=dt, device="cuda", generator=g)
        pidx = np.random.default_rng(seed).integers(0, len(poles), nsys)
        Qa = _sweep(h, "slrf_shifted_spmm", Z, pidx, prec)
        Qb = _sweep(h, "slrf_shifted_spmm_noalloc", Z, pidx, prec)
        assert torch.equal(Qa, Qb), nsys
        assert torch.isfinite(torch.view_as_real(Qb)).all()
    h.close()


def test_noalloc_sweep_rejects_more_systems_than_its_table():
    p = si.q1_kron_pencil(6, 2)
    poles, weights = si.slrf_poles(100.0)
    h = P.Handle.from_pencil(p, 100.0, poles, weights, P.default_options())
    Z = torch.zeros((1, p.n, 16), dtype=torch.complex128, device="cuda")
    pole = np.zeros(65537, dtype=np.int32)
    st = P.lib().slrf_shifted_spmm_noalloc(h._h, len(pole),
                                           pole.ctypes.data_as(C.POINTER(C.c_int32)),
                                           P.SLRF_PREC_FP64, Z.data_ptr(), Z.data_ptr())
    assert st == 1
    assert b"65536" in P.lib().slrf_last_error(h._h)
    h.close()
