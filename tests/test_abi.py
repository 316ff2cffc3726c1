"""The C-ABI library loads on the CPU and exports every declared entry point."""

import re
import os

import numpy as np
import scipy.linalg as sla

import paper_2510_17334_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "slrf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(slrf_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = declared_functions()
    assert "slrf_filter" in names and "slrf_solve" in names and "slrf_setup" in names
    for nm in names:
        assert hasattr(L, nm), nm
    # the binding wraps exactly the declared set
    assert set(names) == set(P.slrf.SIGNATURES)


def test_default_options_are_the_papers():
    o = P.default_options()
    assert o.tol_lin == 1e-10 and o.maxit_lin == 10000  # Section 3.2
    assert o.tol_eig == 1e-8 and o.max_outer == 100
    assert o.precision == P.SLRF_PREC_FP64 and o.restart == 30


def test_status_strings():
    L = P.lib()
    assert L.slrf_status_string(0) == b"ok"
    assert b"argument" in L.slrf_status_string(1)


def _rand_pencil(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A = A + A.T
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    B = Q @ np.diag(np.logspace(0, np.log10(cond), n)) @ Q.T
    return A, 0.5 * (B + B.T)


def test_host_projected_eig_matches_lapack():
    for n, seed in [(1, 0), (2, 1), (17, 2), (160, 3), (300, 4)]:
        A, B = _rand_pencil(n, seed)
        k, th, S = P.host_projected_eig(A, B)
        w = sla.eigh(A, B, eigvals_only=True)
        assert k == n
        scale = np.abs(w).max()
        assert np.max(np.abs(th - w)) <= 1e-11 * scale
        assert np.max(np.abs(S.T @ B @ S - np.eye(n))) <= 1e-10
        assert np.max(np.abs(A @ S - (B @ S) * th)) <= 1e-10 * scale * np.abs(B).max()


def test_host_projected_eig_truncates_singular_gram():
    rng = np.random.default_rng(5)
    U = rng.standard_normal((40, 6))
    U = np.concatenate([U, U[:, :2]], axis=1)  # two duplicated columns
    Kd = np.diag(np.linspace(1, 5, 40))
    A = U.T @ Kd @ U
    B = U.T @ U
    k, th, S = P.host_projected_eig(A, B)
    assert k == 6
    w = sla.eigh(U[:, :6].T @ Kd @ U[:, :6], U[:, :6].T @ U[:, :6], eigvals_only=True)
    assert np.allclose(th[:6], w, rtol=1e-8)
    assert np.all(np.isinf(th[6:]))


def test_host_check_of_gradient_element_data():
    """slrf_eig_grad's host checks (the same code the entry point runs before its
    kernel): dofs in [-1, n), strides 0 or >= ndof_e^2, element matrices inside
    the given lengths; anything else is SLRF_E_ARG."""
    L = P.lib()
    n, nelem, nd = 50, 3, 4
    dofs = np.array([[0, 1, 2, -1], [3, 4, 5, 6], [7, 8, 49, 10]], dtype=np.int32)

    def chk(d=dofs, sa=0, la=16, hb=0, sb=0, lb=0, nn=n, ne=nelem, k=nd):
        return L.slrf_host_check_grad_args(nn, ne, k, d.ctypes.data, sa, la, hb, sb, lb)

    assert chk() == 0
    assert chk(sa=16, la=48) == 0 and chk(hb=1, sb=16, lb=48) == 0
    bad = dofs.copy()
    bad[2, 2] = 50  # = n
    assert chk(d=bad) == 1
    bad[2, 2] = -2
    assert chk(d=bad) == 1
    assert chk(la=15) == 1             # shared matrix shorter than 4 x 4
    assert chk(sa=16, la=47) == 1      # last element's matrix past the end
    assert chk(sa=8, la=100) == 1      # stride below ndof_e^2
    assert chk(hb=1, sb=0, lb=10) == 1
    assert chk(k=6) == 1               # unsupported element size
    assert chk(ne=0, d=np.zeros(0, np.int32), la=0) == 0



def test_coarse_level_floor_is_validated_before_any_device_work():
    """slrf_setup checks its options before it touches the pencil or a device: an
    AMG coarse-level floor outside [0, 2048] is SLRF_E_ARG with its own message
    (host-only structures suffice; a valid floor gets past the check and fails
    later, on this machine for want of a device or a readable pencil)."""
    import ctypes as C
    L = P.lib()
    csr = P.slrf.Csr()
    zd = (P.slrf.Zd * 8)()
    ws = (C.c_char * 4096)()
    msgs = {}
    for cmin in (-1, 2049, 0, 2048):
        o = P.default_options(precond=P.SLRF_PC_AMG, amg_coarse_min=cmin)
        h = C.c_void_p()
        st = L.slrf_setup(C.byref(h), C.byref(csr), C.byref(csr), 1.0, 8, zd, zd, C.byref(o),
                          ws, 4096, None)
        assert st != 0
        msgs[cmin] = (st, L.slrf_last_error(h).decode())
        L.slrf_destroy(h)
    for bad in (-1, 2049):
        assert msgs[bad][0] == 1 and "amg_coarse_min" in msgs[bad][1], msgs[bad]
    for good in (0, 2048):
        assert "amg_coarse_min" not in msgs[good][1], msgs[good]
