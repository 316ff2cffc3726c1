"""ctypes binding of the C ABI declared in include/slrf.h.

Argument marshalling only: tensors are checked for device, dtype and layout and
their data pointers handed to the library; every step of the computation runs
in the HIP kernels of ``libslrf.so``.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libslrf.so")

SLRF_PREC_FP64 = 0
SLRF_PREC_MIXED = 1
SLRF_AMG_HOST = 0
SLRF_AMG_DEVICE = 1
SLRF_PC_NONE = 0
SLRF_PC_JACOBI = 1
SLRF_PC_AMG = 2
KERNEL_CLASSES = ("apply", "orth", "step", "resid", "reduce", "other", "precond", "sweep")
_STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "HIP runtime error",
           4: "breakdown", 5: "iteration cap reached", 6: "NaN/Inf detected", 7: "no usable GPU"}


class SlrfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"slrf status {status} ({_STATUS.get(status, '?')}): {msg}")
        self.status = status


class Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class Zd(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("precond", C.c_int32), ("restart", C.c_int32),
                ("maxit_lin", C.c_int32), ("it_max_lin", C.c_int32), ("max_outer", C.c_int32),
                ("warm_start", C.c_int32), ("lock", C.c_int32), ("timing", C.c_int32),
                ("max_slots", C.c_int32), ("spmm_variant", C.c_int32), ("reorder", C.c_int32),
                ("tol_lin", C.c_double),
                ("inner_rtol", C.c_double),
                ("tol_eig", C.c_double), ("amg_block", C.c_int32),
                ("node_xyz", C.c_void_p), ("amg_setup", C.c_int32),
                ("amg_coarse_min", C.c_int32)]


class FilterStats(C.Structure):
    _fields_ = [("nsystems", C.c_int64), ("total_iters", C.c_int64), ("min_iters", C.c_int32),
                ("max_iters", C.c_int32), ("cycles", C.c_int32), ("converged", C.c_int32),
                ("capped", C.c_int32), ("max_pole_iters_ratio_x1000", C.c_int32),
                ("max_rel_resid", C.c_double), ("seconds", C.c_double),
                ("launches", C.c_int64 * 8), ("bytes", C.c_double * 8), ("ms", C.c_double * 8),
                ("spmm_variant", C.c_int32), ("sweep_systems", C.c_double),
                ("basis_bf16", C.c_int32), ("sys_iters", C.POINTER(C.c_int32))]


class SolveStats(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("nconv", C.c_int32), ("auto_it_max", C.c_int32),
                ("inner_iters", C.c_int64),
                ("seconds", C.c_double), ("filter_seconds", C.c_double),
                ("rr_seconds", C.c_double)]


_lib = None

# name -> (restype, argtypes): every entry point declared in include/slrf.h
SIGNATURES = {
    "slrf_status_string": (C.c_char_p, [C.c_int]),
    "slrf_last_error": (C.c_char_p, [C.c_void_p]),
    "slrf_default_options": (None, [C.POINTER(Options)]),
    "slrf_workspace_size": (C.c_int, [C.POINTER(Csr), C.POINTER(Csr), C.c_int32, C.c_int32,
                                      C.POINTER(Options), C.POINTER(C.c_size_t),
                                      C.POINTER(C.c_size_t)]),
    "slrf_setup": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(Csr), C.POINTER(Csr), C.c_double,
                             C.c_int32, C.POINTER(Zd), C.POINTER(Zd), C.POINTER(Options),
                             C.c_void_p, C.c_size_t, C.c_void_p]),
    "slrf_destroy": (None, [C.c_void_p]),
    "slrf_set_options": (C.c_int, [C.c_void_p, C.POINTER(Options)]),
    "slrf_filter": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.POINTER(FilterStats)]),
    "slrf_rayleigh_ritz": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "slrf_solve": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.POINTER(C.c_int32), C.POINTER(SolveStats)]),
    "slrf_shifted_spmm": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                    C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "slrf_shifted_spmm_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                            C.c_int32, C.c_void_p, C.c_void_p]),
    "slrf_get_n": (C.c_int32, [C.c_void_p]),
    "slrf_get_row_order": (C.c_int, [C.c_void_p, C.c_void_p]),
    "slrf_eig_grad": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                C.c_int64, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p]),
    "slrf_host_check_grad_args": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                              C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                              C.c_int64]),
    "slrf_host_projected_eig": (C.c_int32, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p]),
    "slrf_filter_batch": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                    C.POINTER(C.c_void_p), C.POINTER(FilterStats), C.c_int32]),
    "slrf_solve_batch": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_int32), C.POINTER(SolveStats), C.c_int32]),
}


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libslrf.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"HIP library {_LIB_PATH} is missing; build it with "
                               "`python -m paper_2510_17334_amd.build`")
        L = C.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def default_options(**kw) -> Options:
    o = Options()
    lib().slrf_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def host_projected_eig(Ah: np.ndarray, Bh: np.ndarray):
    """The library's host solve of Ah s = theta Bh s (no GPU)."""
    Ah = np.ascontiguousarray(Ah, dtype=np.float64)
    Bh = np.ascontiguousarray(Bh, dtype=np.float64)
    n = Ah.shape[0]
    th = np.zeros(n)
    S = np.zeros((n, n))
    k = lib().slrf_host_projected_eig(n, Ah.ctypes.data, Bh.ctypes.data, th.ctypes.data,
                                      S.ctypes.data)
    return k, th, S


def _torch():
    import torch
    return torch


def _colmajor(x, n: int):
    """(n, k) float64 CUDA tensor in column-major storage (returns a view or copy)."""
    torch = _torch()
    if x.dim() != 2 or x.shape[0] != n:
        raise ValueError(f"expected an (n={n}, k) block, got {tuple(x.shape)}")
    if x.dtype != torch.float64 or not x.is_cuda:
        raise ValueError("blocks must be float64 CUDA tensors")
    if x.stride(0) == 1 and (x.shape[1] <= 1 or x.stride(1) == n):
        return x
    return x.t().contiguous().t()


def _empty_colmajor(n: int, k: int, device):
    torch = _torch()
    return torch.empty((k, n), dtype=torch.float64, device=device).t()


def workspace_size(A: Csr, B: Csr, L: int, npoles: int, options: Options):
    """(full, minimum) workspace bytes of slrf_workspace_size."""
    full, mn = C.c_size_t(0), C.c_size_t(0)
    st = lib().slrf_workspace_size(C.byref(A), C.byref(B), int(L), int(npoles),
                                   C.byref(options), C.byref(full), C.byref(mn))
    if st != 0:
        raise SlrfError(st, "slrf_workspace_size failed (malformed pencil or options)")
    return full.value, mn.value


class Handle:
    """A pencil bound to the GPU library (slrf_setup ... slrf_destroy).

    ``indptr``/``indices``/``a``/``b`` are host arrays (numpy) of a shared-pattern
    CSR pencil; they are uploaded once and kept alive by the handle.

    The device workspace is a torch uint8 tensor owned by the handle: by default
    slrf_workspace_size's full size for blocks of ``max_cols`` columns (every
    shifted system resident), capped at ``budget`` (a fraction of the free
    device memory when below 1, else bytes; default 0.25) but never below the
    minimum; ``workspace_bytes`` sets the size directly.
    """

    def __init__(self, indptr, indices, a, b, gamma: float, poles, weights,
                 options: Optional[Options] = None, device: str = "cuda", stream=None,
                 max_cols: int = 64, budget: float = 0.25,
                 workspace_bytes: Optional[int] = None, coords=None):
        torch = _torch()
        self._L = lib()
        self.device = torch.device(device)
        self.n = int(len(indptr) - 1)
        self.indptr = torch.as_tensor(np.asarray(indptr, dtype=np.int32), device=self.device)
        self.indices = torch.as_tensor(np.asarray(indices, dtype=np.int32), device=self.device)
        self.a = torch.as_tensor(np.asarray(a, dtype=np.float64), device=self.device)
        self.b = torch.as_tensor(np.asarray(b, dtype=np.float64), device=self.device)
        self.gamma = float(gamma)
        poles = np.asarray(poles, dtype=np.complex128)
        weights = np.asarray(weights, dtype=np.complex128)
        self.npoles = int(poles.shape[0])
        self.poles = poles
        self.weights = weights
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        A = Csr(self.n, int(self.indices.numel()), self.indptr.data_ptr(), self.indices.data_ptr(),
                self.a.data_ptr())
        B = Csr(self.n, int(self.indices.numel()), self.indptr.data_ptr(), self.indices.data_ptr(),
                self.b.data_ptr())
        zp = (Zd * self.npoles)(*[Zd(p.real, p.imag) for p in poles])
        zw = (Zd * self.npoles)(*[Zd(w.real, w.imag) for w in weights])
        self.options = options if options is not None else default_options()
        if coords is not None:
            # node coordinates for the AMG's rigid-body modes (kept alive here)
            self._coords = np.ascontiguousarray(coords, dtype=np.float64)
            opt = Options()
            C.pointer(opt)[0] = self.options
            opt.node_xyz = self._coords.ctypes.data
            self.options = opt
        self._h = C.c_void_p()
        torch.cuda.synchronize(self.device)
        self._A, self._B = A, B
        full, mn = workspace_size(A, B, max_cols, self.npoles, self.options)
        if workspace_bytes is None:
            # free device memory, counting torch's cached but unused blocks
            free = torch.cuda.mem_get_info(self.device)[0] + (
                torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device))
            cap = int(budget * free) if budget <= 1.0 else int(budget)
            workspace_bytes = max(mn, min(full, cap))
        self.workspace_full, self.workspace_min = full, mn
        self.workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        st = self._L.slrf_setup(C.byref(h), C.byref(A), C.byref(B), self.gamma, self.npoles, zp,
                                zw, C.byref(self.options), C.c_void_p(self.workspace.data_ptr()),
                                self.workspace.numel(), C.c_void_p(self.stream.cuda_stream))
        self._h = h
        if st != 0:
            msg = self._L.slrf_last_error(h).decode() if h.value else "setup failed"
            self.close()
            raise SlrfError(st, msg)

    def workspace_sizes(self, L: int):
        """(full, minimum) workspace bytes of this pencil for blocks of L columns."""
        return workspace_size(self._A, self._B, L, self.npoles, self.options)

    @classmethod
    def from_pencil(cls, p, gamma, poles, weights, options=None, **kw):
        """Handle of a slrf_inputs.Pencil (its node coordinates, if any, go to the AMG)."""
        if getattr(p, "coords", None) is not None and "coords" not in kw:
            kw["coords"] = p.coords
        return cls(p.indptr, p.indices, p.a, p.b, gamma, poles, weights, options, **kw)

    def _check(self, st: int, allow=()):
        if st != 0 and st not in allow:
            raise SlrfError(st, self._L.slrf_last_error(self._h).decode())
        return st

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.slrf_destroy(self._h)
        self._h = C.c_void_p()
        self.workspace = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, options: Options):
        self._check(self._L.slrf_set_options(self._h, C.byref(options)))
        self.options = options

    # --- slrf_filter ---------------------------------------------------------
    def slrf_filter(self, X, theta_warm=None, want_sys_iters: bool = False, allow_noconv=False):
        """U = sum_j 2 Re(w_j (A - sigma_j B)^{-1} B X).  Returns (U, stats dict)."""
        torch = _torch()
        X = _colmajor(X, self.n)
        k = X.shape[1]
        U = _empty_colmajor(self.n, k, X.device)
        st = FilterStats()
        its = None
        if want_sys_iters:
            its = np.zeros(k * self.npoles, dtype=np.int32)
            st.sys_iters = its.ctypes.data_as(C.POINTER(C.c_int32))
        th = None
        if theta_warm is not None:
            th = torch.as_tensor(theta_warm, dtype=torch.float64, device=X.device).contiguous()
            if th.numel() != k:
                raise ValueError("theta_warm needs one value per column")
        r = self._L.slrf_filter(self._h, k, X.data_ptr(), th.data_ptr() if th is not None else None,
                                U.data_ptr(), C.byref(st))
        self._check(r, allow=(5,) if allow_noconv else ())
        return U, self._stats_dict(st, its, r)

    @staticmethod
    def _stats_dict(st: FilterStats, its, status):
        d = {f: getattr(st, f) for f, _ in FilterStats._fields_ if f not in
             ("launches", "bytes", "ms", "sys_iters")}
        d["launches"] = dict(zip(KERNEL_CLASSES, list(st.launches)))
        d["bytes"] = dict(zip(KERNEL_CLASSES, list(st.bytes)))
        d["ms"] = dict(zip(KERNEL_CLASSES, list(st.ms)))
        d["sys_iters"] = its
        d["status"] = status
        return d

    # --- slrf_rayleigh_ritz --------------------------------------------------
    def slrf_rayleigh_ritz(self, U, Xlocked=None):
        """Ritz values/vectors of span(U) (B-orthogonalised against Xlocked).

        Returns (V, theta, resid); V is a new column-major block.
        """
        torch = _torch()
        V = _colmajor(U, self.n).t().clone().t()
        k = V.shape[1]
        theta = torch.empty(k, dtype=torch.float64, device=V.device)
        resid = torch.empty(k, dtype=torch.float64, device=V.device)
        nl = 0
        xp = None
        if Xlocked is not None and Xlocked.shape[1] > 0:
            Xl = _colmajor(Xlocked, self.n)
            nl = Xl.shape[1]
            xp = Xl.data_ptr()
        self._check(self._L.slrf_rayleigh_ritz(self._h, k, V.data_ptr(), nl, xp, theta.data_ptr(),
                                               resid.data_ptr()))
        return V, theta, resid

    # --- slrf_solve ----------------------------------------------------------
    def slrf_solve(self, nev: int, V1, allow_noconv=False):
        """Algorithm 1 or 2 (per options).  Returns (theta, X, nconv, stats dict)."""
        torch = _torch()
        V1 = _colmajor(V1, self.n)
        L = V1.shape[1]
        theta = torch.full((nev,), float("nan"), dtype=torch.float64, device=V1.device)
        X = _empty_colmajor(self.n, nev, V1.device)
        nconv = C.c_int32(0)
        st = SolveStats()
        r = self._L.slrf_solve(self._h, nev, L, V1.data_ptr(), theta.data_ptr(), X.data_ptr(),
                               C.byref(nconv), C.byref(st))
        self._check(r, allow=(5,) if allow_noconv else ())
        stats = {f: getattr(st, f) for f, _ in SolveStats._fields_}
        stats["status"] = r
        return theta[:nconv.value], X[:, :nconv.value], nconv.value, stats

    def slrf_get_row_order(self):
        """Internal row order (order[new] = old) used by slrf_shifted_spmm vectors."""
        order = np.zeros(self.n, dtype=np.int32)
        self._check(self._L.slrf_get_row_order(self._h, order.ctypes.data))
        return order

    # --- slrf_eig_grad -------------------------------------------------------
    def slrf_eig_grad(self, X, lam, glam, elem_dofs, dA, dB=None, dA_stride=0, dB_stride=0):
        """grad_e = sum_i glam_i x_{i,e}^T (dA_e - lam_i dB_e) x_{i,e} (device tensor)."""
        torch = _torch()
        X = _colmajor(X, self.n)
        k = X.shape[1]
        dev = X.device
        lam = torch.as_tensor(lam, dtype=torch.float64, device=dev).contiguous()
        glam = torch.as_tensor(glam, dtype=torch.float64, device=dev).contiguous()
        dofs = torch.as_tensor(np.asarray(elem_dofs, dtype=np.int32) if not torch.is_tensor(elem_dofs)
                               else elem_dofs, device=dev).to(torch.int32).contiguous()
        nelem, nd = dofs.shape
        dA = torch.as_tensor(dA, dtype=torch.float64, device=dev).contiguous()
        dBt = None if dB is None else torch.as_tensor(dB, dtype=torch.float64, device=dev).contiguous()
        grad = torch.empty(nelem, dtype=torch.float64, device=dev)
        self._check(self._L.slrf_eig_grad(self._h, k, X.data_ptr(), lam.data_ptr(),
                                          glam.data_ptr(), nelem, nd, dofs.data_ptr(),
                                          dA.data_ptr(), dA_stride, dA.numel(),
                                          dBt.data_ptr() if dBt is not None else None, dB_stride,
                                          dBt.numel() if dBt is not None else 0,
                                          grad.data_ptr()))
        return grad

    # --- slrf_shifted_spmm ---------------------------------------------------
    def slrf_shifted_spmm(self, Z, pole_idx, precision: int = SLRF_PREC_FP64, timed=False):
        """Q = (A - sigma_{pole[s]} B) Z on a panel-layout block (see include/slrf.h)."""
        torch = _torch()
        pole_idx = np.ascontiguousarray(pole_idx, dtype=np.int32)
        nsys = pole_idx.shape[0]
        npad = (nsys + 15) // 16 * 16
        dt = torch.complex128 if precision == SLRF_PREC_FP64 else torch.complex64
        if Z.dtype != dt or not Z.is_cuda or Z.numel() != npad * self.n or not Z.is_contiguous():
            raise ValueError("Z must be a contiguous panel-layout complex CUDA tensor")
        Q = torch.empty_like(Z)
        ms = C.c_double(0.0)
        self._check(self._L.slrf_shifted_spmm(self._h, nsys,
                                              pole_idx.ctypes.data_as(C.POINTER(C.c_int32)),
                                              precision, Z.data_ptr(), Q.data_ptr(),
                                              C.byref(ms) if timed else None))
        return (Q, ms.value) if timed else Q


class EigFn:
    """torch.autograd.Function: eigenvalues in (0, gamma] of a parameterised pencil.

    ``forward(theta, problem)`` assembles A(theta), B(theta) on the host through
    ``problem.assemble(theta_numpy) -> slrf_inputs.Pencil`` (with element data),
    solves with ``slrf_solve`` on the GPU and returns the NEV eigenvalues;
    ``backward`` returns dL/dtheta through the adjoint kernel ``slrf_eig_grad``:
    dL/dtheta_e = sum_i g_i x_i^T (dA/dtheta_e - lambda_i dB/dtheta_e) x_i.
    ``problem`` also provides gamma, nev, V1 (host n x L), poles, weights,
    options and, for the element derivatives, ``dA``/``dB`` (ndof x ndof
    reference matrices; dB may be None) so that dA/dtheta_e = dA on element e.
    """

    @staticmethod
    def _impl():
        torch = _torch()

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, theta, problem):
                p = problem.assemble(theta.detach().cpu().numpy())
                h = Handle.from_pencil(p, problem.gamma, problem.poles, problem.weights,
                                       problem.options, device=str(theta.device)
                                       if theta.is_cuda else "cuda",
                                       max_cols=int(np.asarray(problem.V1).shape[1]))
                V1 = torch.as_tensor(np.ascontiguousarray(np.asarray(problem.V1).T),
                                     device=h.device).t()
                lam, X, nconv, _ = h.slrf_solve(problem.nev, V1)
                if nconv != problem.nev:
                    raise SlrfError(5, f"only {nconv} of {problem.nev} eigenpairs converged")
                ctx.h = h
                ctx.dofs = p.elem_dofs
                ctx.problem = problem
                ctx.save_for_backward(lam, X)
                return lam.to(theta.device)

            @staticmethod
            def backward(ctx, glam):
                lam, X = ctx.saved_tensors
                g = ctx.h.slrf_eig_grad(X, lam, glam.to(lam.device, torch.float64), ctx.dofs,
                                        ctx.problem.dA, getattr(ctx.problem, "dB", None))
                ctx.h.close()
                return g, None

        return _Fn

    @classmethod
    def apply(cls, theta, problem):
        return cls._impl().apply(theta, problem)


def to_panels(Y, n: int):
    """(n, nsys) complex tensor -> contiguous panel layout [nsys/16, n, 16] (padded)."""
    torch = _torch()
    nsys = Y.shape[1]
    npad = (nsys + 15) // 16 * 16
    Z = torch.zeros((n, npad), dtype=Y.dtype, device=Y.device)
    Z[:, :nsys] = Y
    return Z.reshape(n, npad // 16, 16).permute(1, 0, 2).contiguous()


def from_panels(Z, n: int, nsys: int):
    return Z.permute(1, 0, 2).reshape(n, -1)[:, :nsys]


# --- batched entry points -------------------------------------------------------
def _ptrs(ts):
    arr = (C.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def _sync_streams(handles):
    """Order every handle's stream after the caller's current stream."""
    torch = _torch()
    cur = torch.cuda.current_stream()
    for h in handles:
        if h.stream != cur:
            h.stream.wait_stream(cur)


def slrf_filter_batch(handles, Xs, thetas=None, nthreads: int = 0, allow_noconv=False):
    """slrf_filter on every (handle, X) pair, run concurrently (largest first).

    Returns a list of (U, stats dict).  Give each handle its own stream.
    """
    nh = len(handles)
    if len(Xs) != nh or (thetas is not None and len(thetas) != nh):
        raise ValueError("one X (and theta) per handle")
    torch = _torch()
    Xs = [_colmajor(X, h.n) for h, X in zip(handles, Xs)]
    Us = [_empty_colmajor(h.n, X.shape[1], X.device) for h, X in zip(handles, Xs)]
    ths = None
    if thetas is not None:
        ths = [None if t is None else torch.as_tensor(t, dtype=torch.float64,
                                                      device=X.device).contiguous()
               for t, X in zip(thetas, Xs)]
    hs = (C.c_void_p * nh)(*[h._h.value for h in handles])
    nc = (C.c_int32 * nh)(*[X.shape[1] for X in Xs])
    st = (FilterStats * nh)()
    _sync_streams(handles)
    r = lib().slrf_filter_batch(nh, hs, nc, _ptrs(Xs), _ptrs(ths) if ths is not None else None,
                                _ptrs(Us), st, nthreads)
    if r != 0 and not (allow_noconv and r == 5):
        msgs = "; ".join(lib().slrf_last_error(h._h).decode() for h in handles)
        raise SlrfError(r, msgs)
    return [(U, Handle._stats_dict(st[i], None, r)) for i, U in enumerate(Us)]


def slrf_solve_batch(handles, nevs, V1s, nthreads: int = 0, allow_noconv=False):
    """slrf_solve on every handle, run concurrently (largest first).

    Returns a list of (theta, X, nconv, stats dict).
    """
    nh = len(handles)
    torch = _torch()
    V1s = [_colmajor(V, h.n) for h, V in zip(handles, V1s)]
    thetas = [torch.full((k,), float("nan"), dtype=torch.float64, device=V.device)
              for k, V in zip(nevs, V1s)]
    Xs = [_empty_colmajor(h.n, k, V.device) for h, k, V in zip(handles, nevs, V1s)]
    hs = (C.c_void_p * nh)(*[h._h.value for h in handles])
    nev = (C.c_int32 * nh)(*[int(k) for k in nevs])
    Ls = (C.c_int32 * nh)(*[V.shape[1] for V in V1s])
    nconv = (C.c_int32 * nh)()
    st = (SolveStats * nh)()
    _sync_streams(handles)
    r = lib().slrf_solve_batch(nh, hs, nev, Ls, _ptrs(V1s), _ptrs(thetas), _ptrs(Xs), nconv, st,
                               nthreads)
    if r != 0 and not (allow_noconv and r == 5):
        msgs = "; ".join(lib().slrf_last_error(h._h).decode() for h in handles)
        raise SlrfError(r, msgs)
    out = []
    for i in range(nh):
        k = nconv[i]
        d = {f: getattr(st[i], f) for f, _ in SolveStats._fields_}
        out.append((thetas[i][:k], Xs[i][:, :k], k, d))
    return out
