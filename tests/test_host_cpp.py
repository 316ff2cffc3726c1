"""The library's host-side setup code (C++, no GPU) through a small driver
(tests/host_driver.cpp, compiled with g++ at test time):

* locality_order: a permutation; with node blocks it keeps each node's dofs
  together and in order;
* detect_block: 3 on node-major elasticity, 1 on scalar pencils and on a
  pattern with one node row changed;
* build_halo: the halo-tile format reproduces the CSR pencil exactly (every
  entry back through its tile's halo), padding entries are zero, tile and
  slice invariants hold, and an over-wide slice is refused;
* amg_build: every coarse pair is the Galerkin product (P^T A P, P^T B P) to
  rounding, R = P^T, the dense coarsest inverse inverts A_c - sigma B_c, and
  the power-iteration estimate of rho(D^-1 A) is within 10 % below the true
  value;
* fine_image: (A P_0, B P_0) and P_0's values on that pattern, and their
  rectangular halo-tile layout (columns are coarse rows) carrying P as the
  third value array.
"""

import os
import shutil
import struct
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import slrf_inputs as si

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2510_17334_amd", "csrc")


def _halo_entry(sptr_s, j, ln):
    """Position of entry j of row lane ln in a slice: groups of 4 entries per row."""
    return sptr_s * 8 + (j // 4) * 32 + ln * 4 + j % 4


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("host")
    exe = str(d / "host_driver")
    cmd = [gxx, "-O1", "-std=c++17", "-pthread", "-I", CSRC, os.path.join(HERE, "host_driver.cpp"),
           os.path.join(CSRC, "amg_host.cpp"), os.path.join(CSRC, "halo_host.cpp"),
           os.path.join(CSRC, "ugroup_host.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe, d


def _write(p, path):
    with open(path, "wb") as f:
        f.write(struct.pack("ii", p.n, len(p.indices)))
        f.write(np.asarray(p.indptr, np.int32).tobytes())
        f.write(np.asarray(p.indices, np.int32).tobytes())
        f.write(np.asarray(p.a, np.float64).tobytes())
        f.write(np.asarray(p.b, np.float64).tobytes())


class _Reader:
    def __init__(self, path):
        self.buf = open(path, "rb").read()
        self.pos = 0

    def i(self):
        v = struct.unpack_from("q", self.buf, self.pos)[0]
        self.pos += 8
        return v

    def arr(self, dt):
        k = self.i()
        a = np.frombuffer(self.buf, dtype=dt, count=k, offset=self.pos).copy()
        self.pos += k * np.dtype(dt).itemsize
        return a


def _run(driver, p, *args):
    exe, d = driver
    src, out = str(d / "pencil.bin"), str(d / "out.bin")
    _write(p, src)
    subprocess.run([exe, src, out] + [str(a) for a in args], check=True)
    return _Reader(out)


class _Csr:
    """Minimal pencil-like holder for hand-made patterns."""

    def __init__(self, A, B):
        A, B = A.tocsr(), B.tocsr()
        A.sort_indices()
        B.sort_indices()
        self.n = A.shape[0]
        self.indptr, self.indices, self.a, self.b = A.indptr, A.indices, A.data, B.data


def _elastic(ne=4, seed=0):
    return si.hex_elasticity_pencil(ne, np.exp(np.random.default_rng(seed).normal(0, .3, ne ** 3)))


def test_locality_order_permutation_and_blocks(driver):
    p = si.q1_kron_pencil(10, 3)
    order = _run(driver, p, "order", 1).arr(np.int32)
    assert np.array_equal(np.sort(order), np.arange(p.n))
    e = _elastic()
    order = _run(driver, e, "order", 3).arr(np.int32)
    assert np.array_equal(np.sort(order), np.arange(e.n))
    o = order.reshape(-1, 3)
    assert np.all(o % 3 == np.arange(3)) and np.all(o // 3 == (o[:, :1] // 3))


def test_detect_block(driver):
    assert _run(driver, _elastic(), "block").i() == 3
    assert _run(driver, si.q1_kron_pencil(8, 3), "block").i() == 1
    e = _elastic()
    A = sp.csr_matrix((e.a, e.indices, e.indptr)).tolil()
    B = sp.csr_matrix((e.b, e.indices, e.indptr)).tolil()
    j = A.rows[4][-1]  # drop one off-diagonal entry of one dof row (and its mirror)
    for M in (A, B):
        M[4, j] = 0.0
        M[j, 4] = 0.0
    A, B = A.tocsr(), B.tocsr()
    A.eliminate_zeros()
    B = sp.csr_matrix((np.ones_like(A.data), A.indices, A.indptr))  # same pattern
    assert _run(driver, _Csr(A, B), "block").i() == 1


@pytest.mark.parametrize("hmax,cap", [(192, 512), (224, 32)])
@pytest.mark.parametrize("which", ["q1_2d", "random"])
def test_halo_format_reproduces_csr(driver, which, hmax, cap):
    if which == "q1_2d":
        p = si.q1_kron_pencil(30, 2)
    else:
        rng = np.random.default_rng(4)
        n = 603  # ragged last slice
        M = sp.random(n, n, density=0.01, random_state=5, format="csr")
        M = M + M.T + sp.identity(n)
        M.data = rng.standard_normal(M.nnz)
        Bm = M.copy()
        Bm.data = rng.standard_normal(M.nnz)
        p = _Csr(M, Bm)
    r = _run(driver, p, "halo", hmax, cap)
    assert r.i() == 1
    hmx, emax = r.i(), r.i()
    trow, hptr, halo = r.arr(np.int32), r.arr(np.int32), r.arr(np.int32)
    sptr, slen = r.arr(np.int32), r.arr(np.int32)
    lcol, ab = r.arr(np.uint16), r.arr(np.float64).reshape(-1, 2)
    n = p.n
    assert trow[0] == 0 and trow[-1] == n and np.all(np.diff(trow) > 0)
    assert np.all(trow[:-1] % 8 == 0) and np.all(np.diff(trow) <= cap)
    assert np.max(np.diff(hptr)) == hmx <= hmax
    assert np.all(np.diff(sptr) % 4 == 0)
    rows, cols, va, vb = [], [], [], []
    for t in range(len(trow) - 1):
        h = halo[hptr[t]:hptr[t + 1]]
        assert np.all(np.diff(h) > 0)
        for rrow in range(trow[t], trow[t + 1]):
            s, ln = rrow // 8, rrow % 8
            L = slen[rrow]
            k = _halo_entry(sptr[s], np.arange(sptr[s + 1] - sptr[s]), ln)
            assert np.all(ab[k[L:]] == 0.0) and np.all(lcol[k[L:]] == 0)
            rows += [rrow] * L
            cols += list(h[lcol[k[:L]]])
            va += list(ab[k[:L], 0])
            vb += list(ab[k[:L], 1])
    A = sp.csr_matrix((p.a, p.indices, p.indptr), shape=(n, n))
    B = sp.csr_matrix((p.b, p.indices, p.indptr), shape=(n, n))
    A2 = sp.csr_matrix((va, (rows, cols)), shape=(n, n))
    B2 = sp.csr_matrix((vb, (rows, cols)), shape=(n, n))
    assert (A - A2).count_nonzero() == 0 and (B - B2).count_nonzero() == 0
    # the largest 4-slice pass
    passes = [(sptr[min(a + 4, b)] - sptr[a]) * 8 for t in range(len(trow) - 1)
              for a, b in [(trow[t] // 8, (trow[t + 1] + 7) // 8)]
              for a in range(a, b, 4)]
    assert emax == max(passes)
    # a slice referencing more rows than the halo holds is refused
    assert _run(driver, p, "halo", 8, cap).i() == 0


@pytest.mark.parametrize("which", ["q1_diffusion_3d", "elasticity_block"])
def test_amg_galerkin_hierarchy(driver, which):
    if which == "q1_diffusion_3d":
        p = si.q1_diffusion_pencil(9, 3, np.exp(np.random.default_rng(6).normal(0, .5, 1000)))
        block = 1
    else:
        p = _elastic(5, 2)
        block = 3
    sigma = 30.0 + 30.0j
    r = _run(driver, p, "amg", block, sigma.real, sigma.imag)
    assert r.i() == 1
    nl = r.i()
    assert nl >= 2
    levels = []
    for _ in range(nl):
        m = r.i()
        rp, ci, a, b = r.arr(np.int32), r.arr(np.int32), r.arr(np.float64), r.arr(np.float64)
        levels.append((sp.csr_matrix((a, ci, rp), shape=(m, m)),
                       sp.csr_matrix((b, ci, rp), shape=(m, m))))
    Ps = []
    for _ in range(nl - 1):
        nr, nc = r.i(), r.i()
        rp, ci, v = r.arr(np.int32), r.arr(np.int32), r.arr(np.float64)
        P = sp.csr_matrix((v, ci, rp), shape=(nr, nc))
        rn = r.i()
        rp, ci, v = r.arr(np.int32), r.arr(np.int32), r.arr(np.float64)
        R = sp.csr_matrix((v, ci, rp), shape=(rn, nr))
        assert abs(R - P.T).max() == 0.0
        Ps.append(P)
    rho = r.arr(np.float64)
    ncoarse = r.i()
    inv = r.arr(np.complex128).reshape(ncoarse, ncoarse)
    for l, P in enumerate(Ps):
        A0, B0 = levels[l]
        A1, B1 = levels[l + 1]
        if block > 1:
            assert P.shape[1] % block == 0
        for M0, M1 in ((A0, A1), (B0, B1)):
            G = (P.T @ M0 @ P).toarray()
            assert np.abs(M1.toarray() - G).max() <= 1e-12 * np.abs(G).max()
        D = sp.diags(1.0 / A0.diagonal())
        true_rho = np.max(np.abs(np.linalg.eigvals((D @ A0).toarray())))
        assert 0.9 * true_rho <= rho[l] <= true_rho * (1 + 1e-10)
    Ac, Bc = levels[-1]
    Mc = (Ac - sigma * Bc).toarray()
    assert np.abs(inv @ Mc - np.eye(ncoarse)).max() <= 1e-10


@pytest.mark.parametrize("which", ["q1_diffusion_3d", "elasticity_block"])
def test_fine_image_of_prolongator(driver, which):
    if which == "q1_diffusion_3d":
        p = si.q1_diffusion_pencil(9, 3, np.exp(np.random.default_rng(8).normal(0, .5, 1000)))
        block = 1
    else:
        p = _elastic(6, 3)  # large enough for a two-level hierarchy
        block = 3
    r = _run(driver, p, "image", block, 256, 32)
    assert r.i() == 1 and r.i() == 1
    nc = r.i()
    n = p.n
    prp, pci, pv0 = r.arr(np.int32), r.arr(np.int32), r.arr(np.float64)
    P = sp.csr_matrix((pv0, pci, prp), shape=(n, nc))
    rp, ci = r.arr(np.int32), r.arr(np.int32)
    ap, bp, pv = r.arr(np.float64), r.arr(np.float64), r.arr(np.float64)
    A = sp.csr_matrix((p.a, p.indices, p.indptr), shape=(n, n))
    B = sp.csr_matrix((p.b, p.indices, p.indptr), shape=(n, n))
    AP = sp.csr_matrix((ap, ci, rp), shape=(n, nc))
    BP = sp.csr_matrix((bp, ci, rp), shape=(n, nc))
    PP = sp.csr_matrix((pv, ci, rp), shape=(n, nc))
    for M, ref in ((AP, A @ P), (BP, B @ P), (PP, P)):
        d = (M - ref).toarray()
        assert np.abs(d).max() <= 1e-13 * max(np.abs(ref.toarray()).max(), 1.0)
    # the halo layout carries all three arrays entry for entry
    hmax = r.i()
    trow, hptr, halo = r.arr(np.int32), r.arr(np.int32), r.arr(np.int32)
    sptr, slen = r.arr(np.int32), r.arr(np.int32)
    lcol, ab, c3 = r.arr(np.uint16), r.arr(np.float64).reshape(-1, 2), r.arr(np.float64)
    assert np.all(np.diff(trow) <= 32) and hmax == np.max(np.diff(hptr))
    rows, cols, va, vb, vc = [], [], [], [], []
    for t in range(len(trow) - 1):
        h = halo[hptr[t]:hptr[t + 1]]
        assert np.all(h < nc)
        for rrow in range(trow[t], trow[t + 1]):
            s_, ln = rrow // 8, rrow % 8
            L = slen[rrow]
            k = _halo_entry(sptr[s_], np.arange(L), ln)
            rows += [rrow] * L
            cols += list(h[lcol[k]])
            va += list(ab[k, 0]); vb += list(ab[k, 1]); vc += list(c3[k])
    for vals, ref in ((va, AP), (vb, BP), (vc, PP)):
        M = sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))
        assert abs(M - ref).max() == 0.0
    # P's nonzeros again in slices of their own (same tiles, same halo rows):
    # every nonzero exactly once, padding zero, widths padded to 4, and emax
    # the most entries of one tile's pass
    pemax = r.i()
    psptr, plcol, pval = r.arr(np.int32), r.arr(np.uint16), r.arr(np.float64)
    assert len(psptr) == len(sptr) and np.all(np.diff(psptr) % 4 == 0)
    assert np.all(np.diff(psptr) <= np.diff(sptr))
    rows, cols, vals, seen = [], [], [], np.zeros(len(pval), bool)
    emax = 0
    for t in range(len(trow) - 1):
        h = halo[hptr[t]:hptr[t + 1]]
        s0, s1 = trow[t] // 8, (trow[t + 1] + 7) // 8
        emax = max(emax, (psptr[s1] - psptr[s0]) * 8)
        for rrow in range(trow[t], trow[t + 1]):
            s_, ln = rrow // 8, rrow % 8
            W = psptr[s_ + 1] - psptr[s_]
            k = _halo_entry(psptr[s_], np.arange(W), ln)
            seen[k] = True
            nz = pval[k] != 0.0
            rows += [rrow] * int(nz.sum())
            cols += list(h[plcol[k[nz]]])
            vals += list(pval[k[nz]])
    assert pemax == emax and np.all(pval[~seen] == 0.0)
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))
    assert M.nnz == PP.count_nonzero() and abs(M - PP).max() == 0.0


@pytest.mark.parametrize("which,R,U", [("q1_3d", 4, 4), ("elasticity", 4, 4), ("q1_2d_ragged", 3, 2)])
def test_row_group_format_reproduces_csr(driver, which, R, U):
    """The wave-uniform sweep's row groups: per group the distinct columns in
    increasing order with the mask of the rows that use them, every CSR entry
    exactly once with its (a, b), counts padded to multiples of U with
    coefficient-free entries, and 2 U look-ahead entries after the last group."""
    exe, d = driver
    if which == "q1_3d":
        p = si.q1_kron_pencil(7, 3)
    elif which == "elasticity":
        p = si.hex_elasticity_pencil(3, np.exp(np.random.default_rng(3).normal(0, .5, 27)))
    else:
        p = si.q1_diffusion_pencil(8, 2, np.ones(81))  # n = 64: 22 groups, the last of 1 row
    _write(p, d / "pu.bin")
    subprocess.run([exe, str(d / "pu.bin"), str(d / "ou.bin"), "ugroup", str(R), str(U)],
                   check=True)
    rd = _Reader(d / "ou.bin")
    ok = rd.i()
    gptr, ent, ab = rd.arr(np.int32), rd.arr(np.int32), rd.arr(np.float64)
    assert ok == 1
    ng = (p.n + R - 1) // R
    assert len(gptr) == ng + 1 and gptr[0] == 0
    assert len(ent) == gptr[-1] + 2 * U and len(ab) == 2 * R * len(ent)
    assert np.all(np.diff(gptr) % U == 0)
    col = ent & ((1 << 28) - 1)
    mask = (ent.astype(np.int64) >> 28) & 0xF
    ab = ab.reshape(-1, R, 2)
    A, B = p.A().tocsr(), p.B().tocsr()
    for g in range(ng):
        e0, e1 = gptr[g], gptr[g + 1]
        real = mask[e0:e1] != 0
        assert np.all(np.diff(col[e0:e1][real]) > 0)  # distinct, increasing
        assert np.all(ab[e0:e1][~real] == 0.0)
        for r in range(R):
            row = g * R + r
            hit = (mask[e0:e1] >> r) & 1 == 1
            if row >= p.n:
                assert not hit.any()
                continue
            lo, hi = A.indptr[row], A.indptr[row + 1]
            assert np.array_equal(col[e0:e1][hit], A.indices[lo:hi])
            assert np.array_equal(ab[e0:e1, r, 0][hit], A.data[lo:hi])
            assert np.array_equal(ab[e0:e1, r, 1][hit], B.data[lo:hi])
            assert np.all(ab[e0:e1, r][~hit] == 0.0)


def _read_amg(r):
    assert r.i() == 1
    nl = r.i()
    levels = []
    for _ in range(nl):
        m = r.i()
        rp, ci, a, b = r.arr(np.int32), r.arr(np.int32), r.arr(np.float64), r.arr(np.float64)
        levels.append((sp.csr_matrix((a, ci, rp), shape=(m, m)),
                       sp.csr_matrix((b, ci, rp), shape=(m, m))))
    Ps = []
    for _ in range(nl - 1):
        nr, nc = r.i(), r.i()
        rp, ci, v = r.arr(np.int32), r.arr(np.int32), r.arr(np.float64)
        Ps.append(sp.csr_matrix((v, ci, rp), shape=(nr, nc)))
        r.i()
        r.arr(np.int32), r.arr(np.int32), r.arr(np.float64)
    return levels, Ps


@pytest.mark.parametrize("coords", [True, False])
def test_amg_rigid_body_modes_in_the_coarse_space(driver, coords):
    """With node coordinates the first prolongator reproduces all six rigid-body
    modes of 3D elasticity (on an unclamped body they span the kernel of A, so
    P = (I - w D^-1 A) T keeps them exactly); with translations alone the three
    rotations are missing from the coarse space.  The Galerkin property holds
    at every level either way."""
    exe, d = driver
    ne = 6
    p = si.hex_elasticity_pencil(ne, np.exp(np.random.default_rng(2).normal(0, .3, ne ** 3)),
                                 clamp=False)
    args = ["amg", 3, 10.0, 10.0]
    if coords:
        p.coords.astype(np.float64).tofile(d / "xyz.bin")
        args.append(str(d / "xyz.bin"))
    levels, Ps = _read_amg(_run(driver, p, *args))
    assert len(Ps) >= 1
    for l, P in enumerate(Ps):
        for M0, M1 in zip(levels[l], levels[l + 1]):
            G = (P.T @ M0 @ P).toarray()
            assert np.abs(M1.toarray() - G).max() <= 1e-12 * np.abs(G).max()
    x = p.coords
    nn = x.shape[0]
    modes = np.zeros((nn, 3, 6))
    for c in range(3):
        modes[:, c, c] = 1.0
    modes[:, 1, 3], modes[:, 2, 3] = -x[:, 2], x[:, 1]
    modes[:, 0, 4], modes[:, 2, 4] = x[:, 2], -x[:, 0]
    modes[:, 0, 5], modes[:, 1, 5] = -x[:, 1], x[:, 0]
    modes = modes.reshape(3 * nn, 6)
    assert np.abs(p.A() @ modes).max() <= 1e-10 * np.abs(p.A()).max()  # the kernel of A
    P0 = Ps[0].toarray()
    c, *_ = np.linalg.lstsq(P0, modes, rcond=None)
    res = np.linalg.norm(P0 @ c - modes, axis=0) / np.linalg.norm(modes, axis=0)
    if coords:
        assert res.max() <= 1e-10
    else:
        assert res[:3].max() <= 1e-10 and res[3:].min() > 1e-3


@pytest.mark.parametrize("m,cmin,sizes", [
    (32, 0, [32768, 1331, 27]),    # off: plain aggregation down to <= 400
    (32, 64, [32768, 1331, 64]),   # 27 < 64: a raised threshold leaves 64
    (32, 128, [32768, 1331]),      # no halving aggregation leaves >= 128: 1331 is dense-solvable
    (16, 512, [4096, 310]),        # nothing reaches 512, 4096 is too large: the largest halving
    (16, 256, [4096, 310]),        # 216 < 256 on the fine level: a raised threshold leaves 310
])
def test_amg_coarse_min(driver, m, cmin, sizes):
    """options.amg_coarse_min: where the aggregation would leave fewer coarse dofs
    than the minimum, the strength threshold rises to the first value that leaves
    at least that many while halving the level; failing that a dense-solvable
    level becomes the coarsest, and a larger one takes the largest halving
    coarse space the thresholds gave.  Every level stays a Galerkin product and
    every coarsening at least halves."""
    p = si.q1_kron_pencil(m, 3)
    levels, Ps = _read_amg(_run(driver, p, "amg", 1, 10.0, 10.0, f"cmin={cmin}"))
    assert [L[0].shape[0] for L in levels] == sizes
    for l, P in enumerate(Ps):
        n0, n1 = P.shape
        assert 2 * n1 <= n0
        for M0, M1 in zip(levels[l], levels[l + 1]):
            G = (P.T @ M0 @ P).toarray()
            assert np.abs(M1.toarray() - G).max() <= 1e-12 * np.abs(G).max()
