"""Expected eigenvalues of the 64-pencil batch (uneven Q1 diffusion pencils).

For each pencil drawn by ``slrf_inputs.batched_pencils(64, seed=1004)`` the
oracle's shift-invert Lanczos gives the c + 1 smallest eigenvalues of Eq. (1);
the interval (0, gamma] is closed at the middle of the gap between the c-th and
(c + 1)-th.  Writes ``batch64_q1_diffusion.json`` beside this file.  Run from the
repository root: ``python tests/golden/make_batch64_q1_diffusion.py``.
"""

from __future__ import annotations

import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def one(i):
    import oracle
    import slrf_inputs as si

    d = si.batched_pencils(64, seed=1004, only=[i])[0]
    p = d["pencil"]
    c = d["count"]
    lam = oracle.eig.smallest_eigs(p.A(), p.B(), c + 1)
    return {"index": i, "n": int(p.n), "nnz": int(p.nnz), "dim": d["dim"], "m": d["m"],
            "count": c, "L": d["L"], "gamma": float(0.5 * (lam[c - 1] + lam[c])),
            "eigenvalues": [float(x) for x in lam[:c]],
            "next_eigenvalue": float(lam[c])}


def main():
    with ProcessPoolExecutor(max_workers=int(os.environ.get("NPROC", "6"))) as ex:
        rows = list(ex.map(one, range(64)))
    out = {"source": "oracle.eig.smallest_eigs on slrf_inputs.batched_pencils(64, seed=1004)",
           "pencils": rows}
    with open(os.path.join(HERE, "batch64_q1_diffusion.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
