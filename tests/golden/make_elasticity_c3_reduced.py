"""Expected eigenvalues of the large elasticity workload's generator at reduced
meshes (clamped trilinear-hex elasticity, Young's modulus lognormal(0, 0.5) from
seed 1003, nu = 0.3: the 48^3 workload's recipe on 16^3 and 24^3 elements).

The oracle's shift-invert Lanczos gives the 201 smallest eigenvalues of
Eq. (1); the interval (0, gamma] closes at the middle of the gap after the
200th.  Writes ``elasticity_c3_<ne>.json`` beside this file; run from the
repository root: ``python tests/golden/make_elasticity_c3_reduced.py [ne ...]``.
"""

from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import slrf_inputs as si  # noqa: E402


def main(sizes):
    for ne in sizes:
        c = si.config_elasticity(ne, 0.5, 1003, 200, 300)
        p = c["pencil"]
        k = c["count"]
        lam = oracle.eig.smallest_eigs(p.A(), p.B(), k + 1)
        out = {"source": f"oracle.eig.smallest_eigs on slrf_inputs.config_elasticity({ne}, 0.5, "
                         "1003, 200, 300)",
               "ne": ne, "n": int(p.n), "nnz": int(p.nnz), "count": k, "L": c["L"],
               "gamma": float(0.5 * (lam[k - 1] + lam[k])),
               "eigenvalues": [float(x) for x in lam[:k]], "next_eigenvalue": float(lam[k])}
        with open(os.path.join(HERE, f"elasticity_c3_{ne}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(ne, p.n, out["gamma"], flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [16, 24])
