"""Expected eigenvalues of the differentiation workload (clamped hex elasticity,
48^3 elements, Young's modulus lognormal(0, 0.5) from seed 1003, n = 345,744).

The oracle's shift-invert Lanczos gives the 201 smallest eigenvalues of Eq. (1);
the interval (0, gamma] closes at the middle of the gap after the 200th.  Also
records the 20 elements (seed 1006) on which the gradient is sampled.  Writes
``elasticity48.json`` beside this file; run from the repository root:
``python tests/golden/make_elasticity48.py``.
"""

from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import slrf_inputs as si  # noqa: E402


def main():
    c = si.config_elasticity(48, 0.5, 1003, 200, 300)
    p = c["pencil"]
    k = c["count"]
    lam = oracle.eig.smallest_eigs(p.A(), p.B(), k + 1)
    elems = np.sort(np.random.default_rng(1006).choice(48 ** 3, 20, replace=False))
    out = {"source": "oracle.eig.smallest_eigs on slrf_inputs.config_elasticity(48, 0.5, 1003)",
           "n": int(p.n), "nnz": int(p.nnz), "count": k, "L": c["L"],
           "gamma": float(0.5 * (lam[k - 1] + lam[k])),
           "eigenvalues": [float(x) for x in lam[:k]], "next_eigenvalue": float(lam[k]),
           "sample_elements": [int(e) for e in elems]}
    with open(os.path.join(HERE, "elasticity48.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
