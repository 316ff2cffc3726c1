"""Expected eigenvalues of the differentiation workload (clamped hex elasticity,
32^3 elements, Young's modulus lognormal(0, 0.3) from seed 1005, n = 104,544).

The oracle's shift-invert Lanczos gives the 51 smallest eigenpairs of Eq. (1);
the interval (0, gamma] closes at the middle of the gap after the 50th.  Also
records the 20 elements (seed 1006) on which the gradient is sampled and the
oracle's gradient of the loss sum_i lambda_i there, from its own B-orthonormal
eigenvectors (the sum over a whole invariant subspace does not depend on the
basis chosen inside it).  Writes
``elasticity32.json`` beside this file; run from the repository root:
``python tests/golden/make_elasticity32.py``.
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
    c = si.config_elasticity(32, 0.3, 1005, 50, 75)
    p = c["pencil"]
    k = c["count"]
    lam, X = oracle.eig.smallest_eigpairs(p.A(), p.B(), k + 1)
    elems = np.sort(np.random.default_rng(1006).choice(32 ** 3, 20, replace=False))
    grad = oracle.grad.eig_grad(p.elem_dofs[elems], p.ke_ref, None, X[:, :k], lam[:k],
                                np.ones(k))
    out = {"source": "oracle.eig.smallest_eigpairs on slrf_inputs.config_elasticity(32, 0.3, 1005)",
           "n": int(p.n), "nnz": int(p.nnz), "count": k, "L": c["L"],
           "gamma": float(0.5 * (lam[k - 1] + lam[k])),
           "eigenvalues": [float(x) for x in lam[:k]], "next_eigenvalue": float(lam[k]),
           "sample_elements": [int(e) for e in elems],
           "grad_sum_lambda_samples": [float(x) for x in grad]}
    with open(os.path.join(HERE, "elasticity32.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
