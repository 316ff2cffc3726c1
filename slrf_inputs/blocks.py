"""Seeded dense start blocks V_1 (Algorithm 1 and 2 take L random columns)."""

from __future__ import annotations

import numpy as np


def seeded_rng(seed: int) -> np.random.Generator:
    """The one generator used for every seeded draw (PCG64 via default_rng)."""
    return np.random.default_rng(int(seed))


def start_block(n: int, L: int, seed: int) -> np.ndarray:
    """V_1 with i.i.d. N(0, 1) entries, shape (n, L), column-major (Fortran) FP64."""
    rng = seeded_rng(seed)
    v = rng.standard_normal((L, n))  # draw column by column
    return np.asfortranarray(v.T)
