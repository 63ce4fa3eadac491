"""The uniform n x n x n grid on Omega = [-b, b]^3 with h = 2b/n, n even
(section 2.2).  Tensor entries are collocated at cell centres (section 3.2:
the long-range sum is evaluated at the centres of the grid cells)."""
from __future__ import annotations

import numpy as np


def spacing(b: float, n: int) -> float:
    return 2.0 * b / n


def cell_centres(b: float, n: int) -> np.ndarray:
    """x_i = -b + (i + 1/2) h, i = 0..n-1 (mirror symmetric about 0)."""
    return -b + (np.arange(n, dtype=np.float64) + 0.5) * spacing(b, n)


def cell_of(x, b: float, n: int):
    """Index of the cell containing x: floor((x + b)/h), clamped to [0, n-1]
    (ties go to the upper cell)."""
    j = np.floor((np.asarray(x, dtype=np.float64) + b) / spacing(b, n)).astype(np.int64)
    return np.clip(j, 0, n - 1)


def flat_to_ijk(flat, n: int):
    flat = np.asarray(flat, dtype=np.int64)
    return np.stack([flat // (n * n), (flat // n) % n, flat % n], axis=-1)
