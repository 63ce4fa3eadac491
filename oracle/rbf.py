"""Matrix-vector product of the RBF interpolation matrix in RS form
(section 4.1, case (A): the sample points are the n^3 grid points).
TEST INFRASTRUCTURE ONLY (see the package header).

The matrix A[i, j] = p(|x_i - x_j|) of a radial basis function p collocated
on the grid is replaced by the RS sum of the reference tensor's quadrature:
    A[i, j] = sum_k a_k prod_l exp(-t_k^2 ((i_l - j_l) h)^2) * m_k(i - j),
with m_k = 1 for the long-range terms k < R_l and, for the short-range terms
k >= R_l, the window indicator |i_l - j_l| <= w = (n_s - 1)/2 in every mode
(the localised part of the split, section 2.3).  The oracle writes the
product y = A c out entry by entry on small grids.
"""
from __future__ import annotations

import numpy as np

from . import grid as _grid


def rbf_matrix(b: float, n: int, t, a, R_l: int, n_s: int) -> np.ndarray:
    """The n^3 x n^3 matrix A above (small n only), C-order cell index."""
    h = _grid.spacing(b, n)
    idx = np.indices((n, n, n)).reshape(3, -1).T          # (n^3, 3)
    d = idx[:, None, :] - idx[None, :, :]                 # (n^3, n^3, 3)
    w = (n_s - 1) // 2
    inside = np.all(np.abs(d) <= w, axis=2)
    r2 = np.sum((d * h) ** 2, axis=2)
    A = np.zeros((n ** 3, n ** 3))
    for k in range(len(t)):
        term = a[k] * np.exp(-t[k] ** 2 * r2)
        A += term if k < R_l else term * inside
    return A


def rbf_matvec(b: float, n: int, t, a, R_l: int, n_s: int, c) -> np.ndarray:
    """y = A c for c an n x n x n array (returned in the same shape)."""
    A = rbf_matrix(b, n, t, a, R_l, n_s)
    return (A @ np.asarray(c, dtype=np.float64).ravel()).reshape(n, n, n)
