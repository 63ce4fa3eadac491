"""Discrete gradient of an RS tensor on the whole grid (section 4.3, eq
Gradients_Tens).  TEST INFRASTRUCTURE ONLY (see the package header).

The paper applies a univariate finite-difference operator nabla_l along each
axis to the long-range part (which, being separable, only changes one factor)
and locally to every short-range term.  Both are linear, so the discrete
gradient of the whole tensor A = A_l + A_s is the same operator applied to the
full grid.  The paper allows backward or central differences; the reading
taken here is central differences inside and one-sided (forward at the first
cell, backward at the last) at the two ends of each axis, spacing h.
"""
from __future__ import annotations

import numpy as np


def fd_axis(A, h: float, axis: int) -> np.ndarray:
    """nabla_axis A: (A[i+1] - A[i-1]) / 2h inside, (A[1] - A[0]) / h and
    (A[n-1] - A[n-2]) / h at the ends, along `axis`."""
    A = np.moveaxis(np.asarray(A, dtype=np.float64), axis, 0)
    n = A.shape[0]
    if n < 2:
        raise ValueError("need at least two cells along the axis")
    D = np.empty_like(A)
    D[1:n - 1] = (A[2:] - A[:n - 2]) / (2.0 * h)
    D[0] = (A[1] - A[0]) / h
    D[n - 1] = (A[n - 1] - A[n - 2]) / h
    return np.moveaxis(D, 0, axis)


def gradient_grid(T, axis: int) -> np.ndarray:
    """The axis component of the discrete gradient of the RS-Tucker tensor
    T (oracle.rs.RSTucker) at every cell centre."""
    return fd_axis(T.full_grid(), T.h, axis)
