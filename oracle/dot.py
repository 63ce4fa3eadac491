"""Scalar product of two RS tensors on the same grid (section 3.4, item (d)).
TEST INFRASTRUCTURE ONLY (see the package header).

The scalar product is the Euclidean one of the grid tensors,
<A, B> = sum_i A(i) B(i) over all n^3 cells; the oracle writes that
definition out on the full grids (small n only).  The paper reduces it to
cross products of the elementary canonical tensors; the HIP path keeps the
long-range parts in Tucker form (see long_long_tucker below, used only as an
independent pin) and corrects on the cells the short-range windows touch.
"""
from __future__ import annotations

import numpy as np


def scalar_product(TA, TB) -> float:
    """sum_i A(i) B(i) of two RS tensors (oracle.rs.RSTucker) on the same grid."""
    if TA.n != TB.n or TA.b != TB.b:
        raise ValueError("the tensors must live on the same grid")
    return float(np.sum(TA.full_grid() * TB.full_grid()))


def long_long_tucker(TA, TB) -> float:
    """<A_l, B_l> from the Tucker factors alone: with M_l = V_l^A^T V_l^B,
    sum_{abc} sum_{a'b'c'} beta_A[abc] beta_B[a'b'c'] M_1[a,a'] M_2[b,b'] M_3[c,c']."""
    M = [TA.Q[l].T @ TB.Q[l] for l in range(3)]
    X = np.einsum("abc,ax,by,cz->xyz", TA.beta, M[0], M[1], M[2], optimize=True)
    return float(np.sum(X * TB.beta))
