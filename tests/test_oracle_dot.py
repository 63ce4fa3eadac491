"""Pins for oracle.dot (section 3.4, scalar products of RS tensors)."""
import numpy as np
import pytest

import workloads
from oracle import dot, rs


def _pair(seed_a=61, seed_b=62):
    a = workloads.tiny_system(seed_a, 9, 4.0, 24, 16, 6, 5, min_sep=0.4)
    b = workloads.tiny_system(seed_b, 7, 4.0, 24, 20, 8, 7, min_sep=0.4)
    return rs.assemble_system(a), rs.assemble_system(b)


def test_long_long_by_tucker_factors_equals_grid_dot():
    TA, TB = _pair()
    ref = float(np.sum(TA.long_grid() * TB.long_grid()))
    assert abs(dot.long_long_tucker(TA, TB) - ref) <= 1e-12 * abs(ref)


def test_symmetric_and_norm():
    TA, TB = _pair()
    ab, ba = dot.scalar_product(TA, TB), dot.scalar_product(TB, TA)
    assert abs(ab - ba) <= 1e-14 * abs(ab)
    aa = dot.scalar_product(TA, TA)
    assert aa > 0 and abs(aa - np.linalg.norm(TA.full_grid()) ** 2) <= 1e-12 * aa


def test_short_parts_vanish_off_their_windows():
    # outside every window of a tensor its grid equals its long-range part,
    # which is what lets the in-format product correct only on those cells
    TA, _ = _pair()
    from oracle import canonical
    lo, hi = canonical.window_bounds(TA.pos, TA.b, TA.n, TA.n_s)
    mask = np.zeros((TA.n,) * 3, dtype=bool)
    for nu in range(TA.pos.shape[0]):
        mask[lo[nu, 0]:hi[nu, 0] + 1, lo[nu, 1]:hi[nu, 1] + 1, lo[nu, 2]:hi[nu, 2] + 1] = True
    diff = TA.full_grid() - TA.long_grid()
    assert np.max(np.abs(diff[~mask])) == 0.0
    assert np.max(np.abs(diff[mask])) > 0.0


def test_mismatched_grids_are_rejected():
    TA, _ = _pair()
    c = workloads.tiny_system(63, 5, 5.0, 24, 16, 6, 5, min_sep=0.4)
    with pytest.raises(ValueError):
        dot.scalar_product(TA, rs.assemble_system(c))
