"""Pins for oracle.canonical: canonical sums, direct sums, CCT windows."""
import math

import numpy as np
import pytest

import workloads
from oracle import canonical, grid, quadrature
from tests.test_oracle_quadrature import poisson_closed_form


def _system(seed=11, N=12, b=4.0, n=24, R=20, R_l=8, n_s=7):
    return workloads.tiny_system(seed, N, b, n, R, R_l, n_s, min_sep=0.5)


def test_radial_equals_separable():
    s = _system()
    t, a = quadrature.literal_table("newton", s.R)
    rng = np.random.default_rng(0)
    pts = rng.uniform(-s.b, s.b, size=(200, 3))
    r1 = canonical.canonical_potential_radial(pts, s.pos, s.q, t, a)
    r2 = canonical.canonical_potential_separable(pts, s.pos, s.q, t, a)
    assert np.max(np.abs(r1 - r2)) <= 1e-13 * np.max(np.abs(r1))


def test_canonical_minus_direct_is_quadrature_error():
    """P_can - P_dir = sum_nu z_nu e(|y - x_nu|), e from the Poisson closed
    form of the literal rule (independent of the table)."""
    s = _system(N=6)
    t, a = quadrature.literal_table("newton", s.R)
    h, M = quadrature.step_size(s.R), s.R - 1
    rng = np.random.default_rng(1)
    pts = rng.uniform(-s.b, s.b, size=(25, 3))
    diff = canonical.canonical_potential_radial(pts, s.pos, s.q, t, a) - \
        canonical.direct_potential(pts, s.pos, s.q)
    ref = np.zeros(len(pts))
    for nu in range(s.N):
        for m, y in enumerate(pts):
            r = float(np.linalg.norm(y - s.pos[nu]))
            ref[m] += s.q[nu] * (poisson_closed_form(r, h, M) - 1.0 / r)
    scale = np.sum(np.abs(s.q)) * np.max(a.sum())
    assert np.max(np.abs(diff - ref)) <= 1e-13 * scale


def test_window_equals_short_sum_inside_and_bounded_outside():
    s = _system(N=5, n=32, n_s=9)
    t, a = quadrature.literal_table("newton", s.R)
    G = canonical.short_range_grid(s.b, s.n, s.pos, s.q, t, a, s.R_l, s.n_s)
    x = grid.cell_centres(s.b, s.n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    full = canonical.canonical_potential_radial(pts, s.pos, s.q, t, a, ks=range(s.R_l, s.R)).reshape(G.shape)
    lo, hi = canonical.window_bounds(s.pos, s.b, s.n, s.n_s)
    inside_any = np.zeros(G.shape, bool)
    for nu in range(s.N):
        sl = tuple(slice(lo[nu, l], hi[nu, l] + 1) for l in range(3))
        inside_any[sl] = True
    # outside every window the windowed sum is 0 and the true short sum is below the remainder bound
    assert np.all(G[~inside_any] == 0.0)
    w = (s.n_s - 1) // 2
    bound = np.sum(np.abs(s.q)) * quadrature.kernel_sum(np.array([(w + 0.5) * s.h]), t, a, range(s.R_l, s.R))[0]
    assert np.max(np.abs(full - G)) <= bound * (1 + 1e-12)


def test_short_range_at_matches_dense_grid():
    s = _system(N=7, n=20, n_s=5)
    t, a = quadrature.literal_table("newton", s.R)
    G = canonical.short_range_grid(s.b, s.n, s.pos, s.q, t, a, s.R_l, s.n_s)
    idx = grid.flat_to_ijk(np.arange(s.n ** 3), s.n)
    vals = canonical.short_range_at(idx, s.b, s.n, s.pos, s.q, t, a, s.R_l, s.n_s)
    assert np.max(np.abs(vals - G.ravel())) <= 1e-14 * np.max(np.abs(G))


def test_cct_block_orthogonality_and_norm_identity():
    """Proposition Cum_CP_Feature (B): windows that do not intersect give
    orthogonal components; then ||U||^2 = sum c_nu^2 ||U_nu||^2 (property (C),
    with the square the paper's line omits)."""
    b, n, R, R_l, n_s = 8.0, 48, 20, 8, 7
    pos = np.array([[-5.0, -5.0, -5.0], [0.1, 0.2, 0.3], [5.0, 4.0, -3.0]])
    q = np.array([0.7, -1.3, 0.4])
    t, a = quadrature.literal_table("newton", R)
    comps = [canonical.short_range_grid(b, n, pos[i:i + 1], np.ones(1), t, a, R_l, n_s) for i in range(3)]
    for i in range(3):
        for j in range(i + 1, 3):
            assert float(np.sum(comps[i] * comps[j])) == 0.0
    U = sum(q[i] * comps[i] for i in range(3))
    assert abs(np.sum(U * U) - sum(q[i] ** 2 * np.sum(comps[i] ** 2) for i in range(3))) < 1e-12 * np.sum(U * U)


def test_invariants_antisymmetry_permutation_axis_swap():
    s = _system(N=6, n=16, n_s=5)
    t, a = quadrature.literal_table("newton", s.R)
    G = canonical.short_range_grid(s.b, s.n, s.pos, s.q, t, a, s.R_l, s.n_s)
    Gm = canonical.short_range_grid(s.b, s.n, s.pos, -s.q, t, a, s.R_l, s.n_s)
    assert np.array_equal(Gm, -G)
    perm = np.random.default_rng(3).permutation(s.N)
    Gp = canonical.short_range_grid(s.b, s.n, s.pos[perm], s.q[perm], t, a, s.R_l, s.n_s)
    assert np.max(np.abs(Gp - G)) <= 1e-14 * np.max(np.abs(G))
    Gs = canonical.short_range_grid(s.b, s.n, s.pos[:, [1, 0, 2]], s.q, t, a, s.R_l, s.n_s)
    assert np.max(np.abs(Gs - G.transpose(1, 0, 2))) <= 1e-14 * np.max(np.abs(G))
