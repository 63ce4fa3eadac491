"""Pins for oracle.rhosvd and oracle.rs (section 3.2, Appendix)."""
import numpy as np
import pytest

import workloads
from oracle import canonical, grid, quadrature, rhosvd, rs


def _tiny(seed=21, N=10, n=20, R=20, R_l=8, n_s=5, b=5.0):
    return workloads.tiny_system(seed, N, b, n, R, R_l, n_s, min_sep=0.6)


def test_gram_two_ways():
    s = _tiny(n=40, N=15)
    t, a = quadrature.literal_table("newton", s.R)
    U = rhosvd.side_matrix(s.b, s.n, s.pos[:, 1], t[:s.R_l])
    xi = rhosvd.canonical_weights(s.q, a[:s.R_l])
    w = rhosvd.gram_weights(xi)
    G1 = rhosvd.weighted_gram(U, w)
    G2 = rhosvd.weighted_gram_gaussian_product(s.b, s.n, s.pos[:, 1], t[:s.R_l], w)
    assert np.max(np.abs(G1 - G2)) <= 1e-14 * np.max(np.abs(G1)) * 10
    assert np.max(np.abs(G1 - G1.T)) <= 1e-15 * np.max(np.abs(G1)) * 10
    assert abs(np.trace(G1) - np.sum(w * np.sum(U * U, axis=0))) <= 1e-13 * np.trace(G1)
    ev = np.linalg.eigvalsh(G1)
    assert ev.min() >= -1e-13 * ev.max()


def test_svd_singular_values_are_sqrt_gram_eigenvalues():
    s = _tiny(n=32, N=12)
    t, a = quadrature.literal_table("newton", s.R)
    U = rhosvd.side_matrix(s.b, s.n, s.pos[:, 0], t[:s.R_l])
    w = rhosvd.gram_weights(rhosvd.canonical_weights(s.q, a[:s.R_l]))
    _, sig, _ = rhosvd.mode_basis(U, w, 1e-6, s.n)
    ev = np.sort(np.linalg.eigvalsh(rhosvd.weighted_gram(U, w)))[::-1]
    k = int(np.sum(sig > 1e-6 * sig[0]))
    # Gram eigenvalues carry an absolute error of order u * lambda_1
    assert np.max(np.abs(sig[:k] ** 2 - ev[:k])) <= 1e-13 * ev[0]
    assert np.max(np.abs(sig[:4] ** 2 - ev[:4]) / ev[:4]) < 1e-13


def test_full_rank_tucker_reproduces_canonical_long_range_sum():
    s = _tiny()
    t, a = quadrature.literal_table("newton", s.R)
    T = rs.assemble(s.b, s.n, s.pos, s.q, t, a, s.R_l, s.n_s, eps=0.0, fixed_ranks=[s.n] * 3)
    U = rhosvd.side_matrices(s.b, s.n, s.pos, t[:s.R_l])
    xi = rhosvd.canonical_weights(s.q, a[:s.R_l])
    C = rhosvd.canonical_full(U, xi)
    assert np.max(np.abs(T.long_grid() - C)) <= 1e-12 * np.max(np.abs(C))
    # and the canonical tensor equals the separable long-range sum at the cell centres
    x = grid.cell_centres(s.b, s.n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    ref = canonical.canonical_potential_radial(pts, s.pos, s.q, t, a, ks=range(s.R_l)).reshape(C.shape)
    assert np.max(np.abs(ref - C)) <= 1e-13 * np.max(np.abs(C))


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
def test_truncation_error_between_hosvd_lower_bound_and_rhosvd_upper_bound(eps):
    s = _tiny(n=24, N=14)
    t, a = quadrature.literal_table("newton", s.R)
    T = rs.assemble(s.b, s.n, s.pos, s.q, t, a, s.R_l, s.n_s, eps=eps)
    U = rhosvd.side_matrices(s.b, s.n, s.pos, t[:s.R_l])
    xi = rhosvd.canonical_weights(s.q, a[:s.R_l])
    C = rhosvd.canonical_full(U, xi)
    err = np.linalg.norm(T.long_grid() - C)
    # lower bound: any rank-(r1,r2,r3) Tucker tensor leaves at least the tail of each unfolding
    lower = max(np.sqrt(np.sum(rhosvd.unfolding_singular_values(C, l)[T.ranks[l]:] ** 2)) for l in range(3))
    # upper bound (Lemma RHOSVD_CCT with an explicit constant): with A_l = U_l diag(|xi|^(1/3)),
    # ||C - C_r|| <= sum_l tail_l(sigma(A_l)) * sqrt(sum_j prod_{l' != l} ||a_j^{l'}||^2)
    w3 = np.abs(xi) ** (1.0 / 3.0)
    norms = [np.sum((U[l] * w3) ** 2, axis=0) for l in range(3)]
    upper = 0.0
    for l in range(3):
        tail = np.sqrt(np.sum(T.sigma[l][T.ranks[l]:] ** 2))
        other = np.prod([norms[m] for m in range(3) if m != l], axis=0)
        upper += tail * np.sqrt(np.sum(other))
    assert lower <= err * (1 + 1e-9) + 1e-14
    assert err <= upper * (1 + 1e-9) + 1e-14


def test_antisymmetry_of_basis_and_core():
    s = _tiny()
    t, a = quadrature.literal_table("newton", s.R)
    T1 = rs.assemble(s.b, s.n, s.pos, s.q, t, a, s.R_l, s.n_s, eps=1e-6)
    T2 = rs.assemble(s.b, s.n, s.pos, -s.q, t, a, s.R_l, s.n_s, eps=1e-6)
    assert T1.ranks == T2.ranks
    for l in range(3):
        assert np.array_equal(T1.Q[l], T2.Q[l])
    assert np.array_equal(T1.beta, -T2.beta)


def test_rank_saturates_in_N_and_is_flat_in_n():
    """Theorem Rank_LongRange and Remark RankTuck_N0: at fixed box size the
    Tucker rank of the long-range sum grows at most logarithmically in N and
    does not grow with the grid size n."""
    t, a = quadrature.literal_table("newton", 20)
    rng = np.random.default_rng(5)
    ranks = {}
    pos_all = workloads._min_sep_uniform(rng, 256, -6.0, 6.0, 0.8)
    q_all = rng.uniform(-1, 1, 256)
    for N in [16, 64, 256]:
        U = rhosvd.side_matrix(10.0, 128, pos_all[:N, 0], t[:8])
        w = rhosvd.gram_weights(rhosvd.canonical_weights(q_all[:N], a[:8]))
        ranks[N] = rhosvd.mode_basis(U, w, 1e-6, 128)[2]
    assert ranks[256] - ranks[64] <= 0.1 * ranks[64]
    assert ranks[64] >= ranks[16]
    rn = {}
    for n in [128, 256]:
        U = rhosvd.side_matrix(10.0, n, pos_all[:64, 0], t[:8])
        w = rhosvd.gram_weights(rhosvd.canonical_weights(q_all[:64], a[:8]))
        rn[n] = rhosvd.mode_basis(U, w, 1e-6, n)[2]
    assert abs(rn[256] - rn[128]) <= 0.1 * rn[128]
    # the full canonical sum (all terms, short ones included) has rank growing with N
    full = {}
    for N in [16, 64]:
        U = rhosvd.side_matrix(10.0, 128, pos_all[:N, 0], t)
        w = rhosvd.gram_weights(rhosvd.canonical_weights(q_all[:N], a))
        full[N] = rhosvd.mode_basis(U, w, 1e-6, 128)[2]
    assert full[64] > ranks[64]
