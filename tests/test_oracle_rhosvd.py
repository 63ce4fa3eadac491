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


def _factors(s):
    t, a = quadrature.literal_table("newton", s.R)
    U = rhosvd.side_matrices(s.b, s.n, s.pos, t[:s.R_l])
    xi = rhosvd.canonical_weights(s.q, a[:s.R_l])
    return t, a, U, xi, rhosvd.gram_weights(xi)


def test_eigh_basis_spans_the_svd_basis():
    """The Gram route gives the singular subspace of the SVD route: equal
    projectors up to the rounding of the squared spectrum, equal leading
    singular values, the same rank rule."""
    s = _tiny(n=40, N=15)
    t, a, U, xi, w = _factors(s)
    for l in range(3):
        Qs, sig_s, r_s = rhosvd.mode_basis(U[l], w, 1e-6, s.n)
        Qe, sig_e, r_e = rhosvd.mode_basis_eigh(rhosvd.weighted_gram(U[l], w), 1e-6, s.n)
        assert r_s == r_e
        assert np.max(np.abs(sig_s[:4] - sig_e[:4]) / sig_s[:4]) <= 1e-12
        # a gap well above the truncation: leading 8 columns equal up to rounding
        assert np.max(np.abs(Qs[:, :8] - Qe[:, :8])) <= 1e-8
        P_s, P_e = Qs @ Qs.T, Qe @ Qe.T
        # projectors differ only in directions at the threshold (sigma ~ 1e-6 sigma_1)
        A = U[l] * np.sqrt(w)[None, :]
        assert np.linalg.norm((P_s - P_e) @ A, 2) <= 1e-7 * sig_s[0]


def test_chunked_core_equals_core():
    s = _tiny(n=24, N=14)
    t, a, U, xi, w = _factors(s)
    Qs = [rhosvd.mode_basis(U[l], w, 1e-6, s.n)[0] for l in range(3)]
    Ut = [rhosvd.project(Qs[l], U[l]) for l in range(3)]
    b1 = rhosvd.core(Ut, xi)
    for chunk in (1, 7, 64, 10 ** 6):
        b2 = rhosvd.core_chunked(Ut, xi, chunk)
        assert np.max(np.abs(b1 - b2)) <= 1e-13 * np.max(np.abs(b1))


def test_projected_subgrid_equals_tucker_and_full_rank_canonical():
    """The projected canonical sum on an index set equals the Tucker tensor
    there; with full ranks (Q orthogonal, Q Q^T = I) it is the canonical
    long-range sum itself."""
    s = _tiny(n=20, N=9)
    t, a, U, xi, w = _factors(s)
    rng = np.random.default_rng(3)
    I = [np.sort(rng.choice(s.n, size=m, replace=False)) for m in (7, 5, 9)]
    for ranks in ([9, 7, 8], [s.n] * 3):
        Qs = [rhosvd.mode_basis(U[l], w, 0.0, s.n, ranks[l])[0] for l in range(3)]
        Ut = [rhosvd.project(Qs[l], U[l]) for l in range(3)]
        full = rhosvd.tucker_full(rhosvd.core(Ut, xi), Qs)[np.ix_(*I)]
        got = rhosvd.tucker_subgrid_projected(Qs, Ut, xi, *I, chunk=17)
        assert np.max(np.abs(got - full)) <= 1e-13 * np.max(np.abs(full))
        W = rhosvd.projected_side_matrices(Qs, Ut)
        got_w = rhosvd.tucker_subgrid_projected(None, None, xi, *I, chunk=17, W=W)
        assert np.max(np.abs(got_w - full)) <= 1e-13 * np.max(np.abs(full))
    C = rhosvd.canonical_full(U, xi)[np.ix_(*I)]
    assert np.max(np.abs(got - C)) <= 1e-12 * np.max(np.abs(C))


def test_short_range_subgrid_equals_dense_and_pointwise():
    s = _tiny(n=24, N=12, n_s=7)
    t, a = quadrature.literal_table("newton", s.R)
    dense = canonical.short_range_grid(s.b, s.n, s.pos, s.q, t, a, s.R_l, s.n_s)
    rng = np.random.default_rng(4)
    I = [np.sort(rng.choice(s.n, size=m, replace=False)) for m in (10, 6, 13)]
    sub = canonical.short_range_subgrid(*I, s.b, s.n, s.pos, s.q, t, a, s.R_l, s.n_s)
    assert np.array_equal(sub, dense[np.ix_(*I)])
    ijk = np.stack(np.meshgrid(*I, indexing="ij"), -1).reshape(-1, 3)
    pw = canonical.short_range_at(ijk, s.b, s.n, s.pos, s.q, t, a, s.R_l, s.n_s)
    assert np.max(np.abs(pw - sub.ravel())) <= 1e-15 * np.max(np.abs(pw)) * 10
