"""Pins for oracle.als (Appendix, C2T steps (III)-(V), eq alg2)."""
import numpy as np

import workloads
from oracle import als, quadrature, rhosvd, rs


def _setup(seed=81, N=12, n=24, ranks=(6, 5, 7)):
    s = workloads.tiny_system(seed, N, 4.0, n, 16, 7, 5, min_sep=0.4)
    t, a = quadrature.literal_table(s.kernel, s.R, s.lam)
    U = rhosvd.side_matrices(s.b, s.n, s.pos, t[:s.R_l])
    xi = rhosvd.canonical_weights(s.q, a[:s.R_l])
    w = rhosvd.gram_weights(xi)
    Q0 = [rhosvd.mode_basis(U[l], w, 0.0, n, ranks[l])[0] for l in range(3)]
    return U, xi, Q0


def test_one_sweep_is_dense_hooi():
    # textbook higher-order orthogonal iteration on the dense canonical tensor:
    # the mode-l unfolding projected on the other modes' bases, its dominant
    # left singular vectors (a library SVD of the full tensor)
    U, xi, Q0 = _setup()
    A = rhosvd.canonical_full(U, xi)
    Q, beta, _ = als.refine(U, xi, Q0, 1)
    Qd = [q.copy() for q in Q0]
    for l in range(3):
        m, p = [k for k in range(3) if k != l]
        Y = np.moveaxis(A, l, 0)            # (n_l, n_m, n_p) with m < p kept in order
        Y = np.einsum("ijk,jb,kc->ibc", Y, Qd[m], Qd[p]).reshape(A.shape[l], -1)
        Z = np.linalg.svd(Y, full_matrices=False)[0]
        Qd[l] = rhosvd.canonical_signs(Z[:, :Q0[l].shape[1]])
    for l in range(3):
        assert np.max(np.abs(Q[l] - Qd[l])) < 1e-9
    beta_d = np.einsum("ijk,ia,jb,kc->abc", A, Qd[0], Qd[1], Qd[2])
    assert np.max(np.abs(beta - beta_d)) < 1e-9 * np.max(np.abs(beta_d))


def test_core_norm_grows_and_error_falls():
    # each update maximises ||beta|| over one mode's basis, and for orthonormal
    # bases ||A - Tucker||^2 = ||A||^2 - ||beta||^2
    U, xi, Q0 = _setup(seed=82)
    A = rhosvd.canonical_full(U, xi)
    Q, beta, norms = als.refine(U, xi, Q0, 3)
    assert all(norms[i + 1] >= norms[i] * (1 - 1e-13) for i in range(3))
    e0 = np.linalg.norm(A - rhosvd.tucker_full(rhosvd.core([rhosvd.project(Q0[l], U[l]) for l in range(3)], xi), Q0))
    e3 = np.linalg.norm(A - rhosvd.tucker_full(beta, Q))
    assert e3 < e0
    assert abs(e3 ** 2 - (np.linalg.norm(A) ** 2 - norms[-1] ** 2)) <= 1e-9 * np.linalg.norm(A) ** 2
    for l in range(3):
        assert np.max(np.abs(Q[l].T @ Q[l] - np.eye(Q[l].shape[1]))) < 1e-12


def test_full_rank_is_exact():
    n = 16
    U, xi, Q0 = _setup(seed=83, n=n, ranks=(n, n, n))
    Q, beta, _ = als.refine(U, xi, Q0, 1)
    A = rhosvd.canonical_full(U, xi)
    assert np.max(np.abs(rhosvd.tucker_full(beta, Q) - A)) < 1e-11 * np.max(np.abs(A))


def test_partial_image_layout():
    # the unfolding's column (b, c) with c fastest; mode 1's partners are 0, 2
    U, xi, Q0 = _setup(seed=84)
    Ut = [rhosvd.project(Q0[l], U[l]) for l in range(3)]
    M = als.partial_image(U, xi, Ut, 1)
    r0, r2 = Q0[0].shape[1], Q0[2].shape[1]
    i, b, c = 5, 2, 3
    want = sum(U[1][i, j] * xi[j] * Ut[0][b, j] * Ut[2][c, j] for j in range(U[1].shape[1]))
    assert abs(M[i, b * r2 + c] - want) < 1e-12 * (1 + abs(want))
