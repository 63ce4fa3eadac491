"""Pins for oracle.rbf (section 4.1, the RS form of the RBF matrix)."""
import numpy as np

from oracle import quadrature, rbf


def test_long_part_is_the_gaussian_sum_of_the_distance():
    # without short-range terms the entry is S(|x_i - x_j|), S the kernel's
    # quadrature sum: a radial function of the cell distance
    b, n = 2.0, 6
    t, a = quadrature.literal_table("newton", 16)
    A = rbf.rbf_matrix(b, n, t, a, len(t), 1)
    h = 2 * b / n
    idx = np.indices((n, n, n)).reshape(3, -1).T
    for i, j in [(0, 0), (3, 200), (17, 101), (215, 1)]:
        r = np.linalg.norm((idx[i] - idx[j]) * h)
        assert abs(A[i, j] - quadrature.kernel_sum(r, t, a)) < 1e-12 * (1 + abs(A[i, j]))


def test_symmetric_and_translation_invariant():
    b, n = 3.0, 5
    t, a = quadrature.literal_table("newton", 20)
    A = rbf.rbf_matrix(b, n, t, a, 8, 3)
    assert np.max(np.abs(A - A.T)) == 0.0
    # entries depend on i - j only (multilevel Toeplitz)
    T = A.reshape(n, n, n, n, n, n)
    assert abs(T[0, 1, 2, 1, 2, 3] - T[2, 1, 0, 3, 2, 1]) < 1e-15
    assert abs(T[0, 0, 0, 2, 2, 2] - T[1, 1, 1, 3, 3, 3]) < 1e-15


def test_short_terms_vanish_outside_the_window_and_match_the_kernel_inside():
    b, n = 3.0, 7
    t, a = quadrature.literal_table("newton", 20)
    R_l, n_s = 8, 3
    full = rbf.rbf_matrix(b, n, t, a, len(t), 1)      # every term untruncated
    longp = rbf.rbf_matrix(b, n, t, a, R_l, 1)        # window of one cell: short terms on the diagonal only
    A = rbf.rbf_matrix(b, n, t, a, R_l, n_s)
    idx = np.indices((n, n, n)).reshape(3, -1).T
    far = np.any(np.abs(idx[:, None, :] - idx[None, :, :]) > 1, axis=2)
    near = ~far
    lg = rbf.rbf_matrix(b, n, t, a, R_l, 1)
    # outside the window only the long terms remain; inside, every term
    assert np.allclose(A[far], lg[far], rtol=0, atol=1e-14)
    assert np.allclose(A[near], full[near], rtol=1e-14, atol=1e-14)
    assert np.max(np.abs(longp - A)) > 0


def test_matvec_of_a_delta_is_a_column():
    b, n = 2.5, 5
    t, a = quadrature.literal_table("newton", 20)
    A = rbf.rbf_matrix(b, n, t, a, 8, 3)
    c = np.zeros((n, n, n))
    c[1, 3, 2] = 1.0
    y = rbf.rbf_matvec(b, n, t, a, 8, 3, c)
    assert np.max(np.abs(y.ravel() - A[:, np.ravel_multi_index((1, 3, 2), (n, n, n))])) == 0.0
