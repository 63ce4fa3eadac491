"""Pins for oracle.gradient (section 4.3, eq Gradients_Tens)."""
import numpy as np
import pytest

import workloads
from oracle import grid, gradient, quadrature, rhosvd, rs


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fd_matches_numpy_first_order_edges(axis):
    # numpy's gradient with edge_order=1 is the same scheme: central inside,
    # one-sided at both ends
    rng = np.random.default_rng(axis)
    A = rng.normal(size=(9, 10, 11))
    D = gradient.fd_axis(A, 0.37, axis)
    ref = np.gradient(A, 0.37, axis=axis, edge_order=1)
    assert np.max(np.abs(D - ref)) < 1e-13


def test_fd_exact_on_quadratics_inside_and_linear_at_ends():
    b, n = 2.0, 12
    x = grid.cell_centres(b, n)
    h = grid.spacing(b, n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    quad = 3 * X ** 2 - 2 * X * Y + Z
    D = gradient.fd_axis(quad, h, 0)
    exact = 6 * X - 2 * Y
    assert np.max(np.abs(D[1:-1] - exact[1:-1])) < 1e-12
    # a one-sided difference of a quadratic is off by the second derivative
    # times h/2 at each end: f'' = 6
    assert np.allclose(D[0], exact[0] + 3 * h, atol=1e-12)
    assert np.allclose(D[-1], exact[-1] - 3 * h, atol=1e-12)
    lin = 2 * X - Y + 4 * Z
    for ax, c in [(0, 2.0), (1, -1.0), (2, 4.0)]:
        assert np.max(np.abs(gradient.fd_axis(lin, h, ax) - c)) < 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_tucker_form_equals_fd_of_full_grid(axis):
    # the separable long-range part: differencing the grid along one axis is
    # the Tucker tensor with that factor differenced column by column
    rng = np.random.default_rng(10 + axis)
    n = 10
    Q = [np.linalg.qr(rng.normal(size=(n, r)))[0] for r in (3, 4, 5)]
    beta = rng.normal(size=(3, 4, 5))
    h = 0.25
    full = rhosvd.tucker_full(beta, Q)
    Qd = list(Q)
    Qd[axis] = gradient.fd_axis(Q[axis], h, 0)
    assert np.max(np.abs(gradient.fd_axis(full, h, axis) - rhosvd.tucker_full(beta, Qd))) < 1e-12


def test_rs_gradient_approaches_the_coulomb_field():
    # -nabla_h of the assembled potential equals nabla_h of the exact sum
    # sum_k z_k / |x - x_k| up to the potential's own error over h (held at
    # ~1e-8 here by the quadrature, split and Tucker settings), and tends to
    # the field sum_k z_k (x - x_k)/|x - x_k|^3 at second order in h
    pos = np.array([[0.31, -0.22, 0.17], [-0.6, 0.45, -0.33]])
    q = np.array([1.0, -0.7])
    b = 4.0
    errs = []
    for n in (32, 64):
        h = grid.spacing(b, n)
        t, a, _ = quadrature.expsinc_table("newton", 48, h / 4, 2 * np.sqrt(3) * b)
        delta = 1e-9 * float(np.sum(a))
        R_l = quadrature.split_criterion_A(t, a, 0.6, delta)
        n_s = quadrature.derive_window(t, a, R_l, 1e-9, h)
        T = rs.assemble(b, n, pos, q, t, a, R_l=R_l, n_s=n_s, eps=1e-10)
        x = grid.cell_centres(b, n)
        X = np.stack(np.meshgrid(x, x, x, indexing="ij"), axis=-1)
        dist = [np.linalg.norm(X - p, axis=-1) for p in pos]
        exact = sum(z / r for z, r in zip(q, dist))
        rad = np.linalg.norm(X, axis=-1)
        sel = (rad > 2.0) & (rad < 3.0)
        # the potential's own error on the cells the differences reach
        e_pot = np.max(np.abs(T.full_grid() - exact)[(rad > 2.0 - 2 * h) & (rad < 3.0 + 2 * h)])
        assert e_pot < 1e-7
        err = 0.0
        for ax in range(3):
            G = gradient.gradient_grid(T, ax)
            F = sum(z * (X[..., ax] - p[ax]) / r ** 3 for z, p, r in zip(q, pos, dist))
            scale = np.max(np.abs(F[sel]))
            assert np.max(np.abs(G - gradient.fd_axis(exact, h, ax))[sel]) <= e_pot / h
            err = max(err, np.max(np.abs(-G - F)[sel]) / scale)
        errs.append(err)
    assert errs[1] < 2e-2
    assert 3.5 < errs[0] / errs[1] < 5.0
