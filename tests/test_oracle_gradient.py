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


def _small_rs(seed=3, N=6, n=40, b=4.0):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-0.5 * b, 0.5 * b, size=(N, 3))
    q = rng.choice([-1.0, 1.0], size=N) * rng.uniform(0.5, 1.5, size=N)
    h = grid.spacing(b, n)
    t, a, _ = quadrature.expsinc_table("newton", 40, h / 4, 2 * np.sqrt(3) * b)
    R_l = quadrature.split_criterion_A(t, a, 0.8, 1e-8 * float(np.sum(a)))
    n_s = quadrature.derive_window(t, a, R_l, 1e-8, h)
    return rs.assemble(b, n, pos, q, t, a, R_l=R_l, n_s=n_s, eps=1e-10)


def _interior_points(T, rng, M):
    # points whose coordinates sit a quarter cell away from cell faces and
    # from cell centres, so that a step of 1e-6 changes neither the window
    # membership nor the interpolation stencil
    n, b, h = T.n, T.b, T.h
    cells = rng.integers(4, n - 4, size=(M, 3))
    frac = rng.choice([0.1, 0.35, 0.65, 0.9], size=(M, 3))
    return -b + (cells + frac) * h


@pytest.mark.parametrize("part", [0, 1, 2])
def test_point_gradient_matches_central_differences(part):
    from oracle import pointeval
    T = _small_rs()
    rng = np.random.default_rng(7)
    P = _interior_points(T, rng, 40)
    g = pointeval.gradient_points(T, P, part=part)
    eps = 1e-6
    scale = np.max(np.abs(g))
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = eps
        fd = (pointeval.eval_points(T, P + e, part=part) -
              pointeval.eval_points(T, P - e, part=part)) / (2 * eps)
        assert np.max(np.abs(fd - g[:, ax])) < 1e-6 * scale


def test_normal_derivative_is_the_directional_derivative():
    from oracle import pointeval
    T = _small_rs(seed=5)
    rng = np.random.default_rng(8)
    P = _interior_points(T, rng, 30)
    nrm = rng.normal(size=(30, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    dn = pointeval.gradient_points(T, P, part=0, normals=nrm)
    eps = 1e-6
    fd = (pointeval.eval_points(T, P + eps * nrm) - pointeval.eval_points(T, P - eps * nrm)) / (2 * eps)
    # a step along a general direction may cross a face in another axis:
    # those points are left out
    cells_p = grid.cell_of(P + eps * nrm, T.b, T.n)
    cells_m = grid.cell_of(P - eps * nrm, T.b, T.n)
    same = np.all(cells_p == cells_m, axis=1)
    assert np.sum(same) > 20
    assert np.max(np.abs(fd - dn)[same]) < 1e-6 * np.max(np.abs(dn))


def test_long_range_normal_derivative_on_a_far_surface():
    # on a sphere further than the short-range support from every particle
    # the short part is below the split's delta (1e-8 S(0) here, windows may
    # still reach the sphere), so the long part alone gives the
    # interface data, and it agrees with the exact field's normal component
    # to the accuracy of the order-6 interpolant's derivative (h ~ 0.21 at
    # distance ~2 from the charges: a few 1e-4)
    from oracle import pointeval
    T = _small_rs(seed=9, N=5, n=48, b=5.0)
    T.pos *= 0.4          # particles within 0.8 of the origin
    T = rs.assemble(T.b, T.n, T.pos, T.q, T.t, T.a, T.R_l, T.n_s, eps=1e-10)
    rng = np.random.default_rng(10)
    nrm = rng.normal(size=(60, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    P = 2.5 * nrm
    long_dn = pointeval.gradient_points(T, P, part=1, normals=nrm)
    short_dn = pointeval.gradient_points(T, P, part=2, normals=nrm)
    assert np.max(np.abs(short_dn)) < 1e-8 * np.max(np.abs(long_dn))
    d = P[:, None, :] - T.pos[None, :, :]
    r = np.linalg.norm(d, axis=2)
    exact = -np.sum(T.q[None, :] * np.sum(d * nrm[:, None, :], axis=2) / r ** 3, axis=1)
    assert np.max(np.abs(long_dn - exact)) < 1e-3 * np.max(np.abs(exact))
