"""Pins for oracle.pointeval and oracle.pairwise (sections 4.2-4.3)."""
import math

import numpy as np
import pytest

import workloads
from oracle import grid, pairwise, pointeval, quadrature, rs
from tests.test_oracle_quadrature import poisson_closed_form


@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_lagrange_exact_on_polynomials_and_nodes(p):
    b, n = 3.0, 16
    x = grid.cell_centres(b, n)
    rng = np.random.default_rng(p)
    coef = rng.normal(size=p)
    f = lambda y: sum(c * y ** i for i, c in enumerate(coef))
    df = lambda y: sum(i * c * y ** (i - 1) for i, c in enumerate(coef) if i > 0)
    for y in list(rng.uniform(-b, b, 20)) + [-b, b - 1e-12, x[0], x[-1]]:
        s, L, dL = pointeval.lagrange_stencil(y, b, n, p)
        assert 0 <= s <= n - p
        assert abs(L @ f(x[s:s + p]) - f(y)) <= 1e-11 * (1 + abs(f(y)))
        assert abs(dL @ f(x[s:s + p]) - df(y)) <= 1e-9 * (1 + abs(df(y)))
    for i in range(n):
        s, L, _ = pointeval.lagrange_stencil(x[i], b, n, p)
        e = np.zeros(p)
        e[i - s] = 1.0
        assert np.max(np.abs(L - e)) < 1e-12


def test_energy_lemma_on_grid_particles_full_rank():
    """Lemma InterEnergy: for particles on grid points and the exact
    (full-rank) long-range tensor, 1/2 sum_j z_j (P_l(x_j) - z_j P_{R_l}(0))
    equals the pairwise long-range energy 1/2 sum_{i!=j} z_i z_j S_l(r_ij)."""
    b, n, R, R_l = 5.0, 20, 20, 8
    x = grid.cell_centres(b, n)
    rng = np.random.default_rng(7)
    idx = rng.choice(n ** 3, size=9, replace=False)
    ijk = grid.flat_to_ijk(idx, n)
    pos = x[ijk]
    q = rng.uniform(-1, 1, size=9)
    t, a = quadrature.literal_table("newton", R)
    T = rs.assemble(b, n, pos, q, t, a, R_l, 5, eps=0.0, fixed_ranks=[n] * 3)
    E_paper, dq_paper = pointeval.energy(T, self_term="paper")
    E_interp, dq_interp = pointeval.energy(T, self_term="interp")
    E_can, _ = pairwise.energy_canonical(pos, q, t, a, range(R_l))
    assert abs(E_paper - E_can) <= 1e-12 * np.sum(np.abs(q)) ** 2
    assert abs(E_interp - E_paper) <= 1e-13 * np.sum(np.abs(q)) ** 2


def test_energy_link_between_canonical_and_exact():
    """E_can_l - E_exact = 1/2 sum_{i!=j} z_i z_j (e(r_ij) - S_s(r_ij)), with
    e the quadrature error from the Poisson closed form."""
    s = workloads.tiny_system(31, 8, 6.0, 32, 20, 8, 7, min_sep=0.8)
    t, a = quadrature.literal_table("newton", s.R)
    h, M = quadrature.step_size(s.R), s.R - 1
    E_can, _ = pairwise.energy_canonical(s.pos, s.q, t, a, range(s.R_l))
    E_ex, _ = pairwise.energy_exact(s.pos, s.q)
    link = 0.0
    for i in range(s.N):
        for j in range(s.N):
            if i != j:
                r = float(np.linalg.norm(s.pos[i] - s.pos[j]))
                e = poisson_closed_form(r, h, M) - 1.0 / r
                Ss = float(quadrature.kernel_sum(np.array([r]), t, a, range(s.R_l, s.R))[0])
                link += 0.5 * s.q[i] * s.q[j] * (e - Ss)
    assert abs((E_can - E_ex) - link) <= 1e-12 * np.sum(np.abs(s.q)) ** 2


def test_two_particle_exact_energy_and_forces():
    pos = np.array([[0.0, 0.0, 0.0], [0.3, -1.2, 2.0]])
    q = np.array([0.8, -1.5])
    r = np.linalg.norm(pos[1] - pos[0])
    for kernel in ["newton", "yukawa", "newton+yukawa"]:
        E, F = pairwise.energy_exact(pos, q, kernel, 0.5, forces=True)
        assert abs(E - q[0] * q[1] * quadrature.kernel_value(kernel, r, 0.5)) < 1e-15
        # Coulomb: F_0 = z0 z1 (x0 - x1)/r^3 for Newton
        if kernel == "newton":
            assert np.allclose(F[0], q[0] * q[1] * (pos[0] - pos[1]) / r ** 3, rtol=1e-14, atol=0)
        assert np.allclose(F.sum(0), 0.0, atol=1e-15)


def test_pairwise_forces_match_finite_differences():
    s = workloads.tiny_system(41, 7, 5.0, 16, 20, 8, 5, min_sep=0.7)
    t, a = quadrature.literal_table("newton", s.R)
    for fn in [lambda p: pairwise.energy_exact(p, s.q, "yukawa", 0.5, True),
               lambda p: pairwise.energy_canonical(p, s.q, t, a, range(s.R_l), True)]:
        E, F = fn(s.pos)
        hstep = 1e-5
        for j in range(s.N):
            for l in range(3):
                pp, pm = s.pos.copy(), s.pos.copy()
                pp[j, l] += hstep
                pm[j, l] -= hstep
                fd = -(fn(pp)[0] - fn(pm)[0]) / (2 * hstep)
                assert abs(fd - F[j, l]) <= 1e-7 * np.max(np.abs(F))
        assert np.max(np.abs(F.sum(0))) <= 1e-13 * np.max(np.abs(F)) * s.N


def test_rs_energy_and_forces_close_to_pairwise_long_range():
    s = workloads.tiny_system(51, 16, 6.0, 64, 20, 8, 9, min_sep=0.8)
    T = rs.assemble_system(s)
    t, a = T.t, T.a
    E, dq = pointeval.energy(T)
    E_can, F_can = pairwise.energy_canonical(s.pos, s.q, t, a, range(s.R_l), forces=True)
    assert abs(E - E_can) <= 1e-4 * np.sum(np.abs(s.q)) ** 2 / s.N
    F = pointeval.forces(T)
    assert np.max(np.abs(F - F_can)) <= 1e-2 * np.max(np.abs(F_can))


def test_rs_forces_match_finite_differences_of_rs_energy():
    """Central differences of the FP64 RS energy (reassembled for each
    displacement, h = 1e-4) against the frozen-basis analytic forces."""
    s = workloads.tiny_system(61, 6, 4.0, 48, 20, 8, 9, min_sep=0.9, eps_tucker=1e-9)
    T = rs.assemble_system(s)
    F = pointeval.forces(T)
    hstep = 1e-4
    for j in range(2):
        for l in range(3):
            pp, pm = s.pos.copy(), s.pos.copy()
            pp[j, l] += hstep
            pm[j, l] -= hstep
            sp = workloads.System(s.name, pp, s.q, s.b, s.n, s.R, s.R_l, s.n_s, eps_tucker=s.eps_tucker)
            sm = workloads.System(s.name, pm, s.q, s.b, s.n, s.R, s.R_l, s.n_s, eps_tucker=s.eps_tucker)
            fd = -(pointeval.energy(rs.assemble_system(sp))[0] - pointeval.energy(rs.assemble_system(sm))[0]) / (2 * hstep)
            assert abs(fd - F[j, l]) <= 2e-3 * np.max(np.abs(F)), (j, l, fd, F[j, l])


def test_eval_points_exact_at_grid_points():
    s = workloads.tiny_system(71, 5, 4.0, 20, 20, 8, 5, min_sep=0.8)
    T = rs.assemble_system(s)
    x = grid.cell_centres(s.b, s.n)
    rng = np.random.default_rng(2)
    ijk = rng.integers(0, s.n, size=(30, 3))
    pts = x[ijk]
    v = pointeval.eval_points(T, pts, part=0)
    ref = T.at(ijk)
    assert np.max(np.abs(v - ref)) <= 1e-12 * np.max(np.abs(ref))
