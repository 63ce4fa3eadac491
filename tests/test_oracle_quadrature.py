"""Pins for oracle.quadrature (section 2.2-2.3)."""
import math

import mpmath
import numpy as np
import pytest

from oracle import quadrature as Q
from oracle import rhosvd

SQRT_PI = math.sqrt(math.pi)


def poisson_closed_form(r, h, M):
    """Exact value of the folded literal Newton rule by Poisson summation:
    (h/sqrt(pi)) sum_{k=-M}^{M} e^{-k^2 h^2 r^2}
      = (1/r)[1 + 2 sum_{m>=1} e^{-(pi m/(h r))^2}] - (2h/sqrt(pi)) sum_{k>M} e^{-k^2 h^2 r^2}."""
    mp = mpmath.mp
    mp.dps = 40
    r = mpmath.mpf(r)
    h = mpmath.mpf(h)
    alias = mpmath.nsum(lambda m: mpmath.exp(-(mpmath.pi * m / (h * r)) ** 2), [1, mpmath.inf])
    tail = mpmath.nsum(lambda k: mpmath.exp(-(k * h * r) ** 2), [M + 1, mpmath.inf])
    return float((1 + 2 * alias) / r - 2 * h / mpmath.sqrt(mpmath.pi) * tail)


@pytest.mark.parametrize("R", [20, 24, 28, 32])
def test_newton_literal_rule_matches_poisson_closed_form(R):
    t, a = Q.literal_table("newton", R)
    h = Q.step_size(R)
    M = R - 1
    for r in [0.05, 0.3, 0.7, 1.0, 1.9, 3.0, 5.0, 12.0]:
        s = float(Q.kernel_sum(np.array([r]), t, a)[0])
        ref = poisson_closed_form(r, h, M)
        assert abs(s - ref) <= 1e-14 * max(abs(ref), 1.0), (r, s, ref)


def test_step_size_and_term_count():
    # eq hM with C0 = 3: h_M = 3 log(M)/M, and R = M + 1 terms (section 2.2)
    for R in [20, 24, 32]:
        M = R - 1
        t, a = Q.literal_table("newton", R)
        assert len(t) == R and len(a) == R
        assert t[0] == 0.0
        assert abs(t[1] - 3 * math.log(M) / M) < 1e-15
        # folded weights: S(0) = h (2M + 1) / sqrt(pi)
        assert abs(a.sum() - t[1] * (2 * M + 1) / SQRT_PI) < 1e-13


def test_newton_and_yukawa_converge_to_kernel_on_fine_rule():
    # with a fine step (large R) the rule reproduces the kernels on a mid
    # range.  The Yukawa weight exp(-lam^2/4t^2) is not analytic at t = 0,
    # so its trapezoid error decays slowly; it must still decrease with R.
    r = np.linspace(0.5, 3.0, 11)
    t, a = Q.literal_table("newton", 400)
    assert np.max(np.abs(Q.kernel_sum(r, t, a) - 1 / r) * r) < 1e-13
    errs = []
    for R in [100, 200, 400, 800]:
        for kernel in ["yukawa", "newton+yukawa"]:
            t, a = Q.literal_table(kernel, R)
            ref = Q.kernel_value(kernel, r, 0.5)
            errs.append((R, kernel, np.max(np.abs(Q.kernel_sum(r, t, a) - ref) / ref)))
    yk = [e for (R, k, e) in errs if k == "yukawa"]
    assert all(yk[i + 1] < yk[i] for i in range(len(yk) - 1))
    assert yk[-1] < 1e-7


def test_yukawa_laplace_gauss_identity_mpmath():
    # e^{-lam r}/r = (2/sqrt(pi)) int_0^inf exp(-r^2 t^2 - lam^2/(4 t^2)) dt
    mpmath.mp.dps = 30
    lam = 0.5
    for r in [0.3, 1.0, 4.0]:
        f = lambda t: Q.laplace_weight("yukawa", np.array([float(t)]), lam)[0] * mpmath.exp(-(r * t) ** 2)
        val = mpmath.quad(f, [0, 0.1, 1, 10, mpmath.inf])
        assert abs(float(val) - math.exp(-lam * r) / r) < 1e-12 * math.exp(-lam * r) / r


def test_yukawa_weights_vanish_at_zero_and_are_below_newton():
    t, a = Q.literal_table("yukawa", 28)
    tn, an = Q.literal_table("newton", 28)
    assert a[0] == 0.0
    assert np.all(a <= an + 1e-300)


@pytest.mark.parametrize("M,sigma,delta", [(19, 0.7, 1e-3), (23, 0.6, 1e-4), (31, 0.5, 1e-6), (40, 0.9, 1e-5)])
def test_criterion_A_matches_printed_equation(M, sigma, delta):
    """Section 2.3: for C0 = 3 and a(t) = 1, criterion (A) gives R_l solving
    (3 R_l log M / M)^2 sigma^2 = log(h_M / delta)."""
    h = 3 * math.log(M) / M
    t = np.arange(M + 1) * h
    a = np.full(M + 1, h)
    R_l = Q.split_criterion_A(t, a, sigma, delta)
    root = M * math.sqrt(math.log(h / delta)) / (3 * math.log(M) * sigma)
    assert R_l == math.ceil(root - 1e-12)


def test_criterion_A_on_newton_weights_is_min_k():
    t, a = Q.literal_table("newton", 20)
    for sigma in [0.4, 0.6, 0.9]:
        delta = 1e-4 * a.sum()
        R_l = Q.split_criterion_A(t, a, sigma, delta)
        vals = a * np.exp(-(t * sigma) ** 2)
        assert np.all(vals[R_l:] <= delta)
        assert R_l == 0 or vals[R_l - 1] > delta


@pytest.mark.parametrize("R,R_l,b,n", [(20, 8, 10.0, 128), (24, 10, 12.0, 512), (28, 11, 18.0, 512), (32, 12, 25.0, 1024)])
def test_window_excludes_only_small_short_terms(R, R_l, b, n):
    """Brute force: a particle anywhere in its cell; every excluded cell centre
    (outside j +- w in some mode) sees each short term below delta, and the
    next smaller odd window would not guarantee it."""
    t, a = Q.literal_table("newton", R)
    h = 2 * b / n
    delta = 1e-4 * a.sum()
    n_s = Q.derive_window(t, a, R_l, 1e-4, h)
    w = (n_s - 1) // 2
    offs = np.linspace(0.0, 1.0, 41)          # particle offset from its cell's left face, in units of h
    # excluded centres j+w+1 and j-w-1 lie at (w + 3/2 - off) h and (w + 1/2 + off) h
    dists = np.concatenate([(w + 1.5 - offs) * h, (w + 0.5 + offs) * h])
    worst = max(float(np.max(a[k] * np.exp(-(t[k] * dists) ** 2))) for k in range(R_l, R))
    assert worst <= delta * (1 + 1e-12)
    if n_s >= 3:
        w2 = w - 1
        d2 = np.concatenate([(w2 + 1.5 - offs) * h, (w2 + 0.5 + offs) * h])
        worst2 = max(float(np.max(a[k] * np.exp(-(t[k] * d2) ** 2))) for k in range(R_l, R))
        assert worst2 > delta


def test_window_values_of_the_workloads():
    # the configs' stated and derived windows (criterion (A), delta = 1e-4 S(0))
    t, a = Q.literal_table("newton", 20)
    assert Q.derive_window(t, a, 8, 1e-4, 20 / 128) == 9
    t, a = Q.literal_table("newton", 24)
    assert Q.derive_window(t, a, 10, 1e-4, 24 / 512) == 27
    t, a = Q.literal_table("newton", 28)
    assert Q.derive_window(t, a, 11, 1e-4, 36 / 512) == 19


def _golden_ranks():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_canonical_ranks.txt")
    rows = []
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            tab, N, terms, rank = line.split()
            rows.append((tab, int(N), int(terms), int(rank)))
    return rows


@pytest.mark.parametrize("row", _golden_ranks())
def test_initial_canonical_rank_matches_paper_tables(row):
    """The side matrix of the canonical sum has one column per (term,
    particle): its width is the initial rank the paper prints."""
    _, N, terms, rank = row
    rng = np.random.default_rng(N)
    coords = rng.uniform(-5, 5, size=N)
    t = np.arange(terms) * 0.3
    U = rhosvd.side_matrix(10.0, 8, coords, t)
    assert U.shape[1] == rank


# ---- the exponentially convergent rule (substitution t = e^s) ----------------

def _rel_err_mp(kernel, t, a, r_lo, r_hi, lam=0.5, m=400):
    """max |S(r)/p(r) - 1| over a log grid of [r_lo, r_hi], p from mpmath."""
    mpmath.mp.dps = 30
    worst = 0.0
    for x in np.exp(np.linspace(np.log(r_lo), np.log(r_hi), m)):
        xm = mpmath.mpf(float(x))
        if kernel == "newton":
            p = 1 / xm
        elif kernel == "yukawa":
            p = mpmath.exp(-lam * xm) / xm
        else:
            p = (1 + mpmath.exp(-lam * xm)) / xm
        S = mpmath.fsum(mpmath.mpf(float(ak)) * mpmath.exp(-(mpmath.mpf(float(tk)) * xm) ** 2)
                        for tk, ak in zip(t, a))
        worst = max(worst, float(abs(S / p - 1)))
    return worst


@pytest.mark.parametrize("R,b,n", [(20, 10.0, 128), (24, 12.0, 512), (32, 25.0, 1024)])
def test_expsinc_newton_error_within_its_design_bound(R, b, n):
    """Against 1/r evaluated in mpmath: the maximum relative error on
    [h, 2 sqrt(3) b] stays within three times the rule's own design
    accuracy e^{-L} and below 3e-4 (R >= 20)."""
    r_lo, r_hi = Q.default_range(b, n)
    t, a, L = Q.expsinc_table("newton", R, r_lo, r_hi)
    err = _rel_err_mp("newton", t, a, r_lo, r_hi)
    assert err <= 3.0 * math.exp(-L)
    assert err <= 3e-4
    assert np.all(np.diff(t) > 0) and t[0] == 0.0 and np.all(a > 0)


def test_expsinc_converges_exponentially_in_sqrt_M():
    """The error falls like e^{-beta sqrt(M)} (eq sinc_conv): log(err) is
    decreasing and close to linear in sqrt(M) with a negative slope."""
    r_lo, r_hi = Q.default_range(12.0, 512)
    Ms, errs = [], []
    for R in (12, 16, 20, 24, 28, 32, 40):
        t, a, _ = Q.expsinc_table("newton", R, r_lo, r_hi)
        Ms.append(R - 1)
        errs.append(_rel_err_mp("newton", t, a, r_lo, r_hi, m=200))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    slope, icept = np.polyfit(np.sqrt(Ms), np.log(errs), 1)
    assert slope < -1.0
    resid = np.log(errs) - (slope * np.sqrt(Ms) + icept)
    assert np.max(np.abs(resid)) < 1.0


def test_expsinc_tail_weight_is_the_sum_of_the_dropped_nodes():
    """a_0 (t_0 = 0) equals the trapezoid weights h (2/sqrt(pi)) e^{s} of the
    nodes s_1 - h, s_1 - 2h, ... summed by brute force."""
    t, a, L = Q.expsinc_table("newton", 24, 0.05, 40.0)
    s1 = math.log(t[1])
    h = math.log(t[2]) - math.log(t[1])
    brute = sum(2.0 / math.sqrt(math.pi) * h * math.exp(s1 - j * h) for j in range(1, 2000))
    assert abs(a[0] - brute) <= 1e-14 * brute
    assert np.allclose(np.diff(np.log(t[1:])), h, rtol=1e-12, atol=0)


@pytest.mark.parametrize("kernel", ["yukawa", "newton+yukawa"])
def test_expsinc_yukawa_against_mpmath(kernel):
    """The screened kernels with the same nodes (R = 28, lam = 0.5), against
    mpmath: the Newton-plus-Yukawa sum to 1e-3 relative on [h, 2 sqrt(3) b];
    Yukawa alone to 1e-3 relative on [h, 5] and, on the whole range, to
    1e-4 on the scale of 1/r (|S - p| r), since e^{-lam r}/r itself falls
    to 1e-7 of 1/r there; the Yukawa weight at t_0 = 0 is 0."""
    r_lo, r_hi = Q.default_range(18.0, 512)
    t, a, _ = Q.expsinc_table(kernel, 28, r_lo, r_hi, lam=0.5)
    tn, an, _ = Q.expsinc_table("newton", 28, r_lo, r_hi)
    assert np.array_equal(t, tn)
    if kernel == "newton+yukawa":
        assert _rel_err_mp(kernel, t, a, r_lo, r_hi, m=300) <= 1e-3
        return
    assert a[0] == 0.0
    assert _rel_err_mp(kernel, t, a, r_lo, 5.0, m=300) <= 1e-3
    mpmath.mp.dps = 30
    worst = 0.0
    for x in np.exp(np.linspace(np.log(r_lo), np.log(r_hi), 300)):
        xm = mpmath.mpf(float(x))
        S = mpmath.fsum(mpmath.mpf(float(ak)) * mpmath.exp(-(mpmath.mpf(float(tk)) * xm) ** 2)
                        for tk, ak in zip(t, a))
        worst = max(worst, float(abs(S - mpmath.exp(-0.5 * xm) / xm) * xm))
    assert worst <= 1e-4
