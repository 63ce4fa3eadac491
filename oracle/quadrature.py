"""Sinc quadrature of the Laplace-Gauss transform and the range split.

Section 2.2 (eqs laplace, hM, sinc_Newt, sinc_general) and section 2.3
(eqs Split_Qpoints, Split_Tens, Split_crit_max).

Two rules are provided: the paper-literal one (literal_table) and one with
the exponential convergence the paper claims (expsinc_table, reading below).

Readings taken where the paper is ambiguous:
* The rule sums k = -M..M with a_k = a(t_k) h_M for an integral over R+.
  Read as the trapezoid rule on the whole line for the even integrand,
  folded onto k >= 0:  a_0 = h a(0) / 2,  a_k = h a(t_k)  (k >= 1).
  With a(t) = 2/sqrt(pi) (Newton) that gives a_0 = h/sqrt(pi),
  a_k = 2h/sqrt(pi), and R = M + 1 terms as the paper states.
* R_l counts the long-range terms k = 0 .. R_l-1; R_s = R - R_l.
* Criterion (A) threshold delta is taken relative to S(0) = sum_k a_k.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

SQRT_PI = math.sqrt(math.pi)

KERNELS = ("newton", "yukawa", "newton+yukawa")


def laplace_weight(kernel: str, t, lam: float = 0.5):
    """a(t) with p(z) = int_0^inf a(t) exp(-t^2 z^2) dt (eq laplace).

    Newton  1/z:          a(t) = 2/sqrt(pi)                       (section 2.2)
    Yukawa  e^{-lam z}/z: a(t) = 2/sqrt(pi) exp(-lam^2 / (4 t^2))  (textbook
            Laplace-Gauss transform of the Yukawa kernel named in section 2.2;
            a(0) = 0 as the limit t -> 0)
    """
    t = np.asarray(t, dtype=np.float64)
    newton = np.full_like(t, 2.0 / SQRT_PI)
    with np.errstate(divide="ignore", over="ignore"):
        yuk = np.where(t > 0, 2.0 / SQRT_PI * np.exp(-lam * lam / (4.0 * np.where(t > 0, t, 1.0) ** 2)), 0.0)
    if kernel == "newton":
        return newton
    if kernel == "yukawa":
        return yuk
    if kernel == "newton+yukawa":
        return newton + yuk
    raise ValueError(kernel)


def kernel_value(kernel: str, r, lam: float = 0.5):
    """p(r) itself."""
    r = np.asarray(r, dtype=np.float64)
    if kernel == "newton":
        return 1.0 / r
    if kernel == "yukawa":
        return np.exp(-lam * r) / r
    if kernel == "newton+yukawa":
        return (1.0 + np.exp(-lam * r)) / r
    raise ValueError(kernel)


def kernel_derivative(kernel: str, r, lam: float = 0.5):
    """p'(r)."""
    r = np.asarray(r, dtype=np.float64)
    newton = -1.0 / (r * r)
    yuk = -np.exp(-lam * r) * (1.0 / (r * r) + lam / r)
    if kernel == "newton":
        return newton
    if kernel == "yukawa":
        return yuk
    if kernel == "newton+yukawa":
        return newton + yuk
    raise ValueError(kernel)


def step_size(R: int, C0: float = 3.0) -> float:
    """h_M = C0 log(M) / M with M = R - 1 (eq hM; R = M + 1, section 2.2)."""
    M = R - 1
    if M < 2:
        raise ValueError("need R >= 3")
    return C0 * math.log(M) / M


def literal_table(kernel: str, R: int, lam: float = 0.5, C0: float = 3.0) -> Tuple[np.ndarray, np.ndarray]:
    """Quadrature points t_k = k h_M and weights a_k, k = 0..R-1 (eq hM),
    folded onto k >= 0 (see module docstring)."""
    h = step_size(R, C0)
    k = np.arange(R, dtype=np.float64)
    t = k * h
    a = h * laplace_weight(kernel, t, lam)
    a[0] *= 0.5
    return t, a


def expsinc_table(kernel: str, R: int, r_lo: float, r_hi: float, lam: float = 0.5):
    """Quadrature with exponentially convergent error for r in [r_lo, r_hi]
    (the rate claimed in eq sinc_conv), from the substitution t = e^s in
    eq laplace.  Parity unpinned against the paper's own tables: the paper
    prints t_k = k h_M, whose convergence on the half line is not
    exponential, and does not state the substitution it used.

    With t = e^s the Newton integrand is (2/sqrt(pi)) e^{s - r^2 e^{2s}}, in
    u = s + log r the r-free g(u) = e^{u - e^{2u}} (integral sqrt(pi)/2 over
    the real line).  The trapezoid rule with step h on the whole line has
    relative error about exp(-pi^2 / (2h)) (g is analytic in |Im u| < pi/4);
    M = R - 1 nodes s_1, s_1 + h, ... are kept, and the dropped nodes to the
    left, where r e^s << 1 and the Gaussian factor is ~1, are summed as a
    geometric series into one term with t_0 = 0.  With L = -log(eps):
        h(L)     = pi^2 / (2 (L + log 2))                (discretisation ~ eps)
        u_l(L)   = (-L - log 0.38) / 3 + h/2              (left tail, ~ e^{3u}/3 ~ eps)
        u_r(L)   = log(L + 1) / 2                         (right tail e^{-e^{2u}} ~ eps)
    and L solves (M - 1) h(L) = u_r(L) - u_l(L) + log(r_hi / r_lo), so that
    the nodes span u_l at r = r_hi to u_r at r = r_lo; s_1 = u_l - log r_hi.
    Weights: t_0 = 0, a_0 = (2/sqrt(pi)) h e^{s_1} / (e^h - 1);
    t_k = e^{s_k}, a_k = (2/sqrt(pi)) h t_k.  Yukawa multiplies each weight
    by exp(-lam^2 / (4 t_k^2)) (a_0 = 0); the sum kernel adds the two.
    Returns (t, a, L)."""
    M = R - 1
    if M < 2:
        raise ValueError("need R >= 3")
    if not (0 < r_lo < r_hi):
        raise ValueError("need 0 < r_lo < r_hi")
    span = math.log(r_hi / r_lo)

    def h_of(L):
        return math.pi ** 2 / (2.0 * (L + math.log(2.0)))

    def u_left(L):
        return (-L - math.log(0.38)) / 3.0 + 0.5 * h_of(L)

    def u_right(L):
        return 0.5 * math.log(L + 1.0)

    def excess(L):   # node span minus the span the rule must cover; decreasing in L
        return (M - 1) * h_of(L) - (u_right(L) - u_left(L) + span)

    lo, hi = 0.5, 200.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if excess(mid) > 0:
            lo = mid
        else:
            hi = mid
    L = 0.5 * (lo + hi)
    h = h_of(L)
    s1 = u_left(L) - math.log(r_hi)
    t = np.zeros(R)
    t[1:] = np.exp(s1 + h * np.arange(M))
    c = 2.0 / SQRT_PI
    a_newton = np.empty(R)
    a_newton[0] = c * h * math.exp(s1) / math.expm1(h)
    a_newton[1:] = c * h * t[1:]
    yuk = np.zeros(R)
    yuk[1:] = np.exp(-lam * lam / (4.0 * t[1:] ** 2))
    if kernel == "newton":
        a = a_newton
    elif kernel == "yukawa":
        a = a_newton * yuk
    elif kernel == "newton+yukawa":
        a = a_newton * (1.0 + yuk)
    else:
        raise ValueError(kernel)
    return t, a, L


def default_range(b: float, n: int):
    """[r_lo, r_hi] = [h, 2 sqrt(3) b]: from one grid spacing to the largest
    distance between two points of the box [-b, b]^3."""
    return 2.0 * b / n, 2.0 * math.sqrt(3.0) * b


def kernel_sum(r, t, a, ks=None):
    """S(r) = sum_{k in ks} a_k exp(-t_k^2 r^2): the 1D profile of the
    canonical reference tensor P_R along a ray (eq sinc_general)."""
    r = np.asarray(r, dtype=np.float64)
    if ks is None:
        ks = range(len(t))
    out = np.zeros_like(r)
    for k in ks:
        out = out + a[k] * np.exp(-(t[k] * r) ** 2)
    return out


def kernel_sum_derivative(r, t, a, ks=None):
    """d/dr S(r) = -2 r sum_k a_k t_k^2 exp(-t_k^2 r^2)."""
    r = np.asarray(r, dtype=np.float64)
    if ks is None:
        ks = range(len(t))
    out = np.zeros_like(r)
    for k in ks:
        out = out - 2.0 * r * a[k] * t[k] ** 2 * np.exp(-(t[k] * r) ** 2)
    return out


def split_criterion_A(t, a, sigma: float, delta: float) -> int:
    """R_l from criterion (A) (eq Split_crit_max): the short set is the tail
    {t_k : k >= R_l} on which a_k exp(-t_k^2 sigma^2) <= delta holds.
    For the monotone Newton weights this is the paper's "min k"; read as a
    tail so that the Yukawa weights (a_0 = 0) give the same split."""
    R = len(t)
    R_l = R
    for k in range(R - 1, -1, -1):
        if a[k] * math.exp(-(t[k] * sigma) ** 2) <= delta:
            R_l = k
        else:
            break
    return R_l


def short_support_radius(t, a, R_l: int, delta: float) -> float:
    """Smallest sigma for which every short term k >= R_l satisfies
    a_k exp(-t_k^2 sigma^2) <= delta (criterion (A) solved for sigma)."""
    s = 0.0
    for k in range(R_l, len(t)):
        if a[k] > delta:
            s = max(s, math.sqrt(math.log(a[k] / delta)) / t[k])
    return s


def window_width(sigma: float, h: float) -> int:
    """Odd window width n_s = 2w+1 whose excluded cell centres lie at least
    sigma from any point of the particle's own cell: (w + 1/2) h >= sigma,
    i.e. the smallest odd n_s >= 2 sigma / h (section 3.3, sigma* ~ gamma h)."""
    n_s = int(math.ceil(2.0 * sigma / h - 1e-12))
    if n_s < 1:
        n_s = 1
    if n_s % 2 == 0:
        n_s += 1
    return n_s


def derive_window(t, a, R_l: int, delta_rel: float, h: float) -> int:
    """n_s from criterion (A) with delta = delta_rel * S(0)."""
    delta = delta_rel * float(np.sum(a))
    return window_width(short_support_radius(t, a, R_l, delta), h)
