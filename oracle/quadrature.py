"""Sinc quadrature of the Laplace-Gauss transform and the range split.

Section 2.2 (eqs laplace, hM, sinc_Newt, sinc_general) and section 2.3
(eqs Split_Qpoints, Split_Tens, Split_crit_max).

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
