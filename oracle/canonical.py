"""Direct and canonical potential sums, and the short-range cumulated
canonical tensor (CCT) on the grid.

P_0(x) = sum_nu z_nu p(|x - x_nu|)                         (eq PotSum)
P_R  ~ sum_k a_k prod_l exp(-t_k^2 x_l^2)                  (eq sinc_Newt / sinc_general)
P_s  = sum_nu z_nu W_nu(P_{R_s}),  windowed to the gamma-vicinity of the
       particle's cell (Definitions ComCanF, CCT_Uniform; eq Total_Sum)

Particles need not sit on grid points: every Gaussian is collocated at the
true particle coordinate (reading of section 3.2, which assumes on-grid
particles "for technical reasons"); the shift-and-window form is then the
on-grid special case.
"""
from __future__ import annotations

import numpy as np

from . import grid as _grid
from .quadrature import kernel_value


def direct_potential(points, pos, q, kernel: str = "newton", lam: float = 0.5, chunk: int = 1 << 16):
    """P_0(y) = sum_nu z_nu p(|y - x_nu|) at arbitrary points (eq PotSum)."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(points.shape[0])
    for s in range(0, points.shape[0], chunk):
        y = points[s:s + chunk]
        acc = np.zeros(y.shape[0])
        for nu in range(pos.shape[0]):
            r = np.sqrt(np.sum((y - pos[nu]) ** 2, axis=1))
            acc += q[nu] * kernel_value(kernel, r, lam)
        out[s:s + chunk] = acc
    return out


def canonical_potential_radial(points, pos, q, t, a, ks=None, chunk: int = 1 << 16):
    """sum_nu z_nu S(|y - x_nu|) with S(r) = sum_{k in ks} a_k exp(-t_k^2 r^2),
    evaluated radially."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    if ks is None:
        ks = range(len(t))
    ks = list(ks)
    out = np.zeros(points.shape[0])
    for s in range(0, points.shape[0], chunk):
        y = points[s:s + chunk]
        acc = np.zeros(y.shape[0])
        for nu in range(pos.shape[0]):
            r2 = np.sum((y - pos[nu]) ** 2, axis=1)
            for k in ks:
                acc += q[nu] * a[k] * np.exp(-t[k] ** 2 * r2)
        out[s:s + chunk] = acc
    return out


def canonical_potential_separable(points, pos, q, t, a, ks=None):
    """The same sum through the separable form: each Gaussian written as the
    product of three 1D Gaussians (eq sinc_Newt)."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    if ks is None:
        ks = range(len(t))
    out = np.zeros(points.shape[0])
    for nu in range(pos.shape[0]):
        for k in ks:
            g = np.ones(points.shape[0])
            for l in range(3):
                g = g * np.exp(-t[k] ** 2 * (points[:, l] - pos[nu, l]) ** 2)
            out += q[nu] * a[k] * g
    return out


def window_bounds(pos, b: float, n: int, n_s: int):
    """Per particle, the inclusive index range [lo, hi] of its window in each
    mode: the particle's cell j plus/minus w = (n_s - 1)/2, clipped to the
    grid (the gamma-vicinity of Definition ComCanF with gamma = w)."""
    w = (n_s - 1) // 2
    j = _grid.cell_of(pos, b, n)
    return np.clip(j - w, 0, n - 1), np.clip(j + w, 0, n - 1)


def short_range_grid(b: float, n: int, pos, q, t, a, R_l: int, n_s: int):
    """The dense n^3 short-range CCT sum_nu z_nu U_nu, each U_nu the
    short-range part of the reference tensor (terms k >= R_l) collocated at
    x_nu and restricted to its window.  Small n only."""
    x = _grid.cell_centres(b, n)
    out = np.zeros((n, n, n))
    lo, hi = window_bounds(pos, b, n, n_s)
    for nu in range(pos.shape[0]):
        sl = tuple(slice(lo[nu, l], hi[nu, l] + 1) for l in range(3))
        block = np.zeros(tuple(hi[nu] - lo[nu] + 1))
        for k in range(R_l, len(t)):
            g = [np.exp(-t[k] ** 2 * (x[sl[l]] - pos[nu, l]) ** 2) for l in range(3)]
            block += a[k] * np.einsum("i,j,k->ijk", g[0], g[1], g[2])
        out[sl] += q[nu] * block
    return out


def short_range_at(idx3, b: float, n: int, pos, q, t, a, R_l: int, n_s: int):
    """Short-range CCT values at grid indices idx3 (M x 3): for each point,
    the sum over particles nu whose window contains it (the set L(i) of
    Lemma Property_RST_can)."""
    idx3 = np.asarray(idx3, dtype=np.int64).reshape(-1, 3)
    x = _grid.cell_centres(b, n)
    y = x[idx3]
    lo, hi = window_bounds(pos, b, n, n_s)
    out = np.zeros(idx3.shape[0])
    for nu in range(pos.shape[0]):
        inside = np.all((idx3 >= lo[nu]) & (idx3 <= hi[nu]), axis=1)
        if not np.any(inside):
            continue
        d2 = np.sum((y[inside] - pos[nu]) ** 2, axis=1)
        s = np.zeros(d2.shape[0])
        for k in range(R_l, len(t)):
            s += a[k] * np.exp(-t[k] ** 2 * d2)
        out[inside] += q[nu] * s
    return out


def short_range_points(points, b: float, n: int, pos, q, t, a, R_l: int, n_s: int):
    """Short-range part at arbitrary points: particles whose window contains
    the cell of the point contribute their short-range Gaussians evaluated
    at the point itself."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    cells = _grid.cell_of(points, b, n)
    lo, hi = window_bounds(pos, b, n, n_s)
    out = np.zeros(points.shape[0])
    for nu in range(pos.shape[0]):
        inside = np.all((cells >= lo[nu]) & (cells <= hi[nu]), axis=1)
        if not np.any(inside):
            continue
        d2 = np.sum((points[inside] - pos[nu]) ** 2, axis=1)
        s = np.zeros(d2.shape[0])
        for k in range(R_l, len(t)):
            s += a[k] * np.exp(-t[k] ** 2 * d2)
        out[inside] += q[nu] * s
    return out


def short_range_points_grad(points, b: float, n: int, pos, q, t, a, R_l: int, n_s: int):
    """Gradient in y of short_range_points (section 4.3): each windowed term
    z_nu a_k exp(-t_k^2 |y - x_nu|^2) differentiated analytically,
    -2 t_k^2 (y - x_nu) times the term, for the particles whose window holds
    the point's cell.  Result: M x 3."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    cells = _grid.cell_of(points, b, n)
    lo, hi = window_bounds(pos, b, n, n_s)
    out = np.zeros((points.shape[0], 3))
    for nu in range(pos.shape[0]):
        inside = np.all((cells >= lo[nu]) & (cells <= hi[nu]), axis=1)
        if not np.any(inside):
            continue
        d = points[inside] - pos[nu]
        d2 = np.sum(d ** 2, axis=1)
        c = np.zeros(d2.shape[0])
        for k in range(R_l, len(t)):
            c += -2.0 * t[k] ** 2 * a[k] * np.exp(-t[k] ** 2 * d2)
        out[inside] += q[nu] * c[:, None] * d
    return out


def short_range_subgrid(I1, I2, I3, b: float, n: int, pos, q, t, a, R_l: int, n_s: int):
    """The short-range CCT sum_nu z_nu U_nu (as short_range_grid) on the
    index set I1 x I2 x I3 only: each particle adds its windowed local
    tensor at the indices of the set that fall inside its window.  Result:
    |I1| x |I2| x |I3|."""
    idx = [np.asarray(I, dtype=np.int64) for I in (I1, I2, I3)]
    x = _grid.cell_centres(b, n)
    out = np.zeros(tuple(len(I) for I in idx))
    lo, hi = window_bounds(pos, b, n, n_s)
    # particles whose window meets the set in every mode (a count of the set's
    # indices inside [lo, hi] per mode, from sorted copies)
    srt = [np.sort(I) for I in idx]
    touches = np.ones(pos.shape[0], dtype=bool)
    for l in range(3):
        cnt = np.searchsorted(srt[l], hi[:, l], "right") - np.searchsorted(srt[l], lo[:, l], "left")
        touches &= cnt > 0
    for nu in np.nonzero(touches)[0]:
        sel = [np.nonzero((idx[l] >= lo[nu, l]) & (idx[l] <= hi[nu, l]))[0] for l in range(3)]
        if any(s.size == 0 for s in sel):
            continue
        block = np.zeros(tuple(s.size for s in sel))
        for k in range(R_l, len(t)):
            g = [np.exp(-t[k] ** 2 * (x[idx[l][sel[l]]] - pos[nu, l]) ** 2) for l in range(3)]
            block += a[k] * np.einsum("i,j,k->ijk", g[0], g[1], g[2])
        out[np.ix_(sel[0], sel[1], sel[2])] += q[nu] * block
    return out
