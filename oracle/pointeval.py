"""Point evaluation of the RS tensor, the interaction energy and forces.

Energy: Lemma InterEnergy (eq EnergyFree_Tensor)
    E_N = 1/2 sum_j z_j (P_l(x_j) - z_j P_{R_l}(0)),
uses the long-range part only.  Forces: F_j = -grad_{x_j} E_N (section 4.3).
Differentiating the Lemma's expression with the Tucker basis held fixed gives
dE/dx_j = z_j grad P_l(x_j) (the self term has zero gradient) and
dE/dz_j = P_l(x_j) - z_j P_{R_l}(0).

Off-grid evaluation (the paper places particles on grid points and is
silent otherwise): order-p tensor Lagrange interpolation of the Tucker
factor rows on the cell-centred grid; stencil of p consecutive nodes
m - p/2 + 1 .. m + p/2 with m = floor((y + b)/h - 1/2), shifted inward at
the box edges.  It is exact at grid points.
"""
from __future__ import annotations

import math

import numpy as np

from . import canonical, grid
from .rs import RSTucker


def lagrange_stencil(y: float, b: float, n: int, p: int):
    """(start, weights[p], dweights[p]) of the order-p Lagrange interpolant
    at coordinate y; dweights are d/dy."""
    h = grid.spacing(b, n)
    u = (y + b) / h - 0.5
    m = int(math.floor(u))
    start = min(max(m - p // 2 + 1, 0), n - p)
    nodes = np.arange(start, start + p, dtype=np.float64)
    L = np.empty(p)
    dL = np.empty(p)
    for i in range(p):
        num = 1.0
        den = 1.0
        for j in range(p):
            if j != i:
                num *= (u - nodes[j])
                den *= (nodes[i] - nodes[j])
        L[i] = num / den
        d = 0.0
        for mm in range(p):
            if mm == i:
                continue
            prod = 1.0
            for j in range(p):
                if j != i and j != mm:
                    prod *= (u - nodes[j])
            d += prod
        dL[i] = d / den / h
    return start, L, dL


def long_and_grad(T: RSTucker, points, p: int = 6):
    """P_l(y) and grad P_l(y) from the Tucker factors: interpolate each
    factor's rows, then contract with the core."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    vals = np.empty(points.shape[0])
    grads = np.empty((points.shape[0], 3))
    for m, y in enumerate(points):
        qv, dq = [], []
        for l in range(3):
            s, L, dL = lagrange_stencil(y[l], T.b, T.n, p)
            rows = T.Q[l][s:s + p]
            qv.append(L @ rows)
            dq.append(dL @ rows)
        vals[m] = np.einsum("abc,a,b,c->", T.beta, qv[0], qv[1], qv[2])
        grads[m, 0] = np.einsum("abc,a,b,c->", T.beta, dq[0], qv[1], qv[2])
        grads[m, 1] = np.einsum("abc,a,b,c->", T.beta, qv[0], dq[1], qv[2])
        grads[m, 2] = np.einsum("abc,a,b,c->", T.beta, qv[0], qv[1], dq[2])
    return vals, grads


def eval_points(T: RSTucker, points, part: int = 0, p: int = 6):
    """part 0: long + short, 1: long only, 2: short only."""
    out = 0.0
    if part in (0, 1):
        out = out + long_and_grad(T, points, p)[0]
    if part in (0, 2):
        out = out + canonical.short_range_points(points, T.b, T.n, T.pos, T.q, T.t, T.a,
                                                 T.R_l, T.n_s)
    return out


def gradient_points(T: RSTucker, points, part: int = 0, p: int = 6, normals=None):
    """grad P at the points (section 4.3): the long part as the derivative of
    the order-p interpolant (long_and_grad), the short part analytically per
    windowed term.  part 0: both, 1: long, 2: short.  With normals (M x 3),
    the normal derivatives <grad P(y_i), normals_i> instead."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    g = np.zeros((points.shape[0], 3))
    if part in (0, 1):
        g = g + long_and_grad(T, points, p)[1]
    if part in (0, 2):
        g = g + canonical.short_range_points_grad(points, T.b, T.n, T.pos, T.q, T.t, T.a,
                                                  T.R_l, T.n_s)
    if normals is None:
        return g
    return np.sum(g * np.asarray(normals, dtype=np.float64).reshape(-1, 3), axis=1)


def self_long_and_grad(T: RSTucker, p: int = 6):
    """Particle j's own long-range reference term seen through the same
    interpolation operator, at its own position:
        g_j = sum_{k<R_l} a_k prod_l sum_m L_m(x_jl) exp(-t_k^2 (x_{s+m} - x_jl)^2)
    and its gradient in y (centre held at x_j).  For a particle on a grid
    point the weights are a Kronecker delta and g_j = P_{R_l}(0) exactly,
    which is the self term of eq EnergyFree_Tensor."""
    xs = grid.cell_centres(T.b, T.n)
    N = T.pos.shape[0]
    g = np.zeros(N)
    dg = np.zeros((N, 3))
    for j in range(N):
        phi = np.zeros((T.R_l, 3))
        dphi = np.zeros((T.R_l, 3))
        for l in range(3):
            s, L, dL = lagrange_stencil(T.pos[j, l], T.b, T.n, p)
            nodes = xs[s:s + p]
            for k in range(T.R_l):
                e = np.exp(-T.t[k] ** 2 * (nodes - T.pos[j, l]) ** 2)
                phi[k, l] = L @ e
                dphi[k, l] = dL @ e
        for k in range(T.R_l):
            g[j] += T.a[k] * phi[k, 0] * phi[k, 1] * phi[k, 2]
            dg[j, 0] += T.a[k] * dphi[k, 0] * phi[k, 1] * phi[k, 2]
            dg[j, 1] += T.a[k] * phi[k, 0] * dphi[k, 1] * phi[k, 2]
            dg[j, 2] += T.a[k] * phi[k, 0] * phi[k, 1] * dphi[k, 2]
    return g, dg


def energy(T: RSTucker, p: int = 6, self_term: str = "interp"):
    """E_N by eq EnergyFree_Tensor; also returns dE/dz.

    self_term="paper": subtract z_j^2 P_{R_l}(0) as printed (exact when the
    particles sit on grid points).  self_term="interp": subtract particle j's
    own long-range term through the same interpolation as P_l (reading for
    off-grid particles; identical to "paper" on grid points).
    dE/dz_j = P_l(x_j) - z_j g_j, the derivative of the continuous
    functional evaluated with the discrete field."""
    Pl, _ = long_and_grad(T, T.pos, p)
    if self_term == "paper":
        g = np.full(T.pos.shape[0], T.S_l0)
    else:
        g, _ = self_long_and_grad(T, p)
    dEdq = Pl - T.q * g
    return 0.5 * float(np.sum(T.q * dEdq)), dEdq


def forces(T: RSTucker, p: int = 6):
    """F_j = -dE/dx_j = -z_j grad_y [P_l(y) - z_j g_j(y)] at y = x_j: the
    gradient of the field of all other particles, each particle's own
    (interpolated) term removed."""
    _, gP = long_and_grad(T, T.pos, p)
    _, dg = self_long_and_grad(T, p)
    return -T.q[:, None] * (gP - T.q[:, None] * dg)
