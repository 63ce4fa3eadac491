"""Pairwise interaction energies and forces, O(N^2) (eq EnergyLatSum,
section 4.2; forces, section 4.3).

E = 1/2 sum_j z_j sum_{k != j} z_k f(|x_j - x_k|) for f = p (exact kernel) or
f = S_K (a subset K of the Gaussian sum, e.g. the long-range part).
F_j = -dE/dx_j = -z_j sum_{k != j} z_k f'(r_jk) (x_j - x_k)/r_jk.
The force formula printed in section 4.3 carries a spurious factor 1/2; the
expression above is the derivative of eq EnergyLatSum.
"""
from __future__ import annotations

import numpy as np

from . import quadrature


def _pair_loop(pos, q, f, df, want_forces: bool, chunk: int = 256):
    N = pos.shape[0]
    E = 0.0
    F = np.zeros((N, 3)) if want_forces else None
    for s in range(0, N, chunk):
        d = pos[s:s + chunk, None, :] - pos[None, :, :]      # x_j - x_k
        r = np.sqrt(np.sum(d * d, axis=2))
        idx = np.arange(s, min(s + chunk, N))
        r[np.arange(idx.size), idx] = 1.0                   # placeholder for k == j
        mask = np.ones_like(r)
        mask[np.arange(idx.size), idx] = 0.0
        zz = q[s:s + chunk, None] * q[None, :] * mask
        E += 0.5 * float(np.sum(zz * f(r)))
        if want_forces:
            F[s:s + chunk] = -np.sum((zz * df(r) / r)[:, :, None] * d, axis=1)
    return E, F


def energy_exact(pos, q, kernel: str = "newton", lam: float = 0.5, forces: bool = False):
    return _pair_loop(np.asarray(pos), np.asarray(q),
                      lambda r: quadrature.kernel_value(kernel, r, lam),
                      lambda r: quadrature.kernel_derivative(kernel, r, lam), forces)


def energy_canonical(pos, q, t, a, ks, forces: bool = False):
    ks = list(ks)
    return _pair_loop(np.asarray(pos), np.asarray(q),
                      lambda r: quadrature.kernel_sum(r, t, a, ks),
                      lambda r: quadrature.kernel_sum_derivative(r, t, a, ks), forces)
