"""RS-Tucker assembly of the N-particle potential (Definition
RS-Tucker_format):  A = beta x_1 V1 x_2 V2 x_3 V3 + sum_nu z_nu U_nu.

Steps, in the paper's order:
  1. quadrature (t_k, a_k) and split into long k < R_l / short k >= R_l
     (sections 2.2-2.3)
  2. long-range canonical sum of rank R_l N: side matrices and weights
     (eq Long-Range_Sum)
  3. RHOSVD: truncated SVD of the (charge-weighted) side matrices, projection,
     core (Appendix, steps (I)-(II), eqs SVD_SideMatr, alg1, CP_form_RHOSVD)
  4. short-range part as a cumulated canonical tensor of windows
     (Definitions ComCanF, CCT_Uniform)
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import canonical, grid, quadrature, rhosvd


@dataclasses.dataclass
class RSTucker:
    b: float
    n: int
    t: np.ndarray
    a: np.ndarray
    R_l: int
    n_s: int
    pos: np.ndarray
    q: np.ndarray
    Q: List[np.ndarray]
    beta: np.ndarray
    sigma: List[np.ndarray]
    ranks: List[int]

    @property
    def h(self) -> float:
        return grid.spacing(self.b, self.n)

    @property
    def S_l0(self) -> float:
        """P_{R_l}(x = 0): the long-range reference tensor at the origin."""
        return float(np.sum(self.a[:self.R_l]))

    def long_at(self, idx3):
        return rhosvd.tucker_at(self.beta, self.Q, idx3)

    def short_at(self, idx3):
        return canonical.short_range_at(idx3, self.b, self.n, self.pos, self.q, self.t,
                                        self.a, self.R_l, self.n_s)

    def at(self, idx3):
        """Entries of the RS-Tucker tensor at grid indices (Lemma
        Property_RST_Tuck)."""
        return self.long_at(idx3) + self.short_at(idx3)

    def long_grid(self):
        return rhosvd.tucker_full(self.beta, self.Q)

    def short_grid(self):
        return canonical.short_range_grid(self.b, self.n, self.pos, self.q, self.t, self.a,
                                          self.R_l, self.n_s)

    def full_grid(self):
        return self.long_grid() + self.short_grid()


def table_for(kernel: str, R: int, lam: float = 0.5):
    return quadrature.literal_table(kernel, R, lam)


def assemble(b: float, n: int, pos, q, t, a, R_l: int, n_s: int, eps: float,
             r_max: Optional[int] = None, fixed_ranks: Optional[Sequence[int]] = None,
             core_chunk: Optional[int] = None) -> RSTucker:
    """core_chunk: sum the core over blocks of that many terms j
    (rhosvd.core_chunked) instead of one contraction, for large K and ranks."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if r_max is None:
        r_max = n
    t_long, a_long = t[:R_l], a[:R_l]
    U = rhosvd.side_matrices(b, n, pos, t_long)
    xi = rhosvd.canonical_weights(q, a_long)
    w = rhosvd.gram_weights(xi)
    Qs, sig, ranks = [], [], []
    for l in range(3):
        Ql, s, r = rhosvd.mode_basis(U[l], w, eps, r_max,
                                     None if fixed_ranks is None else fixed_ranks[l])
        Qs.append(Ql)
        sig.append(s)
        ranks.append(r)
    Ut = [rhosvd.project(Qs[l], U[l]) for l in range(3)]
    beta = rhosvd.core(Ut, xi) if core_chunk is None else rhosvd.core_chunked(Ut, xi, core_chunk)
    return RSTucker(b, n, np.asarray(t), np.asarray(a), R_l, n_s, pos, q, Qs, beta, sig, ranks)


def assemble_system(sys, fixed_ranks=None, r_max=None, n_s=None, core_chunk=None) -> RSTucker:
    """Assemble a workloads.System with the paper-literal table; the window
    width is the system's, or derived by criterion (A) when it gives none."""
    t, a = quadrature.literal_table(sys.kernel, sys.R, sys.lam)
    if n_s is None:
        n_s = sys.n_s
    if n_s is None:
        n_s = quadrature.derive_window(t, a, sys.R_l, sys.delta_rel, grid.spacing(sys.b, sys.n))
    return assemble(sys.b, sys.n, sys.pos, sys.q, t, a, sys.R_l, n_s, sys.eps_tucker,
                    r_max=r_max, fixed_ranks=fixed_ranks, core_chunk=core_chunk)
