"""ALS refinement of the RHOSVD Tucker approximation (Appendix, steps (III)
to (V) of the canonical-to-Tucker algorithm, eq alg2).  TEST INFRASTRUCTURE
ONLY (see the package header).

Starting from the RHOSVD bases Q_l (n x r_l), one sweep updates l = 1, 2, 3
in turn: the partially projected image of the canonical tensor,
    M_l = U_l diag(xi) (U~_m (.) U~_p)^T        (n x r_m r_p, eq alg2),
with U~ = Q^T U for the two other modes (the Khatri-Rao product taken per
column j), is reduced to its r_l dominant left singular vectors, which
replace Q_l (and U~_l).  After the sweeps the core is the projection of the
last image, beta = sum_j xi_j u~1_j (x) u~2_j (x) u~3_j (step (V)).
Each sweep is one round of higher-order orthogonal iteration on the
canonical tensor, done without forming it.
"""
from __future__ import annotations

import numpy as np

from . import rhosvd


def partial_image(U, xi, Ut, mode: int) -> np.ndarray:
    """M_mode = U_mode diag(xi) (U~_m (.) U~_p)^T with m < p the other two
    modes, as an n x (r_m r_p) matrix (column index (b, c) with c fastest)."""
    m, p = [l for l in range(3) if l != mode]
    return np.einsum("ij,j,bj,cj->ibc", U[mode], xi, Ut[m], Ut[p], optimize=True).reshape(
        U[mode].shape[0], -1)


def refine(U, xi, Q0, sweeps: int):
    """C2T steps (III)-(V) from the bases Q0 (ranks fixed by their columns).
    Returns (Q, beta, core_norms): core_norms[s] = ||beta|| after sweep s
    (index 0: the RHOSVD core)."""
    Q = [np.array(q, dtype=np.float64) for q in Q0]
    Ut = [rhosvd.project(Q[l], U[l]) for l in range(3)]
    norms = [float(np.linalg.norm(rhosvd.core(Ut, xi)))]
    for _ in range(sweeps):
        for l in range(3):
            M = partial_image(U, xi, Ut, l)
            Z, _, _ = np.linalg.svd(M, full_matrices=False)
            Q[l] = rhosvd.canonical_signs(Z[:, :Q[l].shape[1]])
            Ut[l] = rhosvd.project(Q[l], U[l])
        norms.append(float(np.linalg.norm(rhosvd.core(Ut, xi))))
    return Q, rhosvd.core(Ut, xi), norms
