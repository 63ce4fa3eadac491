"""Long-range part: side matrices, charge-weighted Gram, reduced HOSVD
(RHOSVD) basis, core tensor and Tucker reconstruction.

Section 3.2 (eq Long-Range_Sum: the long-range sum is a canonical tensor of
rank R_l N), section 2.1 (eqs CP_form_ContrpTuck, Tucker_form, Tucker_CS) and
the Appendix (eqs SVD_SideMatr, CP_form_RHOSVD, alg1: SVD of the side
matrices, truncation, projection, core).

Column ordering: j = k * N + nu  (k = long-range quadrature index,
nu = particle).  Canonical weights xi_j = z_nu a_k.

Reading of "charge-weighted": the side matrix of mode l is scaled column-wise
by |xi_j|^{1/3} before its SVD, i.e. the weighted Gram is
G_l = U_l diag(|xi|^{2/3}) U_l^T.  This spreads each term's magnitude evenly
over the three modes; it is scale covariant and gives the same basis for z
and -z.  Rank rule: keep sigma_k > eps * sigma_1, capped at r_max.
"""
from __future__ import annotations

import numpy as np

from . import grid as _grid


def side_matrix(b: float, n: int, coords, t_long) -> np.ndarray:
    """U_l[i, k*N + nu] = exp(-t_k^2 (x_i - x_{nu,l})^2), an n x (R_l N)
    matrix of collocated 1D Gaussians (eq Long-Range_Sum, cell-centre
    collocation)."""
    x = _grid.cell_centres(b, n)
    coords = np.asarray(coords, dtype=np.float64)
    cols = []
    for tk in t_long:
        cols.append(np.exp(-tk ** 2 * (x[:, None] - coords[None, :]) ** 2))
    return np.concatenate(cols, axis=1)


def side_matrices(b: float, n: int, pos, t_long):
    return [side_matrix(b, n, pos[:, l], t_long) for l in range(3)]


def canonical_weights(q, a_long) -> np.ndarray:
    """xi[k*N + nu] = z_nu a_k."""
    return np.concatenate([q * ak for ak in a_long])


def gram_weights(xi) -> np.ndarray:
    return np.abs(xi) ** (2.0 / 3.0)


def weighted_gram(U, w) -> np.ndarray:
    """G = U diag(w) U^T by a plain matrix product."""
    return (U * w[None, :]) @ U.T


def weighted_gram_gaussian_product(b: float, n: int, coords, t_long, w) -> np.ndarray:
    """The same Gram through the Gaussian product identity
    exp(-t^2 (x-X)^2) exp(-t^2 (x'-X)^2)
        = exp(-t^2 (x-x')^2 / 2) exp(-2 t^2 ((x+x')/2 - X)^2),
    an independent O(n N R_l + n^2 R_l) route used to cross-check G."""
    x = _grid.cell_centres(b, n)
    N = len(coords)
    G = np.zeros((n, n))
    diff2 = (x[:, None] - x[None, :]) ** 2
    mid = 0.5 * (x[:, None] + x[None, :])
    for k, tk in enumerate(t_long):
        wk = w[k * N:(k + 1) * N]
        s = np.zeros((n, n))
        for nu in range(N):
            s += wk[nu] * np.exp(-2.0 * tk ** 2 * (mid - coords[nu]) ** 2)
        G += np.exp(-0.5 * tk ** 2 * diff2) * s
    return G


def canonical_signs(Q) -> np.ndarray:
    """Flip each column so that its entry of largest magnitude (first one on
    ties) is positive."""
    Q = np.array(Q, copy=True)
    for c in range(Q.shape[1]):
        i = int(np.argmax(np.abs(Q[:, c])))
        if Q[i, c] < 0:
            Q[:, c] = -Q[:, c]
    return Q


def select_rank(sigma, eps: float, r_max: int) -> int:
    """r = #{k : sigma_k > eps * sigma_1}, capped at r_max (Appendix step (I):
    discard singular vectors below the rank threshold)."""
    if sigma.size == 0 or sigma[0] <= 0:
        return 0
    return int(min(int(np.sum(sigma > eps * sigma[0])), r_max))


def mode_basis(U, w, eps: float, r_max: int, fixed_rank=None):
    """Dominant left singular vectors of the weighted side matrix
    U diag(w^{1/2}) (eq SVD_SideMatr, truncated as in Definition RHOSVD).
    Returns (Q n x r with canonical signs, all singular values, r)."""
    A = U * np.sqrt(w)[None, :]
    Z, sigma, _ = np.linalg.svd(A, full_matrices=False)
    r = select_rank(sigma, eps, r_max) if fixed_rank is None else int(fixed_rank)
    return canonical_signs(Z[:, :r]), sigma, r


def project(Q, U) -> np.ndarray:
    """U~ = Q^T U, the side matrix in the reduced basis (eq alg1)."""
    return Q.T @ U


def core(Ut, xi) -> np.ndarray:
    """beta = sum_j xi_j u~1_j (x) u~2_j (x) u~3_j: the RHOSVD core
    (eq CP_form_RHOSVD: xi x_1 U~1 x_2 U~2 x_3 U~3)."""
    return np.einsum("aj,bj,cj->abc", Ut[0] * xi[None, :], Ut[1], Ut[2], optimize=True)


def tucker_full(beta, Q) -> np.ndarray:
    """beta x_1 Q1 x_2 Q2 x_3 Q3 on the full grid (eq Tucker_CS)."""
    return np.einsum("abc,ia,jb,kc->ijk", beta, Q[0], Q[1], Q[2], optimize=True)


def tucker_at(beta, Q, idx3) -> np.ndarray:
    """Entries of the Tucker tensor at grid indices (Lemma Property_RST_Tuck:
    a_i = beta x_1 v1_{i1} x_2 v2_{i2} x_3 v3_{i3})."""
    idx3 = np.asarray(idx3, dtype=np.int64).reshape(-1, 3)
    out = np.empty(idx3.shape[0])
    for m, (i1, i2, i3) in enumerate(idx3):
        out[m] = np.einsum("abc,a,b,c->", beta, Q[0][i1], Q[1][i2], Q[2][i3])
    return out


def canonical_full(U, xi) -> np.ndarray:
    """The long-range canonical tensor sum_j xi_j u1_j (x) u2_j (x) u3_j on
    the full grid (small n only)."""
    return np.einsum("ij,kj,lj,j->ikl", U[0], U[1], U[2], xi, optimize=True)


def unfolding_singular_values(T, mode: int) -> np.ndarray:
    """Singular values of the mode-l unfolding of a dense tensor (the full
    HOSVD of the Appendix, brute force, small n only)."""
    M = np.moveaxis(T, mode, 0).reshape(T.shape[mode], -1)
    return np.linalg.svd(M, compute_uv=False)


def mode_basis_eigh(G, eps: float, r_max: int, fixed_rank=None):
    """The same basis through the weighted Gram G = U diag(w) U^T (eq
    SVD_SideMatr: the left singular vectors of U diag(w^{1/2}) are the
    eigenvectors of G, sigma_k^2 its eigenvalues).  Used where the SVD of an
    n x K side matrix is too slow (K ~ 1e5).  Returns (Q n x r with canonical
    signs, singular values sqrt(max(lambda, 0)) in descending order, r)."""
    lam, Z = np.linalg.eigh(G)
    order = np.argsort(lam)[::-1]
    lam, Z = lam[order], Z[:, order]
    sigma = np.sqrt(np.maximum(lam, 0.0))
    r = select_rank(sigma, eps, r_max) if fixed_rank is None else int(fixed_rank)
    return canonical_signs(Z[:, :r]), sigma, r


def core_chunked(Ut, xi, chunk: int = 512) -> np.ndarray:
    """beta = sum_j xi_j u~1_j (x) u~2_j (x) u~3_j (eq CP_form_RHOSVD) summed
    over consecutive blocks of j, so that the intermediate of the contraction
    stays small for large K."""
    K = xi.shape[0]
    beta = np.zeros((Ut[0].shape[0], Ut[1].shape[0], Ut[2].shape[0]))
    for j0 in range(0, K, chunk):
        js = slice(j0, min(j0 + chunk, K))
        beta += np.einsum("aj,bj,cj->abc", Ut[0][:, js] * xi[None, js], Ut[1][:, js],
                          Ut[2][:, js], optimize=True)
    return beta


def projected_side_matrices(Q, Ut):
    """W_l = Q_l U~_l = Q_l Q_l^T U_l (n x K): the side matrices projected on
    the Tucker bases (the factors of the projected canonical sum)."""
    return [Q[l] @ Ut[l] for l in range(3)]


def tucker_subgrid_projected(Q, Ut, xi, I1, I2, I3, chunk: int = 2048, W=None) -> np.ndarray:
    """Values of the Tucker tensor beta x_1 Q1 x_2 Q2 x_3 Q3, beta the RHOSVD
    core of the canonical sum (xi, U), on the index set I1 x I2 x I3, through
    the projected canonical sum
        A(i) = sum_j xi_j (Q1 u~1_j)(i1) (Q2 u~2_j)(i2) (Q3 u~3_j)(i3)
    (eqs CP_form_RHOSVD and Tucker_CS with the sum over j taken last), which
    needs no core: for K ~ 1e5 and ranks ~ 300 the core itself is out of
    reach on the CPU.  W: projected_side_matrices(Q, Ut) when already
    formed (then Q and Ut are not read).  Result: |I1| x |I2| x |I3|."""
    idx = [np.asarray(I, dtype=np.int64) for I in (I1, I2, I3)]
    if W is None:
        W = [Q[l][idx[l]] @ Ut[l] for l in range(3)]     # |I_l| x K: rows of Q_l Q_l^T U_l
    else:
        W = [W[l][idx[l]] for l in range(3)]
    K = xi.shape[0]
    out = np.zeros((len(idx[0]) * len(idx[1]), len(idx[2])))
    for j0 in range(0, K, chunk):
        js = slice(j0, min(j0 + chunk, K))
        kr = (W[0][:, None, js] * W[1][None, :, js]).reshape(-1, js.stop - js.start)
        out += (kr * xi[None, js]) @ W[2][:, js].T
    return out.reshape(len(idx[0]), len(idx[1]), len(idx[2]))
