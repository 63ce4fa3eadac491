"""Protein-like cloud (N = 10000 charges in 40 Gaussian blobs, n = 1024,
R = 32, R_l = 12, window by criterion (A)) at full size.

The oracle's core (rank ~340 over K = 120000 terms) is out of reach on the
CPU, so the FP64 grid is compared with the oracle's RS-Tucker tensor at the
same ranks on a sampled set through the projected canonical sum (no core
needed): a random 48^3 tensor-product sub-grid, the full windows of 32
particles and the three central axis lines, rel-Linf <= 1e-6.  Also:
- long-range part at cell centres vs the canonical long-range sum
  (Definition of the long-range part): Tucker truncation only;
- short-range part at random points vs the oracle's windowed sum: exact up
  to rounding;
- mixed FP16 / BF16 grid and energy vs FP64, rel-Linf <= 1e-5.
"""
import numpy as np
import pytest

import workloads
from oracle import canonical, grid as ogrid, quadrature, rhosvd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1606_09218_amd as rsm
    ctx = rsm.Context(0)
    s = workloads.cfg3_protein_like()
    f = rsm.Factors(ctx, s.b, s.n, s.R, s.R_l, -1, delta_rel=s.delta_rel)
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    q = torch.tensor(s.q, dtype=torch.float64, device="cuda")
    return rsm, ctx, s, f, pos, q


def test_cfg3_fp64_against_canonical_sums(setup):
    rsm, ctx, s, f, pos, q = setup
    say(f"cfg3: N={s.N} n={s.n} R={s.R} R_l={s.R_l} n_s={f.n_s}")
    T = rsm.assemble(ctx, f, pos, q, None, rsm.make_aopts(s.eps_tucker, r_max=400))
    ranks = list(T.info().ranks)
    say(f"cfg3 ranks {ranks}")
    assert all(60 <= r <= 400 for r in ranks)
    rng = np.random.default_rng(33)
    t = np.array(f.t)
    a = np.array(f.a)
    # long range at cell centres (exact grid values of the Tucker part)
    idx = rng.integers(0, s.n, size=(600, 3))
    xc = ogrid.cell_centres(s.b, s.n)
    pts = xc[idx]
    vals = torch.empty(pts.shape[0], dtype=torch.float64, device="cuda")
    rsm.eval_points(T, torch.tensor(pts, device="cuda"), vals, part=1)
    got = vals.cpu().numpy()
    ref = canonical.canonical_potential_radial(pts, s.pos, s.q, t, a, ks=range(s.R_l))
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say(f"cfg3 long range vs canonical long sum at 600 cell centres: rel-Linf {err:.2e}")
    assert err <= 1e-4
    # short range at random points vs the windowed oracle sum
    pts2 = rng.uniform(-s.b, s.b, size=(600, 3))
    near = s.pos[rng.integers(0, s.N, 200)] + rng.normal(0, 0.3, (200, 3))
    pts2 = np.clip(np.vstack([pts2, near]), -s.b + 1e-9, s.b - 1e-9)
    vals2 = torch.empty(pts2.shape[0], dtype=torch.float64, device="cuda")
    rsm.eval_points(T, torch.tensor(pts2, device="cuda"), vals2, part=2)
    ref2 = canonical.short_range_points(pts2, s.b, s.n, s.pos, s.q, t, a, s.R_l, f.n_s)
    err2 = np.max(np.abs(vals2.cpu().numpy() - ref2)) / max(np.max(np.abs(ref2)), 1e-300)
    say(f"cfg3 short range vs windowed oracle sum at 800 points: rel-Linf {err2:.2e}")
    assert err2 <= 1e-10
    T.free()


@pytest.mark.parametrize("prec", ["mixed_fp16", "mixed_bf16"])
def test_cfg3_mixed_matches_fp64(setup, prec):
    rsm, ctx, s, f, pos, q = setup
    g64 = torch.empty(s.n ** 3, dtype=torch.float64, device="cuda")
    T = rsm.assemble(ctx, f, pos, q, g64, rsm.make_aopts(s.eps_tucker, r_max=400))
    ranks = list(T.info().ranks)
    E64 = torch.empty(1, dtype=torch.float64, device="cuda")
    rsm.energy(T, E64)
    T.free()
    # the same options: the eigen stage is FP64 in both paths, so the ranks
    # and bases agree and only the split-precision contractions differ
    g32 = torch.empty(s.n ** 3, dtype=torch.float32, device="cuda")
    Tm = rsm.assemble(ctx, f, pos, q, g32, rsm.make_aopts(s.eps_tucker, r_max=400, prec=prec))
    assert list(Tm.info().ranks) == ranks
    Em = torch.empty(1, dtype=torch.float64, device="cuda")
    rsm.energy(Tm, Em)
    torch.cuda.synchronize()
    gmax = g64.abs().max().item()
    diff = 0.0
    chunk = 1 << 26
    for c0 in range(0, g64.numel(), chunk):
        d = (g32[c0:c0 + chunk].double() - g64[c0:c0 + chunk]).abs().max().item()
        diff = max(diff, d)
    err = diff / gmax
    e_err = abs(Em.item() - E64.item()) / abs(E64.item())
    say(f"cfg3 {prec}: ranks {ranks}, grid rel-Linf vs FP64 {err:.2e}, energy rel err {e_err:.2e}")
    assert err <= 1e-5
    assert e_err <= 1e-5
    Tm.free()
    del g64, g32


def test_cfg3_fp64_grid_sampled_parity(setup):
    """The FP64 grid at n = 1024 (ranks ~340: the tiled core and the
    32-column panel of the grid expansion) against the oracle's RS-Tucker
    tensor at the same ranks, on the sampled set."""
    rsm, ctx, s, f, pos, q = setup
    T0 = rsm.assemble(ctx, f, pos, q, None, rsm.make_aopts(s.eps_tucker, r_max=400))
    ranks = list(T0.info().ranks)
    T0.free()
    t, a = np.array(f.t), np.array(f.a)
    U = rhosvd.side_matrices(s.b, s.n, s.pos, t[:s.R_l])
    xi = rhosvd.canonical_weights(s.q, a[:s.R_l])
    w = rhosvd.gram_weights(xi)
    Qs, Ut = [], []
    for l in range(3):
        # the SVD of the weighted side matrix itself (the oracle's own basis)
        Q, sig, _ = rhosvd.mode_basis(U[l], w, s.eps_tucker, s.n, ranks[l])
        Qs.append(Q)
        Ut.append(rhosvd.project(Q, U[l]))
        say(f"cfg3 oracle mode {l}: rank {ranks[l]}, sigma_r/sigma_1 {sig[ranks[l] - 1] / sig[0]:.2e}, "
            f"sigma_r+1/sigma_1 {sig[ranks[l]] / sig[0]:.2e}")
    del U
    W = rhosvd.projected_side_matrices(Qs, Ut)
    del Ut
    g = torch.empty(s.n ** 3, dtype=torch.float64, device="cuda")
    T = rsm.assemble(ctx, f, pos, q, g, rsm.make_aopts(s.eps_tucker, fixed_ranks=ranks))
    assert list(T.info().ranks) == ranks
    torch.cuda.synchronize()
    rng = np.random.default_rng(303)
    sets = [[np.sort(rng.choice(s.n, 48, replace=False)) for _ in range(3)]]
    lo, hi = canonical.window_bounds(s.pos[rng.choice(s.N, 32, replace=False)], s.b, s.n, f.n_s)
    sets += [[np.arange(lo[m, l], hi[m, l] + 1) for l in range(3)] for m in range(lo.shape[0])]
    c, ax = np.array([s.n // 2]), np.arange(s.n)
    sets += [[ax, c, c], [c, ax, c], [c, c, ax]]
    worst, scale, count = 0.0, 0.0, 0
    for I in sets:
        ref = rhosvd.tucker_subgrid_projected(None, None, xi, *I, W=W)
        ref += canonical.short_range_subgrid(*I, s.b, s.n, s.pos, s.q, t, a, s.R_l, f.n_s)
        flat = ((I[0][:, None, None] * s.n + I[1][None, :, None]) * s.n + I[2][None, None, :]).ravel()
        got = g[torch.tensor(flat, device="cuda")].cpu().numpy().reshape(ref.shape)
        worst = max(worst, float(np.max(np.abs(got - ref))))
        scale = max(scale, float(np.max(np.abs(ref))))
        count += ref.size
    err = worst / scale
    say(f"cfg3 FP64 grid vs oracle at ranks {ranks} on {count} sampled points: rel-Linf {err:.2e} "
        f"({err / 1e-6:.2f} of the 1e-6 tolerance)")
    assert err <= 1e-6
    T.free()
    del g
