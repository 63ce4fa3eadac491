"""Mixed-precision path (split FP16 / split BF16 core and grid expansion, FP32
grid) against the plain FP64 GPU path and the oracle: rel-Linf <= 1e-5 on the
grid, energy error stated and bounded."""
import numpy as np
import pytest

import workloads
from oracle import pointeval, rs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def rsm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1606_09218_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(rsm):
    return rsm.Context(0)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def run(rsm, ctx, s, prec, ranks):
    f = rsm.Factors(ctx, s.b, s.n, s.R, s.R_l, s.n_s if s.n_s else -1)
    dt = torch.float64 if prec == "fp64" else torch.float32
    g = torch.empty(s.n ** 3, dtype=dt, device="cuda")
    T = rsm.assemble(ctx, f, dev(s.pos), dev(s.q), g, rsm.make_aopts(s.eps_tucker, fixed_ranks=ranks, prec=prec))
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    rsm.energy(T, E)
    torch.cuda.synchronize()
    return g.double().cpu().numpy(), E.item()


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "ragged"])
@pytest.mark.parametrize("prec", ["mixed_fp16", "mixed_bf16"])
def test_mixed_matches_fp64(rsm, ctx, name, prec):
    if name == "cfg1":
        s = workloads.cfg1_plain_small()
    elif name == "cfg2":
        s = workloads.cfg2_lattice()
    else:
        s = workloads.tiny_system(91, 25, 6.0, 72, 24, 10, 11, min_sep=0.6)
    ref = rs.assemble_system(s) if s.n <= 128 else None
    ranks = ref.ranks if ref is not None else [89, 89, 89]
    g64, E64 = run(rsm, ctx, s, "fp64", ranks)
    gmx, Emx = run(rsm, ctx, s, prec, ranks)
    err = float(np.max(np.abs(gmx - g64)) / np.max(np.abs(g64)))
    e_err = abs(Emx - E64) / abs(E64)
    say(f"{name} {prec}: grid rel-Linf vs FP64 {err:.2e}, energy rel {e_err:.2e}")
    assert err <= TOL
    assert e_err <= 1e-5
    if ref is not None:
        full = ref.full_grid().ravel()
        err_o = float(np.max(np.abs(gmx - full)) / np.max(np.abs(full)))
        say(f"   vs oracle {err_o:.2e}")
        assert err_o <= TOL


@pytest.mark.parametrize("ranks", [[12, 10, 8], [40, 33, 20], [70, 50, 19], [100, 64, 40]])
@pytest.mark.parametrize("prec", ["mixed_fp16", "mixed_bf16"])
def test_mixed_core_tile_shapes(rsm, ctx, ranks, prec):
    """The split core at ranks that pick each row-tile height (r1 = 12, 40:
    64-row tiles; 70: 96; 100: 128) and both ways of staging the Khatri-Rao
    factor rows (r3 = 8: a 128-column tile spans 17 b rows, more than the
    8 staged by the common kernel; r3 = 19, 20, 40: within 8), against the
    FP64 path at the same ranks and the oracle."""
    s = workloads.tiny_system(93, 30, 6.0, 104, 24, 10, 9, min_sep=0.6)
    ref = rs.assemble_system(s, fixed_ranks=ranks)
    g64, E64 = run(rsm, ctx, s, "fp64", ranks)
    gmx, Emx = run(rsm, ctx, s, prec, ranks)
    err = float(np.max(np.abs(gmx - g64)) / np.max(np.abs(g64)))
    full = ref.full_grid().ravel()
    err_o = float(np.max(np.abs(gmx - full)) / np.max(np.abs(full)))
    # the energy of 30 random charges nearly cancels, so its error is bounded
    # on its own scale: 1/2 sum_j |z_j| max_j |dE/dz_j| (dE/dz_j = P_l(x_j) -
    # z_j g_j), the bound a field error of 1e-5 of its maximum gives
    _, dEdq = pointeval.energy(ref)
    e_scale = 0.5 * float(np.sum(np.abs(s.q))) * float(np.max(np.abs(dEdq)))
    e_err = abs(Emx - E64) / e_scale
    say(f"ranks {ranks} {prec}: vs FP64 {err:.2e}, energy {abs(Emx - E64) / abs(E64):.2e} "
        f"relative, {e_err:.2e} of its scale, vs oracle {err_o:.2e}")
    assert err <= TOL and err_o <= TOL
    assert e_err <= 1e-5
