"""Mixed-precision path (split FP16 / split BF16 core and grid expansion, FP32
grid) against the plain FP64 GPU path and the oracle: rel-Linf <= 1e-5 on the
grid, energy error stated and bounded."""
import numpy as np
import pytest

import workloads
from oracle import rs

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
