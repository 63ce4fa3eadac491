"""The discrete gradient on the whole grid (section 4.3, eq Gradients_Tens)
through the C ABI against the oracle's finite differences of the full RS
grid: rel-Linf <= 1e-6 for FP64 tensors, 1e-5 for the mixed and FP32
contractions (both relative to the largest entry of the oracle's gradient)."""
import sys

import numpy as np
import pytest

import workloads
from oracle import gradient, rs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


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


def assemble(rsm, ctx, s, ranks, prec="fp64"):
    f = rsm.Factors(ctx, s.b, s.n, s.R, s.R_l, s.n_s)
    T = rsm.assemble(ctx, f, dev(s.pos), dev(s.q), None,
                     rsm.make_aopts(s.eps_tucker, fixed_ranks=ranks, prec=prec))
    return f, T


def gpu_gradient(rsm, T, n, axis, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    g = torch.full((n ** 3,), float("nan"), dtype=dt, device="cuda")
    rsm.gradient_grid(T, axis, g)
    torch.cuda.synchronize()
    return g.double().cpu().numpy().reshape(n, n, n)


CASES = [
    dict(seed=11, N=12, b=5.0, n=32, R=20, R_l=8, n_s=7, box=0.6),
    dict(seed=12, N=7, b=4.0, n=40, R=20, R_l=8, n_s=9, box=0.6),     # n not a multiple of 8
    dict(seed=13, N=1, b=3.0, n=24, R=16, R_l=6, n_s=5, box=0.6),     # one particle
    dict(seed=14, N=30, b=6.0, n=48, R=24, R_l=10, n_s=1, box=0.6),   # window of one cell
    dict(seed=15, N=9, b=5.0, n=66, R=20, R_l=8, n_s=65, box=0.6),    # window wider than a brick
    dict(seed=16, N=20, b=4.0, n=36, R=20, R_l=8, n_s=9, box=0.99),   # windows cut by the grid's faces
]


@pytest.mark.parametrize("case", CASES)
def test_gradient_grid_parity_fp64(rsm, ctx, case):
    s = workloads.tiny_system(case["seed"], case["N"], case["b"], case["n"], case["R"],
                              case["R_l"], case["n_s"], min_sep=0.3, box_frac=case["box"])
    say(f"gradient parity {s.name} n_s={s.n_s}")
    ref = rs.assemble_system(s)
    f, T = assemble(rsm, ctx, s, ref.ranks)
    for axis in range(3):
        want = gradient.gradient_grid(ref, axis)
        got = gpu_gradient(rsm, T, s.n, axis, "fp64")
        err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
        say(f"  axis {axis} rel-Linf {err:.2e}")
        assert np.all(np.isfinite(got))
        assert err <= 1e-6


@pytest.mark.parametrize("prec", ["mixed_fp16", "mixed_bf16", "fp32"])
def test_gradient_grid_parity_reduced(rsm, ctx, prec):
    s = workloads.tiny_system(21, 40, 6.0, 72, 24, 10, 11, min_sep=0.6, box_frac=0.9)
    say(f"gradient parity {s.name} {prec}")
    ref = rs.assemble_system(s)
    f, T = assemble(rsm, ctx, s, ref.ranks, prec=prec)
    for axis in range(3):
        want = gradient.gradient_grid(ref, axis)
        got = gpu_gradient(rsm, T, s.n, axis, prec)
        err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
        say(f"  axis {axis} rel-Linf {err:.2e}")
        assert err <= 1e-5


def test_gradient_grid_cfg1_and_bad_axis(rsm, ctx):
    s = workloads.cfg1_plain_small()
    say(f"gradient parity {s.name}")
    ref = rs.assemble_system(s)
    f, T = assemble(rsm, ctx, s, ref.ranks)
    want = gradient.gradient_grid(ref, 1)
    got = gpu_gradient(rsm, T, s.n, 1, "fp64")
    err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    say(f"  axis 1 rel-Linf {err:.2e}")
    assert err <= 1e-6
    g = torch.empty(s.n ** 3, dtype=torch.float64, device="cuda")
    for axis in (-1, 3):
        with pytest.raises(rsm.RSError):
            rsm.gradient_grid(T, axis, g)
