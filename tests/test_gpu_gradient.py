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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_point_gradient_and_normal_derivative_parity(rsm, ctx, prec):
    """rs_eval_gradient_points against the oracle at random points (every
    part), with and without normals: rel-Linf <= 1e-8 in FP64 (the same
    arithmetic on both sides), 1e-5 for the FP32 field contraction."""
    from oracle import pointeval
    s = workloads.tiny_system(31, 50, 6.0, 64, 24, 10, 11, min_sep=0.5, box_frac=0.8)
    say(f"point gradient parity {s.name} {prec}")
    ref = rs.assemble_system(s)
    f, T = assemble(rsm, ctx, s, ref.ranks, prec=prec)
    rng = np.random.default_rng(32)
    M = 257
    P = rng.uniform(-0.95 * s.b, 0.95 * s.b, size=(M, 3))
    P[:20] = s.pos[:20] + rng.normal(scale=0.05, size=(20, 3))   # inside windows
    nrm = rng.normal(size=(M, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    tol = 1e-8 if prec == "fp64" else 1e-5
    for part in (0, 1, 2):
        want = pointeval.gradient_points(ref, P, part=part)
        got = torch.empty(M * 3, dtype=torch.float64, device="cuda")
        rsm.eval_gradient_points(T, dev(P), got, part=part)
        dn = torch.empty(M, dtype=torch.float64, device="cuda")
        rsm.eval_gradient_points(T, dev(P), dn, normals=dev(nrm), part=part)
        torch.cuda.synchronize()
        got = got.cpu().numpy().reshape(M, 3)
        err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
        want_n = np.sum(want * nrm, axis=1)
        err_n = float(np.max(np.abs(dn.cpu().numpy() - want_n)) / np.max(np.abs(want_n)))
        say(f"  part {part} grad rel-Linf {err:.2e} normal {err_n:.2e}")
        assert err <= tol and err_n <= tol
    # M = 0 is a no-op
    rsm.eval_gradient_points(T, torch.empty(0, dtype=torch.float64, device="cuda"),
                             torch.empty(0, dtype=torch.float64, device="cuda"))
