"""ALS refinement of the RHOSVD Tucker approximation (Appendix, steps (III)
to (V), eq alg2) through the C ABI: the refined grid against the oracle's
refinement from its own RHOSVD bases at the same ranks (rel-Linf 1e-6: the
two start from bases that agree to the subspace accuracy), the Tucker error
against the exact canonical long-range tensor no larger than without the
refinement, and the mixed-precision refinement against the FP64 one."""
import sys

import numpy as np
import pytest

import workloads
from oracle import als, quadrature, rhosvd, rs

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


def run(rsm, ctx, s, ranks, sweeps, prec="fp64"):
    f = rsm.Factors(ctx, s.b, s.n, s.R, s.R_l, s.n_s)
    dt = torch.float64 if prec == "fp64" else torch.float32
    g = torch.empty(s.n ** 3, dtype=dt, device="cuda")
    T = rsm.assemble(ctx, f, dev(s.pos), dev(s.q), g,
                     rsm.make_aopts(s.eps_tucker, fixed_ranks=ranks, prec=prec, als_sweeps=sweeps))
    torch.cuda.synchronize()
    return f, T, g.double().cpu().numpy().reshape((s.n,) * 3)


def oracle_refined(s, ranks, sweeps):
    t, a = quadrature.literal_table(s.kernel, s.R, s.lam)
    U = rhosvd.side_matrices(s.b, s.n, s.pos, t[:s.R_l])
    xi = rhosvd.canonical_weights(s.q, a[:s.R_l])
    w = rhosvd.gram_weights(xi)
    Q0 = [rhosvd.mode_basis(U[l], w, 0.0, s.n, ranks[l])[0] for l in range(3)]
    Q, beta, norms = als.refine(U, xi, Q0, sweeps)
    return Q, beta, norms, U, xi


@pytest.mark.parametrize("case", [
    dict(seed=91, N=20, b=5.0, n=48, R=20, R_l=8, n_s=9, ranks=[12, 14, 10], sweeps=1),
    dict(seed=92, N=35, b=6.0, n=64, R=24, R_l=10, n_s=11, ranks=[20, 18, 22], sweeps=2),
])
def test_als_matches_oracle(rsm, ctx, case):
    s = workloads.tiny_system(case["seed"], case["N"], case["b"], case["n"], case["R"],
                              case["R_l"], case["n_s"], min_sep=0.4)
    say(f"ALS {s.name} ranks {case['ranks']} sweeps {case['sweeps']}")
    Q, beta, norms, U, xi = oracle_refined(s, case["ranks"], case["sweeps"])
    ref = rs.assemble_system(s, fixed_ranks=case["ranks"])
    want = rhosvd.tucker_full(beta, Q) + ref.short_grid()
    f, T, g = run(rsm, ctx, s, case["ranks"], case["sweeps"])
    err = float(np.max(np.abs(g - want)) / np.max(np.abs(want)))
    # the Tucker error against the exact long-range canonical tensor
    A = rhosvd.canonical_full(U, xi)
    f0, T0, g0 = run(rsm, ctx, s, case["ranks"], 0)
    short = ref.short_grid()
    e_als = float(np.linalg.norm(g - short - A))
    e_rhosvd = float(np.linalg.norm(g0 - short - A))
    say(f"  rel-Linf vs oracle {err:.2e}; Tucker error {e_rhosvd:.3e} -> {e_als:.3e}; "
        f"oracle core norms {norms}")
    assert err <= 1e-6
    assert e_als <= e_rhosvd * (1 + 1e-9)
    # orthonormal refined bases
    V = [torch.empty(s.n * r, dtype=torch.float64, device="cuda") for r in case["ranks"]]
    rsm.tensor_export(T, V1=V[0], V2=V[1], V3=V[2])
    torch.cuda.synchronize()
    for l in range(3):
        Vl = V[l].cpu().numpy().reshape(s.n, -1)
        assert np.max(np.abs(Vl.T @ Vl - np.eye(Vl.shape[1]))) < 1e-12


def test_als_mixed_matches_fp64(rsm, ctx):
    s = workloads.tiny_system(93, 30, 6.0, 64, 24, 10, 9, min_sep=0.5)
    ranks = [22, 20, 24]
    _, _, g64 = run(rsm, ctx, s, ranks, 1)
    _, _, gmx = run(rsm, ctx, s, ranks, 1, prec="mixed_fp16")
    err = float(np.max(np.abs(gmx - g64)) / np.max(np.abs(g64)))
    say(f"ALS mixed vs FP64 {err:.2e}")
    assert err <= 1e-5
