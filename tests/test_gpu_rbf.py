"""RBF matrix-vector product in RS form (section 4.1, case (A)) through the
C ABI against the oracle's matrix written out entry by entry: rel-Linf
<= 1e-12 of max |y| (the same FP64 sums in another order)."""
import sys

import numpy as np
import pytest

from oracle import quadrature, rbf

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


@pytest.mark.parametrize("case", [
    dict(b=3.0, n=8, R=16, R_l=6, n_s=3, kernel="newton", seed=1),
    dict(b=4.0, n=12, R=20, R_l=8, n_s=5, kernel="newton", seed=2),
    dict(b=2.5, n=10, R=24, R_l=10, n_s=7, kernel="newton+yukawa", seed=3),   # n not a multiple of 8
])
def test_rbf_matvec_matches_oracle(rsm, ctx, case):
    n = case["n"]
    f = rsm.Factors(ctx, case["b"], n, case["R"], case["R_l"], case["n_s"], kernel=case["kernel"], lam=0.5)
    t, a = quadrature.literal_table(case["kernel"], case["R"], 0.5)
    rng = np.random.default_rng(case["seed"])
    c = rng.normal(size=(n, n, n))
    want = rbf.rbf_matvec(case["b"], n, t, a, case["R_l"], case["n_s"], c)
    cd = torch.tensor(c.ravel(), dtype=torch.float64, device="cuda")
    y = torch.full_like(cd, float("nan"))
    rsm.rbf_matvec(ctx, f, cd, y)
    torch.cuda.synchronize()
    got = y.cpu().numpy().reshape(n, n, n)
    err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    say(f"rbf n={n} R={case['R']} R_l={case['R_l']} n_s={case['n_s']}: rel-Linf {err:.2e}")
    assert err <= 1e-12


def test_rbf_matvec_linear_and_symmetric(rsm, ctx):
    """At 64^3: <u, A v> = <A u, v> (A symmetric) and A (2u - v) = 2 A u - A v."""
    n = 64
    f = rsm.Factors(ctx, 10.0, n, 20, 8, 9)
    g = torch.Generator(device="cpu").manual_seed(5)
    u = torch.randn(n ** 3, dtype=torch.float64, generator=g).cuda()
    v = torch.randn(n ** 3, dtype=torch.float64, generator=g).cuda()
    Au, Av, Aw = (torch.empty_like(u) for _ in range(3))
    rsm.rbf_matvec(ctx, f, u, Au)
    rsm.rbf_matvec(ctx, f, v, Av)
    rsm.rbf_matvec(ctx, f, (2 * u - v).contiguous(), Aw)
    torch.cuda.synchronize()
    s1, s2 = float(torch.dot(u, Av)), float(torch.dot(Au, v))
    say(f"rbf 64^3: <u,Av> {s1:.12e} <Au,v> {s2:.12e}")
    assert abs(s1 - s2) <= 1e-11 * abs(s1)
    assert float((Aw - (2 * Au - Av)).abs().max()) <= 1e-11 * float(Aw.abs().max())
