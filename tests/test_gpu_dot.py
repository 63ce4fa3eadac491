"""Scalar products of RS tensors (section 3.4, item (d)) through the C ABI
against the oracle's product of the full grids: relative error <= 1e-10 for
FP64 tensors at the oracle's ranks (the same arithmetic summed in another
order), 1e-6 for split-precision tensors (whose cores carry the split
error), and against the product of the GPU's own materialised grids."""
import sys

import numpy as np
import pytest

import workloads
from oracle import dot as odot, rs

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


def build(rsm, ctx, s, ranks, prec="fp64", with_grid=False):
    f = rsm.Factors(ctx, s.b, s.n, s.R, s.R_l, s.n_s, kernel=s.kernel, lam=s.lam)
    g = None
    if with_grid:
        g = torch.empty(s.n ** 3, dtype=torch.float64 if prec == "fp64" else torch.float32, device="cuda")
    T = rsm.assemble(ctx, f, dev(s.pos), dev(s.q), g, rsm.make_aopts(s.eps_tucker, fixed_ranks=ranks, prec=prec))
    return f, T, g


def gpu_dot(rsm, A, B):
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    rsm.dot(A, B, out)
    torch.cuda.synchronize()
    return out.item()


PAIRS = [
    # different particles, charges, split and window
    (dict(seed=71, N=14, b=5.0, n=40, R=20, R_l=8, n_s=7), dict(seed=72, N=9, b=5.0, n=40, R=24, R_l=10, n_s=9)),
    # the same particles (the paper's setting), another kernel for B
    (dict(seed=73, N=20, b=6.0, n=48, R=20, R_l=8, n_s=9), dict(seed=73, N=20, b=6.0, n=48, R=28, R_l=11, n_s=9, kernel="newton+yukawa")),
    # windows cut by the grid's faces, one particle against many
    (dict(seed=74, N=1, b=4.0, n=32, R=16, R_l=6, n_s=5, box=0.99), dict(seed=75, N=25, b=4.0, n=32, R=20, R_l=8, n_s=11, box=0.99)),
]


def system(c):
    return workloads.tiny_system(c["seed"], c["N"], c["b"], c["n"], c["R"], c["R_l"], c["n_s"],
                                 min_sep=0.3, box_frac=c.get("box", 0.6),
                                 kernel=c.get("kernel", "newton"))


@pytest.mark.parametrize("pair", PAIRS)
def test_dot_matches_oracle_fp64(rsm, ctx, pair):
    sa, sb = system(pair[0]), system(pair[1])
    say(f"dot {sa.name} . {sb.name}")
    ra, rb = rs.assemble_system(sa), rs.assemble_system(sb)
    fa, A, _ = build(rsm, ctx, sa, ra.ranks)
    fb, B, _ = build(rsm, ctx, sb, rb.ranks)
    want = odot.scalar_product(ra, rb)
    got = gpu_dot(rsm, A, B)
    got_t = gpu_dot(rsm, B, A)
    aa = gpu_dot(rsm, A, A)
    want_aa = odot.scalar_product(ra, ra)
    say(f"  <A,B> {got:.15e} oracle {want:.15e} rel {abs(got - want) / abs(want):.2e}; "
        f"<A,A> rel {abs(aa - want_aa) / want_aa:.2e}")
    assert abs(got - want) <= 1e-10 * abs(want)
    assert abs(got_t - got) <= 1e-12 * abs(got)
    assert abs(aa - want_aa) <= 1e-10 * want_aa


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp16"])
def test_dot_matches_own_grids(rsm, ctx, prec):
    """Against the product of the grids the GPU itself materialises (cfg1
    size, 128^3 cells), in the tensors' own precision."""
    s1 = workloads.cfg1_plain_small()
    s2 = workloads.tiny_system(76, 40, s1.b, s1.n, 20, 8, 9, min_sep=0.5)
    r1, r2 = rs.assemble_system(s1), rs.assemble_system(s2)
    f1, A, ga = build(rsm, ctx, s1, r1.ranks, prec, with_grid=True)
    f2, B, gb = build(rsm, ctx, s2, r2.ranks, prec, with_grid=True)
    got = gpu_dot(rsm, A, B)
    ref = float(torch.dot(ga.double(), gb.double()).item())
    want = odot.scalar_product(r1, r2)
    say(f"dot {prec}: {got:.12e} own grids {ref:.12e} oracle {want:.12e}")
    tol = 1e-10 if prec == "fp64" else 1e-6
    assert abs(got - want) <= tol * abs(want)
    # the FP32 grids round each value: their product agrees to ~1e-6
    assert abs(got - ref) <= (1e-10 if prec == "fp64" else 1e-5) * abs(ref)


def test_dot_rejects_other_grids(rsm, ctx):
    sa = system(PAIRS[0][0])
    sb = workloads.tiny_system(77, 5, 5.0, 48, 16, 6, 5, min_sep=0.3)
    fa, A, _ = build(rsm, ctx, sa, rs.assemble_system(sa).ranks)
    fb, B, _ = build(rsm, ctx, sb, rs.assemble_system(sb).ranks)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(rsm.RSError):
        rsm.dot(A, B, out)


def test_dot_dense_columns_against_own_grids(rsm, ctx):
    """Dense windows on a 192^3 grid (1500 and 900 particles in [-6, 6]^3):
    brick columns with many touched bricks (several groups of four per
    column) and bricks listed by several particles, A and B with different
    windows and quadratures; FP64 tensors at the rank rule's ranks against
    the product of their own FP64 grids at 1e-10."""
    sa = workloads.tiny_system(81, 1500, 6.0, 192, 24, 10, 13, min_sep=0.35)
    sb = workloads.tiny_system(82, 900, 6.0, 192, 20, 8, 9, min_sep=0.35)
    out = []
    for s in (sa, sb):
        f = rsm.Factors(ctx, s.b, s.n, s.R, s.R_l, s.n_s, kernel=s.kernel, lam=s.lam)
        g = torch.empty(s.n ** 3, dtype=torch.float64, device="cuda")
        T = rsm.assemble(ctx, f, dev(s.pos), dev(s.q), g, rsm.make_aopts(s.eps_tucker, r_max=192))
        out.append((f, T, g))
    (fa, A, ga), (fb, B, gb) = out
    got = gpu_dot(rsm, A, B)
    ref = float(torch.dot(ga, gb).item())
    aa = gpu_dot(rsm, A, A)
    ref_aa = float(torch.dot(ga, ga).item())
    say(f"dense dot: ranks {list(A.info().ranks)} {list(B.info().ranks)}: <A,B> {got:.15e} "
        f"grids {ref:.15e} rel {abs(got - ref) / abs(ref):.2e}; <A,A> rel {abs(aa - ref_aa) / ref_aa:.2e}")
    assert abs(got - ref) <= 1e-10 * abs(ref)
    assert abs(aa - ref_aa) <= 1e-10 * ref_aa
    for f, T, _ in out:
        T.free()
        f.close()
