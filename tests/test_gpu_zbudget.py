"""The context's admission budget (rs_ctx_set_hbm_budget): an assembly whose
footprint bound exceeds it is refused with RS_E_NOMEM before anything is
allocated, and the same context assembles once the budget covers the bound."""
import sys

import pytest

import workloads

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


def dev(a):
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def test_budget_refuses_then_admits(rsm):
    s = workloads.tiny_system(41, 37, 5.0, 72, 20, 8, 9, min_sep=0.4)
    say(f"hbm budget {s.name}")
    c = rsm.Context(0, hbm_budget=1)
    f = rsm.Factors(c, s.b, s.n, s.R, s.R_l, s.n_s)
    opts = rsm.make_aopts(s.eps_tucker, r_max=64)
    N = int(s.q.shape[0])
    with pytest.raises(rsm.RSError) as e:
        rsm.assemble(c, f, dev(s.pos), dev(s.q), None, opts)
    assert e.value.status == 2   # RS_E_NOMEM
    need = rsm.footprint_bytes(f, N, 64, "fp64", with_grid=False)
    assert need > 1
    c.set_hbm_budget(2 * need)
    T = rsm.assemble(c, f, dev(s.pos), dev(s.q), None, opts)
    torch.cuda.synchronize()
    assert all(r > 0 for r in T.info().ranks)
    T.free()
    c.set_hbm_budget(0)
    f.close()
    c.close()
