"""The allocation-free energy and forces entry point, rs_energy_forces_noalloc,
against rs_energy_forces through the C ABI.  Both run the same kernels in the
same order, so the results must agree bitwise (stronger than the 1e-8
energy / 1e-6 force tolerance of the parity tests).  Two calls in a row, the
second with a smaller system (the static scratch array keeps the first
call's values); a system above the array's limit is rejected before anything
is enqueued."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def test_noalloc_energy_forces_matches_allocating_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1606_09218_amd as rsm
    ctx = rsm.Context(0)
    for seed, N, n in [(41, 60, 64), (42, 17, 48)]:
        s = workloads.tiny_system(seed, N, 5.0, n, 20, 8, 7, min_sep=0.5)
        print(f"noalloc: {s.name}", flush=True)
        f = rsm.Factors(ctx, s.b, s.n, s.R, s.R_l, s.n_s)
        T = rsm.assemble(ctx, f, dev(s.pos), dev(s.q), None, rsm.make_aopts(r_max=40))
        out = []
        for call in (rsm.energy_forces, rsm.energy_forces_noalloc):
            E = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
            F = torch.full((3 * N,), np.nan, dtype=torch.float64, device="cuda")
            dq = torch.full((N,), np.nan, dtype=torch.float64, device="cuda")
            call(T, E, F, 0.7, dq)
            out.append((E, F, dq))
        torch.cuda.synchronize()
        (E1, F1, q1), (E2, F2, q2) = out
        assert torch.isfinite(E1).all() and torch.isfinite(F1).all()
        assert torch.equal(E1, E2) and torch.equal(F1, F2) and torch.equal(q1, q2)
        T.free()
        f.close()
    # above the scratch array's 131072 particles: rejected, outputs untouched
    N = 131073
    s = workloads.tiny_system(43, N, 5.0, 16, 6, 1, 3)
    f = rsm.Factors(ctx, s.b, s.n, s.R, s.R_l, s.n_s)
    T = rsm.assemble(ctx, f, dev(s.pos), dev(s.q), None, rsm.make_aopts(r_max=8))
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    F = torch.zeros(3 * N, dtype=torch.float64, device="cuda")
    with pytest.raises(rsm.RSError) as e:
        rsm.energy_forces_noalloc(T, E, F)
    assert e.value.status == rsm.RS_E_INVALID
    torch.cuda.synchronize()
    assert float(E.abs().max()) == 0.0 and float(F.abs().max()) == 0.0
    T.free()
    f.close()
    ctx.close()
