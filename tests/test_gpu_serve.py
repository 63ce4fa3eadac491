"""Serving on the GPU: requests overlap on the device through per-slot
streams, and every result is the same alone and in the mix."""
import dataclasses

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ex():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1606_09218_amd.serve import GpuExecutor
    return GpuExecutor(0, prec="mixed_fp16", r_max=128)


def small_trace():
    tr = workloads.cfg5_trace(seed=55, n_requests=12, rate_hz=400.0, n_choices=(64, 128), N_lo=16,
                              N_hi=600)
    for r in tr:
        r.b = 25.0
    return tr


def test_mix_equals_alone(ex):
    from paper_1606_09218_amd.serve import Server, summarize
    tr = small_trace()
    mix = Server(ex, n_slots=4, hbm_budget=64 << 30).run_trace(tr)
    alone = Server(ex, n_slots=1, hbm_budget=64 << 30).run_trace(tr, time_scale=0.0)
    s = summarize(mix)
    print(f"mix: {s}", flush=True)
    assert s["completed"] == len(tr)
    for a, b in zip(mix, alone):
        assert a.error is None and b.error is None, (a.error, b.error)
        assert a.result["energy"] == b.result["energy"]      # bitwise
        assert a.result["ranks"] == b.result["ranks"]
