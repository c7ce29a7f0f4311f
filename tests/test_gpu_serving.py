"""Continuous batching: requests admitted while others run give the same result as alone,
also when a small HBM budget makes them queue."""
import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu, run_gpu, say
from paper_2306_11544_amd import binding as B
from paper_2306_11544_amd.serve import Server

pytestmark = pytest.mark.gpu


def _requests(k=10, rate=400.0):
    return workloads.request_stream(k, rate_per_s=rate, seed=77, size_lo=1000, size_hi=12000,
                                    steps_lo=5, steps_hi=60)


@pytest.mark.parametrize("budget_mb,live", [(2048, None), (4, None), (2048, 20000)])
def test_serving_results_equal_solo(budget_mb, live):
    require_gpu()
    reqs = _requests()
    pops = {r.rid: workloads.request_population(r) for r in reqs}
    params = B.make_params((0, 0, 0), (1, 1, 1), c_adh=workloads.C_ADH_2, precision=B.MECH_FP32)
    say("serving", budget_mb, [r.n for r in reqs])
    srv = Server(params, budget_mb << 20, max_slots=64, steps_per_chunk=7, max_live_cells=live)
    try:
        done = srv.run(reqs, lambda r: pops[r.rid], keep_results=True)
        stats = srv.stats
    finally:
        srv.close()
    assert sorted(d.rid for d in done) == [r.rid for r in reqs]
    if budget_mb == 4 or live is not None:
        assert stats["max_queue"] >= 1  # the budget or the live-cell limit made requests wait
    if budget_mb > 4:
        assert stats["max_live_slots"] >= 2  # requests overlapped on the device
    for d in done:
        assert d.done_s >= d.admit_s >= d.arrival_s - 1e-6
        solo = run_gpu(pops[d.rid], d.steps, precision=B.MECH_FP32)
        assert np.array_equal(d.pos, solo["pos"]) and np.array_equal(d.vel, solo["vel"])
