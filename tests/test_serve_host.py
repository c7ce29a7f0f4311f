"""Host logic of the serving loop (no GPU): a request that cannot fit even an empty arena
is rejected instead of being retried forever, and the requests behind it still run."""
from types import SimpleNamespace

import pytest

import workloads
from paper_2306_11544_amd import binding as B
from paper_2306_11544_amd.serve import Server


class StubBatch:
    """Stands in for the device batch: admits requests of at most `fit` cells, finishes
    each admitted one at the next poll after a step, and records what it was asked."""

    def __init__(self, fit):
        self.fit, self.slots, self.finished, self.steps = fit, {}, [], 0

    def capacity(self):
        return dict(max_cells=self.fit, max_voxels=self.fit, max_slots=8, arena_bytes=1)

    def mark_clock(self):
        pass

    def step(self, n):
        self.steps += n
        self.finished = list(self.slots)

    def admit_pop(self, pop, n_steps):
        if pop.n > self.fit:
            raise B.MechError(B.MECH_E_BUDGET, f"{pop.n} cells do not fit {self.fit}")
        slot = len(self.slots) + len(self.finished) + 100
        self.slots[slot] = pop.n
        return slot

    def sync(self):
        pass

    def poll(self):
        out, self.finished = self.finished, []
        for s in out:
            self.slots.pop(s)
        return out

    def done_ms(self, slot):
        return 1.0

    def retire(self, slot):
        pass

    def close(self):
        pass


class StubServer(Server):
    def make_batch(self):
        return StubBatch(fit=1000)


@pytest.mark.timeout(60)
def test_request_larger_than_the_arena_is_rejected():
    p = B.make_params((0, 0, 0), (1, 1, 1), c_adh=workloads.C_ADH_2, precision=B.MECH_FP32)
    srv = StubServer(p, 1 << 20, steps_per_chunk=5)
    reqs = [SimpleNamespace(rid=0, arrival_s=0.0, n=5000, steps=10),
            SimpleNamespace(rid=1, arrival_s=0.0, n=800, steps=10),
            SimpleNamespace(rid=2, arrival_s=0.01, n=9000, steps=10),
            SimpleNamespace(rid=3, arrival_s=0.02, n=300, steps=10)]
    done = srv.run(reqs, lambda r: SimpleNamespace(n=r.n))
    assert sorted(d.rid for d in done) == [1, 3]
    assert [x[0] for x in srv.rejected] == [0, 2]
    assert srv.stats["rejected"] == 2 and srv.stats["requests"] == 2
