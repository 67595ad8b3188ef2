"""CPU test of the serving scheduler (admission by footprint, first come first
served, retirement frees memory) with a fake executor that simulates the number
of steps each solve takes (no GPU)."""
from paper_2409_16172_amd import serve


class FakeServer(serve.Server):
    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.order = []
        self.left = {}

    def _admit(self, r, now, dev, torch):
        self.order.append(r.rid)
        r.admitted = now
        self.in_use += r.footprint
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        self.left[r.rid] = 3 + r.rid % 4
        self.active.append((r, None, None, None, None, None))

    def _progress(self, item, t0):
        r = item[0]
        self.left[r.rid] -= self.steps
        if self.left[r.rid] <= 0:
            r.finished = r.admitted + 1.0
            return True
        return False


def _reqs(n, gib):
    out = []
    for i in range(n):
        r = serve.Request(i, 0.0005 * i, workload=None)
        r.footprint = gib << 30
        out.append(r)
    return out


def test_admission_respects_budget_and_fifo():
    srv = FakeServer(hbm_budget_bytes=7 << 30, max_active=4, steps_per_turn=1)
    done = srv.run(_reqs(10, 3), dev=False)
    assert len(done) == 10
    assert srv.order == list(range(10))          # first come, first served
    assert srv.peak_in_use <= 7 << 30            # two 3 GiB requests at a time at most
    assert srv.in_use == 0 and not srv.active


def test_slot_limit_and_oversized_request_runs_alone():
    srv = FakeServer(hbm_budget_bytes=1 << 30, max_active=2, steps_per_turn=2)
    reqs = _reqs(3, 4)                           # each larger than the budget
    done = srv.run(reqs, dev=False)
    assert len(done) == 3 and srv.peak_in_use == 4 << 30
    srv2 = FakeServer(hbm_budget_bytes=64 << 30, max_active=2, steps_per_turn=1)
    srv2.run(_reqs(6, 1), dev=False)
    assert srv2.peak_in_use <= 2 << 30           # at most max_active at once
