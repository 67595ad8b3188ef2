"""GPU tests of resumable solves and of the continuous-batching server: a solve
driven step by step equals the blocking solve, and every request served in a
mix of concurrent requests gives the same result (bit for bit, since every
reduction has a fixed order and each request owns its plan) as when solved
alone; all reach the FP64 true residual rtol checked by the oracle."""
import numpy as np
import pytest

from paper_2409_16172_amd import inputs
from tests.util import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_solver_session_equals_blocking_solve(dev):
    from paper_2409_16172_amd import binding
    w = inputs.workload("2d_1024_grf", n=256)
    plan = binding.plan_from_workload(w)
    f = torch.from_numpy(w.f).to(dev)
    xb, ib = plan.solve(f, rtol=1e-8)
    s = binding.Solver(plan, 1, rtol=1e-8)
    stream = torch.cuda.Stream(device=dev)
    x = s.start(f, stream=stream)
    turns = 0
    while not s.advance(2):
        turns += 1
        assert turns < 100000
    x, info = s.result()
    s.close()
    assert info[0].status == 0 and info[0].iters == ib[0].iters
    assert torch.equal(x, xb)


def test_served_mix_equals_alone(orc, dev):
    from paper_2409_16172_amd import binding, serve
    reqs = serve.stream_requests(6, rate_per_s=400.0, grids=((64, 64), (128, 128), (256, 256)), precision="fp64",
                                 n_lambda=(8.0, 40.0))
    srv = serve.Server(hbm_budget_bytes=64 << 30, max_active=4, steps_per_turn=2)
    done = srv.run(reqs, dev=dev)
    assert len(done) == 6
    overlapped = sum(1 for a in done for b in done if a.rid < b.rid and a.admitted < b.finished and b.admitted < a.finished)
    print(f"[serve] pairs overlapping in time: {overlapped}", flush=True)
    assert overlapped >= 1
    for r in done:
        w = r.workload
        assert r.info[0].status == 0
        plan = binding.plan_from_workload(w, max_nrhs=1)
        x1, i1 = plan.solve(torch.from_numpy(w.f[:1]).to(dev), rtol=1e-8)
        assert torch.equal(x1, r.x), r.rid
        res = rel(orc.from_workload(w).matvec(r.x.cpu().numpy()[0]), w.f[0])
        assert res <= 1e-8 * 1.001, (r.rid, res)
        plan.close()
    st = serve.latency_stats(done)
    assert st["latency_ms_p99"] >= st["latency_ms_p50"] > 0
