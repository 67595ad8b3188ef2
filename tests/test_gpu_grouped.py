"""Grouped Arnoldi steps (hp_solver_advance_group): several solves of different grids,
media and frequencies advanced together, the steps of the mixed-precision ones running
as one launch per pass over all of them.  Every result must equal, bit for bit, the same
request solved alone, and reach rtol in the oracle's FP64 residual."""
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


@pytest.fixture(scope="module")
def hp():
    from paper_2409_16172_amd import binding
    binding.load_library()
    return binding


def _workloads():
    """Uneven grids and options: 2-D 256^2 to 1024^2 and 3-D 128^3 (mixed precision, the
    grouped kernels' domain), a cubic-Lagrange plan, a bivariate (c, a) plan, and two that
    step on their own (an FP64 plan and a 512 x 256 grid whose lines the grouped passes
    cover, but in FP64)."""
    ws = []
    for n, nl, seed in ((256, 24.0, 1), (512, 40.0, 2), (1024, 60.0, 3), (256, 50.0, 4)):
        ws.append((inputs.workload("2d_1024_grf", n=n, n_lambda=nl, width=max(8, n // 32), seed=seed,
                                   precision="mixed"), {}))
    w3 = inputs.workload("3d_256_grf", n=128, n_lambda=16.0, nrhs=1, seed=5)
    w3.precision = "mixed"
    ws.append((w3, {}))
    ws.append((inputs.workload("2d_1024_grf", n=256, n_lambda=30.0, width=8, seed=6, precision="mixed"),
               {"interp_order": 3}))
    wb = inputs.workload("2d_1024_grf", n=512, n_lambda=30.0, width=16, seed=7, precision="mixed")
    ws.append((wb, {"bivariate": True}))
    ws.append((inputs.workload("2d_1024_grf", n=256, n_lambda=20.0, width=8, seed=8, precision="fp64"), {}))
    return ws


def _plan(hp, w, opts):
    if opts.get("bivariate"):
        n = w.shape[0]
        a = inputs.gaussian_random_field(w.shape, 12.0, 99, lo=0.03 * w.omega, hi=0.3 * w.omega)
        return hp.Plan(w.shape, w.omega, w.c, a, None, m_real=8, m_damp=3, precision=w.precision, max_nrhs=1,
                       a_floor=0.05 * w.omega), a
    kw = {k: v for k, v in opts.items() if k != "bivariate"}
    return hp.plan_from_workload(w, max_nrhs=1, **kw), None


def _alone(hp, w, opts, dev):
    p, a = _plan(hp, w, opts)
    s = hp.Solver(p, 1, rtol=1e-8)
    s.start(torch.from_numpy(w.f[:1]).to(dev))
    x, info = s.result()
    s.close()
    p.close()
    return x, info[0]


def test_grouped_steps_equal_solves_alone(orc, hp, dev):
    ws = _workloads()
    print("[case] grouped advance over " + ", ".join(f"{w.shape}/{w.precision}" for w, _ in ws), flush=True)
    stream = torch.cuda.Stream(device=dev)
    plans, solvers, xs = [], [], []
    for w, opts in ws:
        p, _ = _plan(hp, w, opts)
        s = hp.Solver(p, 1, rtol=1e-8)
        with torch.cuda.stream(stream):
            f = torch.from_numpy(w.f[:1]).to(dev)
        stream.synchronize()
        xs.append(s.start(f, stream=stream))
        plans.append(p)
        solvers.append(s)
    done = [False] * len(solvers)
    turns = 0
    while not all(done):
        done = hp.advance_group(solvers, 3)
        turns += 1
        assert turns < 200000
    for k, ((w, opts), s) in enumerate(zip(ws, solvers)):
        x, info = s.result()
        xa, ia = _alone(hp, w, opts, dev)
        print(f"[grouped] {k} {w.shape} {w.precision} {opts} iters {info[0].iters} alone {ia.iters}", flush=True)
        assert info[0].status == 0 and ia.status == 0
        assert info[0].iters == ia.iters and torch.equal(x, xa), k
        if not opts.get("bivariate"):
            res = rel(orc.from_workload(w, **{k2: v for k2, v in opts.items()}).matvec(x.cpu().numpy()[0]), w.f[0])
            assert res <= 1e-8 * 1.001, (k, res)
        s.close()
    for p in plans:
        p.close()


def test_grouped_more_members_than_one_launch(hp, dev):
    """Ten 256^2 requests: two launches per pass per round (at most eight members each)."""
    print("[case] grouped advance of 10 requests", flush=True)
    stream = torch.cuda.Stream(device=dev)
    ws = [inputs.workload("2d_1024_grf", n=256, n_lambda=20.0 + 2 * k, width=8, seed=40 + k, precision="mixed")
          for k in range(10)]
    plans = [hp.plan_from_workload(w, max_nrhs=1) for w in ws]
    solvers = [hp.Solver(p, 1, rtol=1e-8) for p in plans]
    for w, s in zip(ws, solvers):
        with torch.cuda.stream(stream):
            f = torch.from_numpy(w.f[:1]).to(dev)
        stream.synchronize()
        s.start(f, stream=stream)
    done = [False] * 10
    while not all(done):
        done = hp.advance_group(solvers, 4)
    for w, s, p in zip(ws, solvers, plans):
        x, info = s.result()
        xa, ia = _alone(hp, w, {}, dev)
        assert info[0].status == 0 and torch.equal(x, xa)
        s.close()
        p.close()


def test_grouped_advance_errors(hp, dev):
    print("[case] grouped advance error paths", flush=True)
    w = inputs.workload("2d_1024_grf", n=256, n_lambda=20.0, width=8, seed=3, precision="mixed")
    p, p2 = hp.plan_from_workload(w, max_nrhs=1), hp.plan_from_workload(w, max_nrhs=1)
    s1, s2 = hp.Solver(p, 1), hp.Solver(p2, 1)
    f = torch.from_numpy(w.f[:1]).to(dev)
    with pytest.raises(hp.HelmpreError):          # not started
        hp.advance_group([s1], 1)
    st1, st2 = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    s1.start(f, stream=st1)
    with pytest.raises(hp.HelmpreError):          # listed twice
        hp.advance_group([s1, s1], 1)
    s2.start(f.clone(), stream=st2)
    hp.advance_group([s1, s2], 1)                 # two streams: two groups of one
    s1.result()
    s2.result()
    s1.close()
    s2.close()
    p.close()
    p2.close()


def test_grouped_server_equals_alone(orc, dev):
    """The serving loop with grouped steps: uneven grids admitted over time share the
    launches; each result equals the request solved alone."""
    from paper_2409_16172_amd import binding, serve
    reqs = serve.stream_requests(6, rate_per_s=300.0, seed=20240930,
                                 grids=((256, 256), (512, 512), (128, 128, 128)), precision="mixed",
                                 n_lambda=(10.0, 40.0))
    print("[case] grouped server " + ", ".join(str(r.workload.shape) for r in reqs), flush=True)
    srv = serve.Server(hbm_budget_bytes=64 << 30, max_active=4, steps_per_turn=2, grouped=True)
    done = srv.run(reqs, dev=dev)
    assert len(done) == 6
    for r in done:
        w = r.workload
        assert r.info[0].status == 0
        x1, _ = _alone(binding, w, {}, dev)
        assert torch.equal(x1, r.x), r.rid
        res = rel(orc.from_workload(w).matvec(r.x.cpu().numpy()[0]), w.f[0])
        assert res <= 1e-8 * 1.001, (r.rid, res)
