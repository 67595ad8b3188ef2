"""Arnoldi steps captured as HIP graphs (small grids): every replay gives what the eager
launches give, bitwise — across solves, sides, right-hand-side counts, sessions and a
re-tuned plan, with other eager work and synchronisations between the replays."""
import numpy as np
import pytest
import torch

from paper_2409_16172_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def hp():
    from paper_2409_16172_amd import binding
    binding.load_library()
    return binding


def _problem(n, seed, nrhs=1):
    w = inputs.workload("2d_1024_grf", n=n, n_lambda=12.0 * n / 128, width=8, seed=seed, nrhs=nrhs)
    return w


def _solve(hp, plan, f, graphs, monkeypatch, **kw):
    monkeypatch.setenv("HP_STEP_GRAPHS", "1" if graphs else "0")
    x, info = plan.solve(f, **kw)
    torch.cuda.synchronize()
    return x.clone(), [(i.iters, i.cycles, i.rel_true_residual) for i in info]


@pytest.mark.parametrize("side", ["right", "left", "none"])
def test_graph_replays_match_eager(hp, dev, side, monkeypatch):
    print(f"[case] step graphs 128^2 side={side}", flush=True)
    w = _problem(128, 11)
    plan = hp.plan_from_workload(w)
    f = torch.from_numpy(w.f).to(dev)
    kw = dict(rtol=1e-9, restart=20, side=side, max_cycles=5 if side == "none" else 200)
    x0, i0 = _solve(hp, plan, f, False, monkeypatch, **kw)
    other = _problem(128, 12)
    pother = hp.plan_from_workload(other)
    fo = torch.from_numpy(other.f).to(dev)
    for rep in range(3):
        x1, i1 = _solve(hp, plan, f, True, monkeypatch, **kw)
        assert i1 == i0 and torch.equal(x1, x0), rep
        _solve(hp, pother, fo, False, monkeypatch, rtol=1e-8)   # eager work between the replays
        pother.apply(fo)
        torch.cuda.synchronize()


def test_graphs_batched_and_restart_change(hp, dev, monkeypatch):
    print("[case] step graphs batch of 3, two restart lengths", flush=True)
    w = _problem(128, 13, nrhs=3)
    plan = hp.plan_from_workload(w, max_nrhs=3)
    f = torch.from_numpy(w.f).to(dev)
    for restart in (30, 12, 30):
        x0, i0 = _solve(hp, plan, f, False, monkeypatch, rtol=1e-9, restart=restart)
        x1, i1 = _solve(hp, plan, f, True, monkeypatch, rtol=1e-9, restart=restart)
        assert i1 == i0 and torch.equal(x1, x0)
    # one right-hand side on the same plan and workspace
    x0, i0 = _solve(hp, plan, f[:1].contiguous(), False, monkeypatch, rtol=1e-9)
    x1, i1 = _solve(hp, plan, f[:1].contiguous(), True, monkeypatch, rtol=1e-9)
    assert i1 == i0 and torch.equal(x1, x0)


def test_graphs_in_sessions_and_after_autotune(hp, dev, monkeypatch, tmp_path):
    print("[case] step graphs in sessions, re-tuned plan", flush=True)
    monkeypatch.setenv("HP_TUNE_CACHE", str(tmp_path / "tune.txt"))
    w = _problem(128, 14)
    plan = hp.plan_from_workload(w)
    f = torch.from_numpy(w.f).to(dev)
    res = {}
    for graphs in (False, True, True):
        monkeypatch.setenv("HP_STEP_GRAPHS", "1" if graphs else "0")
        s = hp.Solver(plan, rtol=1e-9)
        s.start(f)
        while not s.advance(3):
            pass
        x, info = s.result()
        torch.cuda.synchronize()
        res.setdefault(graphs, []).append((x.clone(), info[0].iters))
        s.close()
    (xe, ie), = res[False]
    for x, it in res[True]:
        assert it == ie and torch.equal(x, xe)
    _solve(hp, plan, f, True, monkeypatch, rtol=1e-9)   # graphs of the untuned plan
    plan.autotune()
    x0, i0 = _solve(hp, plan, f, False, monkeypatch, rtol=1e-9)
    x1, i1 = _solve(hp, plan, f, True, monkeypatch, rtol=1e-9)
    assert i1 == i0 and torch.equal(x1, x0)
