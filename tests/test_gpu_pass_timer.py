"""The pass timer (hp_plan_time_pass / hp_plan_pass_times): one event-timed record per
launch of the chosen pass, in applies and solves, none while it is off or for launches
captured into a step graph; timing changes no result."""
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


def test_timer_counts_launches(hp, dev, monkeypatch):
    print("[case] pass timer 128^2", flush=True)
    monkeypatch.setenv("HP_STEP_GRAPHS", "0")
    w = inputs.workload("2d_1024_grf", n=128, n_lambda=12.0, width=8, seed=3, nrhs=2)
    plan = hp.plan_from_workload(w, max_nrhs=2)
    f = torch.from_numpy(w.f).to(dev)
    u0 = plan.apply(f).clone()
    x0, i0 = plan.solve(f, rtol=1e-9)
    torch.cuda.synchronize()
    assert plan.pass_times() == []                     # off by default
    plan.time_pass(2)
    for _ in range(3):
        u = plan.apply(f)                              # one launch of pass B per apply (both RHS)
    t = plan.pass_times()
    assert len(t) == 3 and all(0.0 < x < 1000.0 for x in t)
    assert torch.equal(u, u0)
    x, info = plan.solve(f, rtol=1e-9)
    t = plan.pass_times()
    # every Arnoldi step applies Q once, each cycle adds one more apply; launches
    # enqueued after a cycle's end are recorded too
    steps = max(i.iters for i in info)
    assert len(t) >= steps and all(x > 0.0 for x in t)
    assert [(i.iters, i.cycles) for i in info] == [(i.iters, i.cycles) for i in i0] and torch.equal(x, x0)
    assert plan.pass_times() == []                     # a read clears the record
    plan.time_pass(4)
    plan.apply(f)
    assert len(plan.pass_times()) == 1
    plan.time_pass(None)
    plan.apply(f)
    assert plan.pass_times() == []
    with pytest.raises(hp.HelmpreError):
        plan.time_pass(5)


def test_timer_skips_captured_launches(hp, dev, monkeypatch):
    print("[case] pass timer with step graphs", flush=True)
    w = inputs.workload("2d_1024_grf", n=128, n_lambda=12.0, width=8, seed=4)
    plan = hp.plan_from_workload(w)
    f = torch.from_numpy(w.f).to(dev)
    monkeypatch.setenv("HP_STEP_GRAPHS", "0")
    x0, i0 = plan.solve(f, rtol=1e-9)
    plan.time_pass(2)
    plan.solve(f, rtol=1e-9)
    eager = len(plan.pass_times())
    monkeypatch.setenv("HP_STEP_GRAPHS", "1")
    x1, i1 = plan.solve(f, rtol=1e-9)
    captured = len(plan.pass_times())
    plan.time_pass(None)
    torch.cuda.synchronize()
    assert torch.equal(x1, x0) and i1[0].iters == i0[0].iters
    # the Arnoldi steps' applies run inside graphs: only the applies outside them remain
    assert eager >= i0[0].iters and captured < eager
