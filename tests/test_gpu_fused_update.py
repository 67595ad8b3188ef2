"""The Arnoldi update fused with the next step's row transform (FP64 2-D grids whose
rows have 512, 1024 or 2048 points): solves reach the oracle's true residual, a batch
equals its right-hand sides solved one by one (bitwise), and two solver sessions of
one plan advanced in turns on one stream equal the same solves run alone (each step
finds its own row transform in the plan's workspace, or transforms again)."""
import time

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


def _thin(shape, seed, nrhs):
    """A 2-D grid of shape (n0, n1) with the benchmark's kind of medium."""
    n0, n1 = shape
    c = inputs.gaussian_random_field(shape, max(2.0, n0 / 4), seed, lo=0.8, hi=1.2)
    width = max(2, n0 // 8)
    c = inputs.blend_to_background(c, width, 1.0, taper=2)
    zeta = inputs.frame_layer(shape, width, 0.133)
    omega = 2 * np.pi * n0 / 8
    a = np.full(shape, 0.05 * omega)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((nrhs,) + shape) + 1j * rng.standard_normal((nrhs,) + shape)
    return c, a, zeta, omega, f


def _problem(name):
    if name == "thin_64x1024":
        shape = (64, 1024)
        c, a, zeta, omega, f = _thin(shape, 75, 2)
        kw = dict(m_real=6, m_layer=2, a_floor=0.05 * omega)
        return shape, omega, c, a, zeta, f, kw
    if name == "2d_512_grf":    # rows of 512 points
        w = inputs.workload("2d_1024_grf", n=512, nrhs=2, precision="fp64")
    else:                       # rows of 2048 points
        w = inputs.workload("2d_2048_grf", nrhs=2, precision="fp64")
    kw = dict(m_real=w.m_real, m_layer=w.m_layer, a_floor=w.a_floor)
    return w.shape, w.omega, w.c, w.a, w.zeta, w.f, kw


@pytest.mark.parametrize("name", ["thin_64x1024", "2d_512_grf", "2d_2048_grf"])
def test_fused_update_batch_and_oracle(orc, hp, dev, name):
    print(f"[case] fused update {name}", flush=True)
    shape, omega, c, a, zeta, f, kw = _problem(name)
    plan = hp.Plan(shape, omega, c, a, zeta, precision="fp64", max_nrhs=2, **kw)
    ft = torch.from_numpy(f).to(dev)
    x, info = plan.solve(ft, rtol=1e-8, restart=30)
    ref = orc.Problem(shape, omega, c, a, zeta, **kw)
    for r in range(2):
        res = rel(ref.matvec(x[r].cpu().numpy()), f[r])
        print(f"[fused {name}] rhs {r} iters {info[r].iters} cycles {info[r].cycles} oracle residual {res:.3e}",
              flush=True)
        assert info[r].status == 0 and res <= 1e-8 * 1.001
        assert abs(info[r].rel_true_residual - res) <= 1e-12
        x1, i1 = plan.solve(ft[r:r + 1].clone(), rtol=1e-8, restart=30)
        assert i1[0].iters == info[r].iters and torch.equal(x1[0], x[r])
    plan.close()


def test_fused_update_sessions_in_turns(hp, dev):
    """Two sessions of one plan on one stream, advanced a step at a time in turns: each
    step after the other session's must transform its own vector again."""
    shape = (64, 1024)
    print(f"[case] fused update, two sessions of one plan in turns {shape}", flush=True)
    c, a, zeta, omega, f = _thin(shape, 75, 2)
    kw = dict(m_real=6, m_layer=2, a_floor=0.05 * omega)
    plan = hp.Plan(shape, omega, c, a, zeta, precision="fp64", max_nrhs=1, **kw)
    fa = torch.from_numpy(f[:1]).to(dev)
    fb = torch.from_numpy(f[1:]).to(dev)
    xa0, ia0 = plan.solve(fa, rtol=1e-8, restart=30)
    xb0, ib0 = plan.solve(fb, rtol=1e-8, restart=30)
    stream = torch.cuda.Stream(device=dev)
    sa = hp.Solver(plan, 1, rtol=1e-8, restart=30)
    sb = hp.Solver(plan, 1, rtol=1e-8, restart=30)
    sa.start(fa, stream=stream)
    sb.start(fb, stream=stream)
    da = db = False
    t_end = time.monotonic() + 60.0
    while not (da and db):
        if not da:
            da = sa.advance(1)
        if not db:
            db = sb.advance(1)
        assert time.monotonic() < t_end
    xa, ia = sa.result()
    xb, ib = sb.result()
    print(f"[turns] iters {ia[0].iters}/{ia0[0].iters} and {ib[0].iters}/{ib0[0].iters}", flush=True)
    assert ia[0].status == 0 and ib[0].status == 0
    assert ia[0].iters == ia0[0].iters and ib[0].iters == ib0[0].iters
    assert torch.equal(xa, xa0) and torch.equal(xb, xb0)
    sa.close()
    sb.close()
    plan.close()
