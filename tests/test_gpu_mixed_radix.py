"""GPU parity on grids whose lengths are not powers of two (N = 2^a 3^b 5^c, the
grids of Example 1, Section 5.1): mixed-radix lines held in LDS, compared with the
CPU oracle through the C ABI."""
import numpy as np
import pytest
import torch

from paper_2409_16172_amd import inputs
from tests.util import rel

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


def _case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _media(shape, seed, layer=True):
    n = min(shape)
    c = inputs.gaussian_random_field(shape, max(2.0, n / 10), seed)
    if not layer:
        return c, None
    width = max(2, n // 8)
    c = inputs.blend_to_background(c, width, 1.0, taper=max(2, min(8, n // 8)))
    return c, inputs.frame_layer(shape, width, 0.133)


def _rand(shape, seed, nrhs=1):
    rng = np.random.default_rng(seed)
    sh = (nrhs,) + tuple(shape)
    return rng.standard_normal(sh) + 1j * rng.standard_normal(sh)


CASES = [((12, 20), True), ((48, 60), True), ((90, 72), True), ((180, 180), False), ((24, 256), True),
         ((256, 24), True), ((4800, 8), False), ((8, 2400), False), ((12, 20, 18), True), ((24, 16, 30), False)]


@pytest.mark.parametrize("shape,layer", CASES)
def test_apply_fp64_mixed_radix(orc, hp, dev, shape, layer):
    _case("mixed_radix_apply_fp64", shape=shape, layer=layer)
    c, zeta = _media(shape, sum(shape), layer)
    omega = 2 * np.pi * min(shape) / 10
    a = np.full(shape, 0.05 * omega)
    kw = dict(m_real=6, m_layer=3, a_floor=0.05 * omega)
    plan = hp.Plan(shape, omega, c, a, zeta, max_nrhs=2, **kw)
    ref = orc.Problem(shape, omega, c, a, zeta, **kw)
    v = _rand(shape, 3, nrhs=2)
    u = plan.apply(torch.from_numpy(v).to(dev)).cpu().numpy()
    ue = ref.apply(v)
    for r in range(2):
        assert rel(u[r], ue[r]) < 1e-12, (r, rel(u[r], ue[r]))


@pytest.mark.parametrize("shape", [(60, 90), (12, 20, 18), (360, 40)])
def test_apply_mixed_precision_mixed_radix(orc, hp, dev, shape):
    _case("mixed_radix_apply_mixed", shape=shape)
    c, zeta = _media(shape, 5 + sum(shape))
    omega = 2 * np.pi * min(shape) / 10
    a = np.full(shape, 0.05 * omega)
    kw = dict(m_real=8, m_layer=3, a_floor=0.05 * omega)
    plan = hp.Plan(shape, omega, c, a, zeta, precision="mixed", **kw)
    ref = orc.Problem(shape, omega, c, a, zeta, **kw)
    v = _rand(shape, 9)
    u = plan.apply(torch.from_numpy(v).to(dev).to(torch.complex64)).cpu().numpy()
    assert rel(u, ref.apply(v.astype(np.complex64).astype(np.complex128))) < 1e-5


def test_inclusion_apply_full_row_180(orc, hp, dev):
    """Example 1's medium at N = 180 (the first grid of Table 1), M = 2, 4, 8."""
    w = inputs.workload("2d_inclusion", n=180, delta=4.0)
    v = _rand(w.shape, 21)
    for m in (2, 4, 8):
        _case("inclusion_apply", n=180, M=m)
        plan = hp.plan_from_workload(w, m_real=m)
        u = plan.apply(torch.from_numpy(v).to(dev)).cpu().numpy()
        assert rel(u, orc.from_workload(w, m_real=m).apply(v)) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_inclusion_solve_mixed_radix(orc, hp, dev, prec):
    """Right-preconditioned GMRES(10) on Example 1's problem at N = 120 reaches rtol 1e-8 in
    the oracle's FP64 true residual."""
    _case("inclusion_solve", n=120, prec=prec)
    w = inputs.workload("2d_inclusion", n=120, precision=prec)
    plan = hp.plan_from_workload(w)
    x, info = plan.solve(torch.from_numpy(w.f).to(dev), rtol=1e-8, restart=10)
    assert info[0].status == 0
    ref = orc.from_workload(w)
    assert rel(ref.matvec(x.cpu().numpy()[0]), w.f[0]) <= 1e-8 * 1.001


@pytest.mark.parametrize("shape", [(12, 20), (90, 72), (12, 20, 18)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("mixed", 1e-6)])
def test_matvec_mixed_radix(orc, hp, dev, shape, prec, tol):
    """The periodic stencil wraps correctly on lengths that are not powers of two."""
    _case("mixed_radix_matvec", shape=shape, prec=prec)
    c, zeta = _media(shape, 2 + sum(shape))
    omega = 2 * np.pi * min(shape) / 10
    a = np.full(shape, 0.05 * omega)
    plan = hp.Plan(shape, omega, c, a, zeta, m_real=4, m_layer=3, a_floor=0.05 * omega, precision=prec)
    ref = orc.Problem(shape, omega, c, a, zeta, m_real=4, m_layer=3, a_floor=0.05 * omega)
    u = _rand(shape, 4)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    if prec == "mixed":
        u = u.astype(np.complex64).astype(np.complex128)
    y = plan.matvec(torch.from_numpy(u).to(dev).to(dt)).cpu().numpy()
    assert rel(y, ref.matvec(u)) < tol


def test_plain_and_left_gmres_match_oracle(orc, hp, dev):
    """side="none": plain restarted GMRES(10) on P_N x = f (the unpreconditioned reference of the
    GMRES comparison in Section 5.1) and side="left": Q P_N x = Q f as Eqn. MainDiscretePrecond
    is written, both against the oracle's GMRES on the same side."""
    _case("plain_left_gmres", n=36)
    w = inputs.workload("2d_inclusion", n=36, ppw=6.0)
    plan = hp.plan_from_workload(w)
    ref = orc.from_workload(w)
    f = torch.from_numpy(w.f).to(dev)
    for side, rtol in (("none", 1e-6), ("left", 1e-9)):
        x, info = plan.solve(f, rtol=rtol, restart=10, max_cycles=400, side=side)
        xr, res = ref.gmres(w.f[0], restart=10, rtol=rtol, max_cycles=400, side=side)
        assert info[0].status == 0 and res["status"] == 0, side
        true = rel(ref.matvec(x.cpu().numpy()[0]), w.f[0])
        assert abs(info[0].rel_true_residual - true) <= 1e-6 * true + 1e-15, (side, info[0], true)
        if side == "none":
            assert true <= rtol * 1.001
        assert abs(info[0].iters - res["iters"]) <= max(3, res["iters"] // 20), (side, info[0].iters, res["iters"])
    # a fixed budget of 30 steps: the preconditioned residual is far below the plain one
    _, ip = plan.solve(f, rtol=1e-15, restart=10, max_cycles=3)
    _, iq = plan.solve(f, rtol=1e-15, restart=10, max_cycles=3, side="none")
    assert ip[0].iters == iq[0].iters == 30
    assert ip[0].rel_true_residual < 1e-2 * iq[0].rel_true_residual


def test_long_restart_gmres_matches_oracle(orc, hp, dev):
    """GMRES(64): Arnoldi steps past 32 take the eight-wave dot-product sweep and stage more
    than 1024 Hessenberg entries in the finishing kernel; plain (many steps per cycle) and
    right-preconditioned solves against the oracle's GMRES(64)."""
    _case("long_restart_gmres", n=36)
    w = inputs.workload("2d_inclusion", n=36, ppw=6.0)
    plan = hp.plan_from_workload(w)
    ref = orc.from_workload(w)
    f = torch.from_numpy(w.f).to(dev)
    for side, rtol in (("none", 1e-10), ("right", 1e-12)):
        x, info = plan.solve(f, rtol=rtol, restart=64, max_cycles=100, side=side)
        xr, res = ref.gmres(w.f[0], restart=64, rtol=rtol, max_cycles=100, side=side)
        assert info[0].status == 0 and res["status"] == 0, side
        true = rel(ref.matvec(x.cpu().numpy()[0]), w.f[0])
        assert true <= rtol * 1.001, (side, true)
        assert abs(info[0].rel_true_residual - true) <= 1e-6 * true + 1e-15, (side, info[0], true)
        assert abs(info[0].iters - res["iters"]) <= max(2, res["iters"] // 50), (side, info[0].iters, res["iters"])
        if side == "none":
            assert res["iters"] > 64      # a full cycle of 64 steps and a second one


@pytest.mark.parametrize("shape,precision", [((4096, 8), "fp64"), ((8, 4096), "fp64"), ((4096, 8), "mixed"),
                                             ((8, 4096), "mixed"), ((2048, 16), "fp64"), ((8, 4096, 8), "fp64")])
def test_longest_power_of_two_lines(orc, hp, dev, shape, precision):
    """Power-of-two lines at the length limit in every role (strided axis 0, the 3-D middle
    axis and the contiguous last axis), in both precisions, against the oracle.  FP64 columns
    longer than 2048 take the LDS-resident kernels (the register-tile one would not fit)."""
    _case("pow2_limit_apply", shape=shape, precision=precision)
    c, zeta = _media(shape, 7 + sum(shape), False)
    omega = 2 * np.pi * min(shape) / 4
    a = np.full(shape, 0.05 * omega)
    kw = dict(m_real=6, m_layer=3, a_floor=0.05 * omega)
    plan = hp.Plan(shape, omega, c, a, zeta, precision=precision, **kw)
    ref = orc.Problem(shape, omega, c, a, zeta, **kw)
    v = _rand(shape, 4)
    if precision == "fp64":
        u = plan.apply(torch.from_numpy(v).to(dev)).cpu().numpy()
        assert rel(u, ref.apply(v)) < 1e-12
    else:
        u = plan.apply(torch.from_numpy(v).to(dev).to(torch.complex64)).cpu().numpy()
        assert rel(u, ref.apply(v.astype(np.complex64).astype(np.complex128))) < 1e-5
