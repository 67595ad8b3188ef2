"""GPU parity at every transform length the benchmark workloads instantiate, through the
C ABI, against the CPU oracle, element by element as well as by the 2-norm.

The pass kernels are compiled per line length, and the long lines use different
workgroup shapes and LDS sizes from the short ones.  Thin grids reach each long-line
kernel cheaply: (2048, 16) puts 2048-point lines on the strided axis (the symbol pass),
(16, 2048) on the contiguous axis (the forward and combine passes); (16, 256, 16) and
(16, 128, 16) put them on the middle axis of a 3-D grid (its forward and inverse passes).
The full 2048^2 applies (FP64 and mixed), the 1024^2 FP64 solve of the benchmark (its
steps compute the stencil inside the dot-product sweep) and a mixed-precision served mix
with 128^3 requests complete the list.

Bars: FP64 apply <= 1e-12 and mixed <= 1e-5, both as ||u - u_o|| / ||u_o|| and as
max |u - u_o| / max |u_o| (no single point may be off by more than that fraction of the
field's largest value); solves reach the FP64 true residual rtol recomputed by the oracle.
"""
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


def maxrel(a, b):
    """max |a - b| over the field / max |b|."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _media(shape, seed):
    nmin = min(shape)
    width = max(2, nmin // 8)
    c = inputs.gaussian_random_field(shape, max(2.0, nmin / 4), seed)
    c = inputs.blend_to_background(c, width, 1.0, taper=2)
    zeta = inputs.frame_layer(shape, width, 0.133)
    return c, zeta


def _v32(shape, seed, nrhs=None):
    """Random complex values exactly representable in complex64, so that the FP64 and the
    mixed plan see the same input and one oracle apply serves both."""
    rng = np.random.default_rng(seed)
    sh = tuple(shape) if nrhs is None else (nrhs,) + tuple(shape)
    v = (rng.standard_normal(sh) + 1j * rng.standard_normal(sh)).astype(np.complex64)
    return v.astype(np.complex128)


def _check(u, ue, tol, what):
    r2, rm = rel(u, ue), maxrel(u, ue)
    print(f"[{what}] rel2 {r2:.3e} relmax {rm:.3e}", flush=True)
    assert r2 <= tol and rm <= tol, (what, r2, rm)


THIN = [
    ((2048, 16), 16), ((16, 2048), 16), ((1024, 16), 16), ((16, 1024), 16),
    ((16, 256, 16), 8), ((16, 128, 16), 8), ((256, 16, 16), 8), ((16, 16, 256), 8),
]


@pytest.mark.parametrize("shape,M", THIN)
def test_long_line_kernels_match_oracle(orc, hp, dev, shape, M):
    _case("long_lines", shape=shape, M=M)
    c, zeta = _media(shape, seed=sum(shape) + len(shape))
    omega = 2 * np.pi * min(shape) / 4
    a = np.full(shape, 0.05 * omega)
    kw = dict(m_real=M, m_layer=3, a_floor=0.05 * omega)
    ref = orc.Problem(shape, omega, c, a, zeta, **kw)
    v = _v32(shape, 31, nrhs=2)
    ue = ref.apply(v)
    for prec, dt, tol in (("fp64", torch.complex128, 1e-12), ("mixed", torch.complex64, 1e-5)):
        plan = hp.Plan(shape, omega, c, a, zeta, precision=prec, max_nrhs=2, **kw)
        u = plan.apply(torch.from_numpy(v).to(dev).to(dt)).cpu().numpy()
        for r in range(2):
            _check(u[r], ue[r], tol, f"{prec} {shape} rhs {r}")
        plan.close()


def test_full_2048_applies_match_oracle(orc, hp, dev):
    """The 2048^2 workload (24 + 3 nodes) at full size, mixed (its benchmark precision) and
    FP64, against one oracle apply of the same complex64-exact input."""
    w = inputs.workload("2d_2048_grf")
    _case("apply_full_2048", K=w.m_real + w.m_layer)
    v = _v32(w.shape, 41)
    print("[oracle] 2048^2 apply (about 10-20 s)", flush=True)
    ue = orc.from_workload(w).apply(v)
    for prec, dt, tol in (("mixed", torch.complex64, 1e-5), ("fp64", torch.complex128, 1e-12)):
        plan = hp.plan_from_workload(w, precision=prec)
        u = plan.apply(torch.from_numpy(v).to(dev).to(dt)).cpu().numpy()
        _check(u, ue, tol, f"{prec} 2048^2")
        plan.close()


def test_full_1024_mixed_apply_matches_oracle(orc, hp, dev):
    """The 1024^2 workload in mixed precision (the benchmark's mixed leg)."""
    w = inputs.workload("2d_1024_grf")
    _case("apply_full_1024_mixed", K=w.m_real + w.m_layer)
    v = _v32(w.shape, 43)
    ue = orc.from_workload(w).apply(v)
    plan = hp.plan_from_workload(w, precision="mixed")
    u = plan.apply(torch.from_numpy(v).to(dev).to(torch.complex64)).cpu().numpy()
    _check(u, ue, 1e-5, "mixed 1024^2")
    plan.close()


def test_full_1024_fp64_apply_pointwise(orc, hp, dev):
    """The 1024^2 FP64 apply of the benchmark, point by point."""
    w = inputs.workload("2d_1024_grf")
    _case("apply_full_1024_fp64_pointwise", K=w.m_real + w.m_layer)
    v = _v32(w.shape, 47)
    ue = orc.from_workload(w).apply(v)
    plan = hp.plan_from_workload(w)
    u = plan.apply(torch.from_numpy(v).to(dev)).cpu().numpy()
    _check(u, ue, 1e-12, "fp64 1024^2")
    plan.close()


def test_full_1024_fp64_solve_oracle_residual(orc, hp, dev):
    """The benchmark's solve (1024^2, FP64, rtol 1e-8): on this grid every Arnoldi step
    computes the stencil inside the dot-product sweep; the oracle recomputes the true
    residual of the returned solution, and the reported residual must equal it."""
    w = inputs.workload("2d_1024_grf")
    _case("solve_full_1024_fp64")
    plan = hp.plan_from_workload(w)
    f = torch.from_numpy(w.f).to(dev)
    x, info = plan.solve(f, rtol=1e-8, restart=30)
    ref = orc.from_workload(w)
    xh = x.cpu().numpy()[0]
    res = rel(ref.matvec(xh), w.f[0])
    print(f"[solve 1024^2] iters {info[0].iters} reported {info[0].rel_true_residual:.6e} oracle {res:.6e}",
          flush=True)
    assert info[0].status == 0 and res <= 1e-8
    assert abs(info[0].rel_true_residual - res) <= 1e-12
    plan.close()


def test_mixed_served_mix_with_3d_requests(orc, dev):
    """Continuous batching in mixed precision with 128^3 requests among 2-D ones: every
    served result equals the same request solved alone (bitwise) and reaches rtol in the
    oracle's FP64 residual."""
    from paper_2409_16172_amd import binding, serve
    reqs = serve.stream_requests(5, rate_per_s=200.0, seed=20240922,
                                 grids=((128, 128, 128), (256, 256), (128, 128)), precision="mixed",
                                 n_lambda=(8.0, 40.0))
    assert sum(len(r.workload.shape) == 3 for r in reqs) >= 1
    _case("serve_mixed", shapes=[r.workload.shape for r in reqs])
    srv = serve.Server(hbm_budget_bytes=64 << 30, max_active=4, steps_per_turn=2)
    done = srv.run(reqs, dev=dev)
    assert len(done) == 5
    for r in done:
        w = r.workload
        assert r.info[0].status == 0, (r.rid, r.info)
        plan = binding.plan_from_workload(w, max_nrhs=1)
        x1, i1 = plan.solve(torch.from_numpy(w.f[:1]).to(dev), rtol=1e-8)
        assert torch.equal(x1, r.x), r.rid
        res = rel(orc.from_workload(w).matvec(r.x.cpu().numpy()[0]), w.f[0])
        print(f"[serve] rid {r.rid} shape {w.shape} iters {r.info[0].iters} oracle residual {res:.3e}",
              flush=True)
        assert res <= 1e-8 * 1.001, (r.rid, res)
        plan.close()


@pytest.mark.parametrize("shape,mode", [((32, 256), "lagrange"), ((16, 1024), "lagrange"), ((24, 512), "bilinear"),
                                        ((16, 1024), "bilinear"), ((16, 16, 256), "lagrange"),
                                        ((16, 2048), "lagrange"), ((16, 2048), "bilinear")])
def test_mixed_combine_modes_on_long_rows(orc, hp, dev, shape, mode):
    """Mixed-precision combines of 256- to 1024-point rows (one row per wavefront) in the
    higher-degree and bilinear interpolation modes, against the oracle; FP64 too for
    1024- and 2048-point rows."""
    _case("combine_modes_long_rows", shape=shape, mode=mode)
    nmin = min(shape)
    omega = 2 * np.pi * nmin / 4
    if mode == "lagrange":
        c, zeta = _media(shape, seed=sum(shape) + 5)
        a = np.full(shape, 0.05 * omega)
        kw = dict(m_real=7, m_layer=3, a_floor=0.05 * omega, interp_order=3)
    else:
        c = inputs.gaussian_random_field(shape, max(2.0, nmin / 4), sum(shape), lo=0.8, hi=1.3)
        a = inputs.gaussian_random_field(shape, max(2.0, nmin / 3), sum(shape) + 1, lo=0.05 * omega, hi=0.6 * omega)
        zeta = None
        kw = dict(m_real=5, m_damp=3)
    v = _v32(shape, 53, nrhs=2)
    ue = orc.Problem(shape, omega, c, a, zeta, **kw).apply(v)
    precs = [("mixed", torch.complex64, 1e-5)]
    if shape[-1] >= 1024:   # FP64 1024- and 2048-point rows take the lane exchange in every combine mode
        precs.append(("fp64", torch.complex128, 1e-12))
    for prec, dt, tol in precs:
        plan = hp.Plan(shape, omega, c, a, zeta, precision=prec, max_nrhs=2, **kw)
        u = plan.apply(torch.from_numpy(v).to(dev).to(dt)).cpu().numpy()
        for r in range(2):
            _check(u[r], ue[r], tol, f"{prec} {mode} {shape} rhs {r}")
        plan.close()
