"""GPU parity of the bivariate (c, a) interpolation (m_damp >= 2: nodes (c_m, a_r), tensor-
product hat weights; the extension of Section 4.1 the concluding remarks of the paper call
for when the damping does not depend on the wave speed) against the oracle, through the
C ABI."""
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


def _media(shape, seed, omega):
    n = min(shape)
    c = inputs.gaussian_random_field(shape, max(2.0, n / 8), seed, lo=0.8, hi=1.3)
    a = inputs.gaussian_random_field(shape, max(2.0, n / 6), seed + 1000, lo=0.05 * omega, hi=0.6 * omega)
    return c, a


SHAPES = [((64, 64), 5, 4), ((128, 96), 6, 3), ((60, 40), 4, 4), ((32, 16, 24), 4, 3), ((16, 16), 2, 2)]


@pytest.mark.parametrize("shape,M,Ma", SHAPES)
def test_bivariate_apply_matches_oracle(orc, hp, dev, shape, M, Ma):
    print(f"[case] bivariate_apply shape={shape} M={M} Ma={Ma}", flush=True)
    omega = 2 * np.pi * min(shape) / 8
    c, a = _media(shape, 11 + sum(shape), omega)
    ref = orc.Problem(shape, omega, c, a, m_real=M, m_damp=Ma)
    st = ref.setup()
    plan = hp.Plan(shape, omega, c, a, m_real=M, m_damp=Ma)
    info = plan.info()
    assert info["K"] == st["K"] == M * Ma and info["m_damp"] == Ma
    assert np.abs(info["anode"] - st["anode"]).max() <= 1e-12 * st["anode"].max()
    assert np.abs(info["ahat"] - st["ahat"]).max() <= 1e-12 * st["ahat"].max()
    rng = np.random.default_rng(M + Ma)
    v = rng.standard_normal((2,) + shape) + 1j * rng.standard_normal((2,) + shape)
    ue = ref.apply(v)
    u = plan.apply(torch.from_numpy(v).to(dev)).cpu().numpy()
    err = max(rel(u[r], ue[r]) for r in range(2))
    print(f"    FP64 {err:.2e}", flush=True)
    assert err < 1e-12
    p32 = hp.Plan(shape, omega, c, a, m_real=M, m_damp=Ma, precision="mixed")
    u32 = p32.apply(torch.from_numpy(v).to(dev).to(torch.complex64)).cpu().numpy()
    assert max(rel(u32[r], ue[r]) for r in range(2)) < 1e-5


def test_bivariate_solve_reaches_tolerance_in_the_oracle_residual(orc, hp, dev):
    print("[case] bivariate_solve 128^2", flush=True)
    shape = (128, 128)
    omega = 2 * np.pi * 12
    c, a = _media(shape, 5, omega)
    f = inputs.gaussian_source(shape, 2.0, (0.1, -0.05))[None].astype(np.complex128)
    ref = orc.Problem(shape, omega, c, a, m_real=6, m_damp=4)
    plan = hp.Plan(shape, omega, c, a, m_real=6, m_damp=4)
    x, info = plan.solve(torch.from_numpy(f).to(dev), rtol=1e-9)
    xr = x.cpu().numpy()[0]
    r = np.linalg.norm(f[0] - ref.matvec(xr)) / np.linalg.norm(f[0])
    print(f"    iters {info[0].iters}, oracle residual {r:.2e}", flush=True)
    assert info[0].status == 0 and r <= 1.5e-9
    # the GPU's iteration count matches the oracle's GMRES with the same preconditioner
    # (same Krylov space; the orthogonalisations differ in rounding only)
    _, oinfo = ref.gmres(f[0], rtol=1e-9)
    print(f"    oracle GMRES iters {oinfo['iters']}", flush=True)
    assert abs(info[0].iters - oinfo["iters"]) <= 2


def test_bivariate_uniform_damping_falls_back(hp, dev):
    shape = (64, 64)
    omega = 2 * np.pi * 6
    c, _ = _media(shape, 3, omega)
    a = np.full(shape, 0.2 * omega)
    p2 = hp.Plan(shape, omega, c, a, m_real=5, m_damp=4)
    p1 = hp.Plan(shape, omega, c, a, m_real=5)
    assert p2.info()["m_damp"] == 0 and p2.info()["K"] == 5
    v = torch.from_numpy(np.random.default_rng(1).standard_normal(shape) + 0j).to(dev)
    assert torch.equal(p2.apply(v), p1.apply(v))


def test_bivariate_error_paths(hp, dev):
    shape = (64, 64)
    omega = 2 * np.pi * 6
    c, a = _media(shape, 4, omega)
    with pytest.raises(hp.HelmpreError):      # K = 9 * 8 > 64
        hp.Plan(shape, omega, c, a, m_real=9, m_damp=8)
    with pytest.raises(hp.HelmpreError):      # no higher-degree basis in the bivariate scheme
        hp.Plan(shape, omega, c, a, m_real=5, m_damp=3, interp_order=2)
    zeta = inputs.frame_layer(shape, 6, 0.133)
    cb = inputs.blend_to_background(c, 6, 1.0, taper=4)
    with pytest.raises(hp.HelmpreError):      # no absorbing layer
        hp.Plan(shape, omega, cb, a, zeta, m_real=5, m_damp=3)
