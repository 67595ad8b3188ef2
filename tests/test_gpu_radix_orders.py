"""Mixed-radix lines under every radix schedule the plans offer (largest radix first,
ascending, largest last, radices 2-5 only), forced through the tuning cache: each
schedule's applies agree with the oracle on 2-D and 3-D grids whose lines take
composite stage radices 6, 8, 9, 10, 12, 15 and 16 (and 2880-, 3600- and 4800-point lines)."""
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


def _problem(shape, seed):
    n = min(shape)
    c = inputs.gaussian_random_field(shape, max(2.0, n / 6), seed, lo=0.8, hi=1.3)
    width = max(2, n // 8)
    c = inputs.blend_to_background(c, width, 1.0, taper=max(2, min(8, n // 8)))
    zeta = inputs.frame_layer(shape, width, 0.133)
    omega = 2 * np.pi * n / 6
    return c, np.full(shape, 0.05 * omega), zeta, omega


CASES = [((240, 360), "fp64"), ((150, 96), "mixed"), ((18, 4800), "fp64"), ((36, 90, 80), "fp64"),
         ((30, 12, 18), "mixed"), ((4800, 10), "mixed"), ((10, 3600), "mixed"), ((2880, 12), "fp64")]


@pytest.mark.parametrize("order", [0, 1, 2, 3])
@pytest.mark.parametrize("shape,precision", CASES)
def test_radix_order_apply_matches_oracle(orc, hp, dev, shape, precision, order, tmp_path, monkeypatch):
    print(f"[case] radix order {order} shape={shape} {precision}", flush=True)
    c, a, zeta, omega = _problem(shape, 7 + sum(shape))
    kw = dict(m_real=5, m_layer=2, a_floor=0.05 * omega)
    probe = hp.Plan(shape, omega, c, a, zeta, precision=precision, **kw)
    K = probe.info()["K"]
    probe.close()
    n = list(shape) + [1] * (3 - len(shape))
    prec = 0 if precision == "fp64" else 1
    path = tmp_path / "tune.txt"
    path.write_text("".join(f"hp-tune {len(shape)} {n[0]} {n[1]} {n[2]} {prec} {K} {s} 0 0 {order} 0\n"
                            for s in range(5)))
    monkeypatch.setenv("HP_TUNE_CACHE", str(path))
    plan = hp.Plan(shape, omega, c, a, zeta, precision=precision, **kw)
    rng = np.random.default_rng(order + 11)
    v_np = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    u = plan.apply(torch.from_numpy(v_np).to(dev).to(dt)).cpu().numpy()
    ref = orc.Problem(shape, omega, c, a, zeta, **kw).apply(v_np)
    err = rel(u, ref)
    print(f"    tune {plan.info()['tune']} rel err {err:.2e}", flush=True)
    assert err < (1e-12 if precision == "fp64" else 1e-5)
    plan.close()
