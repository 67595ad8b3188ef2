"""hp_apply_precond_static (the apply for callers that cannot allocate) against
hp_apply_precond, through the C ABI: the same kernels on the library's static device
workspace instead of the plan's, so the results must be bitwise the same.  Two calls in
a row, the second on a smaller input; a call whose input holds NaN and Inf (which leaves
non-finite values in the shared workspace) followed by a clean call, which must not see
them; 3-D and mixed-radix grids; a batch larger than the workspace holds at once; and the
refusal of a field that does not fit."""
import numpy as np
import pytest

from paper_2409_16172_amd import inputs

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


def _plan(hp, shape, precision, M, seed, max_nrhs=1):
    nmin = min(shape)
    width = max(2, nmin // 8)
    c = inputs.gaussian_random_field(shape, max(2.0, nmin / 8), seed)
    c = inputs.blend_to_background(c, width, 1.0, taper=2)
    zeta = inputs.frame_layer(shape, width, 0.133)
    omega = 2 * np.pi * nmin / 8
    a = np.full(shape, 0.05 * omega)
    return hp.Plan(shape, omega, c, a, zeta, m_real=M, m_layer=3, a_floor=0.05 * omega, precision=precision,
                   max_nrhs=max_nrhs)


def _v(shape, seed, nrhs, dt, dev):
    rng = np.random.default_rng(seed)
    sh = (nrhs,) + tuple(shape)
    v = rng.standard_normal(sh) + 1j * rng.standard_normal(sh)
    return torch.from_numpy(v).to(dev).to(dt)


def _same(hp, plan, v, what):
    ref = plan.apply(v)
    torch.cuda.synchronize()
    out = torch.empty_like(v)
    got = plan.apply_static(v, out=out)
    torch.cuda.synchronize()
    assert got.data_ptr() == out.data_ptr()
    assert torch.isfinite(ref).all(), what
    assert torch.equal(got, ref), (what, (got - ref).abs().max().item())
    print(f"[no_alloc] {what}: bitwise equal to hp_apply_precond", flush=True)


def test_static_apply_two_calls_second_smaller(hp, dev):
    print("[case] static apply 256^2 fp64 x2, then 64^2 mixed", flush=True)
    big = _plan(hp, (256, 256), "fp64", 16, 1, max_nrhs=2)
    small = _plan(hp, (64, 64), "mixed", 8, 2)
    _same(hp, big, _v((256, 256), 3, 2, torch.complex128, dev), "256^2 fp64, 2 fields")
    _same(hp, small, _v((64, 64), 4, 1, torch.complex64, dev), "64^2 mixed, 1 field")
    big.close()
    small.close()


def test_static_apply_ignores_stale_nonfinite_scratch(hp, dev):
    print("[case] static apply with NaN/Inf input, then a clean smaller call", flush=True)
    p1 = _plan(hp, (128, 128), "fp64", 12, 5)
    v = _v((128, 128), 6, 1, torch.complex128, dev)
    v[0, 3, 4] = float("nan")
    v[0, 70, 9] = float("inf")
    p1.apply_static(v)
    torch.cuda.synchronize()
    p2 = _plan(hp, (64, 32), "fp64", 6, 7)
    _same(hp, p2, _v((64, 32), 8, 1, torch.complex128, dev), "64x32 fp64 after a non-finite call")
    p1.close()
    p2.close()


@pytest.mark.parametrize("shape,prec", [((32, 32, 32), "fp64"), ((16, 64, 32), "mixed"), ((120, 96), "fp64"),
                                        ((60, 40), "mixed")])
def test_static_apply_3d_and_mixed_radix(hp, dev, shape, prec):
    print(f"[case] static apply {shape} {prec}", flush=True)
    p = _plan(hp, shape, prec, 6, sum(shape))
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    _same(hp, p, _v(shape, 9, 1, dt, dev), f"{shape} {prec}")
    p.close()


def test_static_apply_batch_in_chunks_and_refusal(hp, dev):
    print("[case] static apply batch of 5 at 256^2 fp64 (chunks), refusal at 1024^2", flush=True)
    p = _plan(hp, (256, 256), "fp64", 16, 11, max_nrhs=5)
    # one field needs 20 * 2^16 * 16 B = 20 MiB: three fit in the 64 MiB workspace
    _same(hp, p, _v((256, 256), 12, 5, torch.complex128, dev), "256^2 fp64, 5 fields in chunks")
    p.close()
    big = _plan(hp, (1024, 1024), "fp64", 16, 13)
    v = _v((1024, 1024), 14, 1, torch.complex128, dev)
    with pytest.raises(hp.HelmpreError) as e:
        big.apply_static(v)
    assert e.value.code == hp.HP_E_INVALID and "static workspace holds" in str(e.value)
    big.close()
