"""Pins of the oracle's layer tensor: interpolation on a tensor grid of (Re gamma, Im gamma)
nodes (the second form of the bivariate extension), so that the wave speed need not equal
c_o inside the absorbing layer (the restriction of the two-leg scheme of Eqn. 405).

* the tensor-product hat weights sum to one and reproduce Re gamma = c and Im gamma = -c zeta;
* media whose (c, -c zeta) are node values: Q_M equals the exact operator of Eqn. Precond
  with the complex speed of Eqn. Complex_wave_speed (brute force) to rounding;
* smooth c varying through the layer: the error against the exact operator falls about 4x
  when both node spacings halve;
* the two-leg scheme rejects such media; on media it accepts (c = c_o in the layer, c_o a
  speed node) the tensor scheme is the same operator.
"""
import numpy as np
import pytest

from paper_2409_16172_amd import inputs
from tests.util import rel


def _layer_media(n, seed, width=5):
    shape = (n, n)
    c = inputs.gaussian_random_field(shape, n / 6, seed, lo=0.9, hi=1.3)   # varies in the layer too
    zeta = inputs.frame_layer(shape, width, 0.2)
    return shape, c, zeta


def test_tensor_weights_reproduce_re_and_im_gamma(orc):
    shape, c, zeta = _layer_media(16, 1)
    p = orc.Problem(shape, 20.0, c, None, zeta, m_real=5, m_layer=3, layer_tensor=True)
    st = p.setup()
    assert st["tensor"] == 1 and st["Ma"] == 4 and st["K"] == 20 and st["Mt"] == 0
    cn, gn = st["cnode"], st["anode"]
    assert gn[-1] == 0.0 and abs(gn[0] + (c * zeta).max()) < 1e-15
    rng = np.random.default_rng(3)
    for _ in range(50):
        cv = rng.uniform(cn[0], cn[-1])
        gv = rng.uniform(gn[0], 0.0)
        w = p.weights_ca(cv, gv)
        W = w.reshape(4, 5)
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs((W * cn[None, :]).sum() - cv) < 1e-13
        assert abs((W * gn[:, None]).sum() - gv) < 1e-13
    gam = st["gamma"].reshape(4, 5)
    assert np.all(gam.real == cn[None, :]) and np.all(gam.imag == gn[:, None])


def test_node_valued_layer_media_give_the_exact_operator(orc):
    n = 16
    shape = (n, n)
    rng = np.random.default_rng(8)
    cvals = np.array([1.0, 1.25, 1.5])
    delta = 0.1
    c = cvals[rng.integers(0, 3, size=shape)]
    j = rng.integers(0, 4, size=shape)
    c.flat[:3] = cvals
    j.flat[0] = 3
    zeta = j * delta / c                       # -c zeta = -j delta, a node value
    omega = 2 * np.pi * 2.1
    a = np.full(shape, 3.0)
    p = orc.Problem(shape, omega, c, a, zeta, m_real=3, m_layer=3, layer_tensor=True)
    st = p.setup()
    assert np.allclose(st["anode"], [-0.3, -0.2, -0.1, 0.0], rtol=0, atol=1e-15)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert rel(p.apply(v), p.exact_psdo(v)) < 1e-13
    with pytest.raises(orc.OracleError):       # the two-leg scheme needs c = c_o in the layer
        orc.Problem(shape, omega, c, a, zeta, m_real=3, m_layer=3).setup()


def test_second_order_in_both_parts_of_gamma(orc):
    shape, c, zeta = _layer_media(32, 2, width=8)
    omega = 2 * np.pi * 3
    a = np.full(shape, 0.3 * omega)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    errs = []
    # spacings halve along Re gamma (2, 4, 8 intervals) and Im gamma (1, 2, 4); K up to 45
    for m, ml in ((3, 1), (5, 2), (9, 4)):
        p = orc.Problem(shape, omega, c, a, zeta, m_real=m, m_layer=ml, layer_tensor=True)
        errs.append(rel(p.apply(v), p.exact_psdo(v)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 2.8 < r1 < 5.5 and 2.8 < r2 < 5.5, errs


def test_reduces_to_the_two_leg_scheme_when_c_is_c_o_in_the_layer(orc):
    # with c = c_o in the layer and c_o among the equidistant speed nodes, the tensor grid's
    # row Im gamma = 0 carries the real leg and its column c_o the layer leg of Eqn. 405,
    # and every other node has zero weight: the two schemes are the same operator
    shape, c, zeta = _layer_media(32, 4, width=6)
    c = inputs.blend_to_background(c, 6, 1.0, taper=3)
    inner = zeta == 0
    c[inner] = 0.9 + (c[inner] - c[inner].min()) * (0.4 / (c[inner].max() - c[inner].min()))
    c[~inner] = 1.0                            # speeds [0.9, 1.3]: c_o = 1.0 is a node of 5
    omega = 2 * np.pi * 3
    a = np.full(shape, 0.3 * omega)
    v = np.random.default_rng(9).standard_normal(shape) + 1j * np.random.default_rng(10).standard_normal(shape)
    two = orc.Problem(shape, omega, c, a, zeta, m_real=5, m_layer=3)
    ten = orc.Problem(shape, omega, c, a, zeta, m_real=5, m_layer=3, layer_tensor=True)
    assert np.allclose(two.setup()["cnode"], ten.setup()["cnode"], rtol=0, atol=1e-15)
    assert rel(ten.apply(v), two.apply(v)) < 1e-14
    assert rel(ten.apply(v), ten.exact_psdo(v)) < 0.1
