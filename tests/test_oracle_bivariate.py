"""Pins of the oracle's bivariate (c, a) interpolation: the extension the concluding
remarks of the paper call for when the damping a(x) is independent of the wave speed
(the interpolation of Section 4.1 over [c_min, c_max] x [a_min, a_max]).

* the tensor-product hat weights sum to one and reproduce c and a (bilinear reproduction);
  at a node they select that node;
* media whose values are node values: Q_M equals the exact operator of Eqn. Precond
  (brute force, with a(x) pointwise) to rounding;
* smooth independent c and a: the error against the exact operator falls about 4x when
  both node spacings halve (second order in each variable), and is far below that of the
  univariate scheme, whose single damping per speed node cannot follow a;
* uniform a reduces the scheme to the univariate one.
"""
import numpy as np
import pytest

from paper_2409_16172_amd import inputs
from tests.util import rel


def _smooth_media(n, seed, alo=2.0, ahi=30.0):
    shape = (n, n)
    c = inputs.gaussian_random_field(shape, n / 6, seed, lo=0.9, hi=1.3)
    a = inputs.gaussian_random_field(shape, n / 5, seed + 100, lo=alo, hi=ahi)
    return shape, c, a


def test_bilinear_weights_reproduce_c_and_a(orc):
    shape, c, a = _smooth_media(16, 1)
    p = orc.Problem(shape, 20.0, c, a, m_real=5, m_damp=4)
    st = p.setup()
    assert st["Ma"] == 4 and st["K"] == 20
    cn, an = st["cnode"], st["anode"]
    assert cn[0] == c.min() and cn[-1] == c.max() and an[0] == a.min() and an[-1] == a.max()
    rng = np.random.default_rng(3)
    for _ in range(50):
        cv = rng.uniform(cn[0], cn[-1])
        av = rng.uniform(an[0], an[-1])
        w = p.weights_ca(cv, av)
        W = w.reshape(4, 5)            # node m + M r
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs((W * cn[None, :]).sum() - cv) < 1e-13
        assert abs((W * an[:, None]).sum() - av) < 1e-12
        assert np.count_nonzero(w) <= 4 and w.min() >= 0.0
    w = p.weights_ca(cn[2], an[1])
    assert w[2 + 5 * 1] == 1.0 and np.count_nonzero(w) == 1
    g = st["gamma"].reshape(4, 5)
    ah = st["ahat"].reshape(4, 5)
    assert np.all(g.real == cn[None, :]) and np.all(g.imag == 0)
    assert np.all(ah == an[:, None])


def test_node_valued_media_give_the_exact_operator(orc):
    n = 16
    shape = (n, n)
    rng = np.random.default_rng(5)
    cvals = np.array([1.0, 1.25, 1.5])
    avals = np.array([0.0, 10.0, 20.0])
    c = cvals[rng.integers(0, 3, size=shape)]
    a = avals[rng.integers(0, 3, size=shape)]
    c.flat[:3] = cvals
    a.flat[:3] = avals
    omega = 2 * np.pi * 2.3
    p = orc.Problem(shape, omega, c, a, m_real=3, m_damp=3)
    st = p.setup()
    assert np.allclose(st["cnode"], cvals, rtol=0, atol=1e-15) and np.allclose(st["anode"], avals, rtol=0, atol=1e-14)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert rel(p.apply(v), p.exact_psdo(v)) < 1e-13
    # the univariate scheme cannot be exact here: one damping per speed node
    p1 = orc.Problem(shape, omega, c, a, m_real=3)
    assert rel(p1.apply(v), p1.exact_psdo(v)) > 1e-3


def test_second_order_in_both_variables(orc):
    # damping bounded away from zero keeps q smooth in a near the resonance |xi| = omega/c,
    # where q ~ 1/(i omega a); with a near zero the decay is pre-asymptotic
    shape, c, a = _smooth_media(32, 2, 20.0, 40.0)
    omega = 2 * np.pi * 3
    rng = np.random.default_rng(7)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    errs = []
    for m in (2, 3, 5):      # node spacings h, h/2, h/4 in both variables (K up to 25)
        p = orc.Problem(shape, omega, c, a, m_real=m, m_damp=m)
        errs.append(rel(p.apply(v), p.exact_psdo(v)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 2.8 < r1 < 5.5 and 2.8 < r2 < 5.5, errs
    uni = orc.Problem(shape, omega, c, a, m_real=25)
    assert rel(uni.apply(v), uni.exact_psdo(v)) > 10 * errs[2]


def test_uniform_damping_reduces_to_the_univariate_scheme(orc):
    shape, c, _ = _smooth_media(16, 4)
    a = np.full(shape, 7.5)
    v = np.random.default_rng(9).standard_normal(shape) + 0j
    p2 = orc.Problem(shape, 15.0, c, a, m_real=6, m_damp=4)
    assert p2.setup()["Ma"] == 1 and p2.setup()["K"] == 6
    p1 = orc.Problem(shape, 15.0, c, a, m_real=6)
    assert np.abs(p2.apply(v) - p1.apply(v)).max() == 0.0


def test_bivariate_rejects_layer_and_higher_degree(orc):
    shape, c, a = _smooth_media(16, 6)
    zeta = inputs.frame_layer(shape, 3, 0.2)
    cb = inputs.blend_to_background(c, 3, 1.0, taper=2)
    with pytest.raises(orc.OracleError):
        orc.Problem(shape, 15.0, cb, a, zeta, m_real=5, m_damp=3).setup()
    with pytest.raises(orc.OracleError):
        orc.Problem(shape, 15.0, c, a, m_real=5, m_damp=3, interp_order=2).setup()
