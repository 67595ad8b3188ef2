"""Pins of the oracle's interpolated preconditioner Q_M (Eqn. 103/105, 403/405).

T3  weights: a node is reproduced exactly, the weights sum to one and
    reproduce the complex speed linearly (piecewise-linear hats, Section 4.1/4.4).
T4  a single Fourier mode is mapped to [sum_n w_n(x) q_n(k)] times the mode
    (Eqn. 403 applied to one mode); a non-square grid catches a swapped axis.
T5  media that only take node values: Q_M equals the exact operator Q of
    Eqn. Precond, computed by brute force.
T6  the interpolation error decays like h_M^2 (Lemma 3, Theorem 2), with the
    pointwise bound h^2/8 max |d^2 q/dc^2| built from the paper's printed
    second derivative.
    The printed first and second c-derivatives of q_{-2} (Section 4.3) match
    finite differences of the oracle's symbol.
Q_1 special case (Eqn. OneInterpPoint) and the homogeneous case: with the
stencil's own symbol Q_1 inverts P_N exactly (one-term expansion, Section 3).
"""
import numpy as np
import pytest

from paper_2409_16172_amd import inputs
from tests.util import rel


def _mode(shape, k, length=1.0):
    xs = inputs.mesh(shape, length)
    ph = sum(2 * np.pi * kk / length * (x + 0.5 * length) for kk, x in zip(k, xs))
    return np.exp(1j * ph)


def _xi2(shape, k, length=1.0):
    return sum((2 * np.pi * kk / length) ** 2 for kk in k)


def _layer_medium(n=32, width=4):
    shape = (n, n)
    xs = inputs.mesh(shape)
    c = 1.0 + 0.25 * np.exp(-(xs[0] ** 2 + xs[1] ** 2) / 0.02) - 0.1 * np.exp(-((xs[0] - 0.2) ** 2 + xs[1] ** 2) / 0.005)
    c = inputs.blend_to_background(c, width, 1.0, taper=3)
    zeta = inputs.frame_layer(shape, width, 0.2)
    return shape, c, zeta


# ---------------------------------------------------------------- T3
def test_weights_reproduce_nodes_and_sum_to_one(orc):
    shape, c, zeta = _layer_medium()
    omega = 2 * np.pi * 4
    p = orc.Problem(shape, omega, c, np.full(shape, 3.0), zeta, m_real=6, m_layer=3)
    st = p.setup()
    M, Mt, K, mo = st["M"], st["Mt"], st["K"], st["mo"]
    assert K == M + Mt and Mt == 3 and abs(st["cnode"][mo] - 1.0) == 0
    for m, cn in enumerate(st["cnode"]):                   # real nodes, no layer
        w = p.weights(cn, 0.0)
        e = np.zeros(K)
        e[m] = 1
        assert np.array_equal(w, e), (m, w)
    for j in range(1, Mt + 1):                             # layer nodes
        w = p.weights(1.0, st["znode"][j])
        e = np.zeros(K)
        e[M + j - 1] = 1
        assert np.abs(w - e).max() < 1e-15, (j, w)
    rng = np.random.default_rng(3)
    gam = st["gamma"]
    for _ in range(200):
        if rng.random() < 0.5:
            cv, zv = rng.uniform(st["cmin"], st["cmax"]), 0.0
        else:
            cv, zv = 1.0, rng.uniform(0, st["zmax"])
        w = p.weights(cv, zv)
        assert np.count_nonzero(w) <= 2
        assert abs(w.sum() - 1) < 1e-15
        g = np.dot(w, gam)
        assert abs(g.real - cv) < 1e-14 and abs(g.imag - (-cv * zv)) < 1e-14


def test_node_placement_contains_background(orc):
    """With a layer c_o is a node (Section 4.4) and the end nodes are c_min, c_max (Section 4.1)."""
    shape = (16, 16)
    c = np.full(shape, 1.0)
    c[5:9, 5:9] = 1.3
    c[10, 10] = 0.7
    zeta = inputs.frame_layer(shape, 2, 0.1)
    for M in (2, 3, 5, 8, 16):
        st = orc.Problem(shape, 10.0, c, None, zeta, m_real=M, a_floor=1.0).setup()
        nodes = st["cnode"]
        assert nodes[0] == 0.7 and nodes[-1] == 1.3 and st["M"] == max(M, 3)
        assert nodes[st["mo"]] == 1.0 and np.all(np.diff(nodes) > 0)
    st = orc.Problem(shape, 10.0, c, None, None, m_real=5, a_floor=1.0).setup()
    assert np.allclose(np.diff(st["cnode"]), 0.15, rtol=0, atol=1e-15)   # equidistant without layer


# ---------------------------------------------------------------- T4
@pytest.mark.parametrize("shape,k", [((16, 32), (3, -5)), ((32, 32), (0, 7)), ((8, 8, 16), (1, -2, 5)),
                                     ((24, 36), (5, -11)), ((12, 20, 10), (-3, 4, 2))])
def test_fourier_mode_closed_form(orc, shape, k):
    n = shape[0]
    xs = inputs.mesh(shape)
    r2 = sum(x ** 2 for x in xs)
    c = 1.0 + 0.3 * np.exp(-r2 / 0.03)
    width = max(2, n // 8)
    c = inputs.blend_to_background(c, width, 1.0, taper=2)
    zeta = inputs.frame_layer(shape, width, 0.15)
    omega = 2 * np.pi * 3.3
    a = 0.7 * omega
    p = orc.Problem(shape, omega, c, np.full(shape, a), zeta, m_real=5, m_layer=3)
    st = p.setup()
    v = _mode(shape, k)
    u = p.apply(v)
    xi2 = _xi2(shape, k)
    qn = 1.0 / (omega ** 2 + 1j * omega * st["ahat"] - st["gamma"] ** 2 * xi2)
    ww = np.array([p.weights(cv, zv) for cv, zv in zip(c.ravel(), zeta.ravel())])
    expect = (ww @ qn).reshape(shape) * v
    assert np.abs(u - expect).max() < 1e-13 * np.abs(qn).max()


# ---------------------------------------------------------------- T5
def test_node_valued_media_equal_exact_operator(orc):
    n = 16
    shape = (n, n)
    rng = np.random.default_rng(11)
    nodes = np.array([0.8, 0.9, 1.0, 1.15, 1.3])
    c = nodes[rng.integers(0, len(nodes), size=shape)]
    width = 3
    e = inputs.boundary_distance_cells(shape)
    znodes = np.array([0.05, 0.1, 0.2])
    zeta = np.where(e < width, znodes[rng.integers(0, 3, size=shape)], 0.0)
    zeta[e == 0] = 0.2
    c[e < width] = 1.0
    omega = 2 * np.pi * 2.5
    a = np.full(shape, 4.0)
    p = orc.Problem(shape, omega, c, a, zeta, nodes_real=nodes, nodes_zeta=znodes)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert rel(p.apply(v), p.exact_psdo(v)) < 1e-13
    # automatic nodes on media whose values are the equidistant nodes themselves
    c2 = np.linspace(0.9, 1.2, 4)[rng.integers(0, 4, size=shape)]
    c2[0, 0], c2[0, 1] = 0.9, 1.2
    p2 = orc.Problem(shape, omega, c2, a, None, m_real=4)
    assert rel(p2.apply(v), p2.exact_psdo(v)) < 1e-13


# ---------------------------------------------------------------- T6
def test_interpolation_error_rate(orc):
    n = 32
    shape = (n, n)
    xs = inputs.mesh(shape)
    c = 1.0 + 0.3 * np.exp(-(xs[0] ** 2 + xs[1] ** 2) / 0.05)
    omega = 2 * np.pi * 4
    a = np.full(shape, 0.5 * omega)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    Qv = orc.Problem(shape, omega, c, a, m_real=2).exact_psdo(v)
    Ms = [3, 5, 9, 17, 33]
    err = [rel(orc.Problem(shape, omega, c, a, m_real=M).apply(v), Qv) for M in Ms]
    ratios = np.array(err[:-1]) / np.array(err[1:])
    assert np.all(ratios > 2.9) and np.all(ratios < 5.0), ratios
    slope = np.polyfit(np.log([1.0 / (M - 1) for M in Ms]), np.log(err), 1)[0]
    assert 1.7 < slope < 2.3, slope


def _d2q_paper(c, omega, a, xi2):
    """Second c-derivative of q_{-2} as printed in Section 4.3."""
    p = omega ** 2 + 1j * omega * a - c ** 2 * xi2
    return (2 * xi2 * p + 8 * c ** 2 * xi2 ** 2) / p ** 3


def _dq_paper(c, omega, a, xi2):
    p = omega ** 2 + 1j * omega * a - c ** 2 * xi2
    return 2 * c * xi2 / p ** 2


def _symbol_via_q1(orc, cval, omega, a, shape, k):
    """q(c, xi_k) read off the oracle's one-node preconditioner applied to a mode."""
    p = orc.Problem(shape, omega, np.full(shape, cval), np.full(shape, a), None, c0=cval, m_real=1)
    v = _mode(shape, k)
    return (p.apply(v) / v).mean()


def test_symbol_derivatives_match_paper(orc):
    shape, k = (16, 16), (2, 3)
    omega, a = 2 * np.pi * 3, 5.0
    xi2 = _xi2(shape, k)
    for c0 in (0.8, 1.0, 1.3):
        hh = 1e-4
        qm, q0, qp = (_symbol_via_q1(orc, c0 + s * hh, omega, a, shape, k) for s in (-1, 0, 1))
        d1 = (qp - qm) / (2 * hh)
        d2 = (qp - 2 * q0 + qm) / hh ** 2
        assert abs(d1 - _dq_paper(c0, omega, a, xi2)) < 1e-6 * abs(_dq_paper(c0, omega, a, xi2))
        assert abs(d2 - _d2q_paper(c0, omega, a, xi2)) < 1e-4 * abs(_d2q_paper(c0, omega, a, xi2))


def test_pointwise_lemma3_bound(orc):
    """|q - q_M| <= h_M^2/8 max|d^2 q/dc^2| on each interval (Lemma 3 with the explicit
    constant of linear interpolation), checked through single Fourier modes."""
    n = 16
    shape = (n, n)
    rng = np.random.default_rng(5)
    c = rng.uniform(0.8, 1.2, size=shape)
    c[0, 0], c[0, 1] = 0.8, 1.2
    omega, a = 2 * np.pi * 2, 6.0
    for M in (3, 6):
        p = orc.Problem(shape, omega, c, np.full(shape, a), None, m_real=M)
        nodes = p.setup()["cnode"]
        for k in [(1, 2), (3, 0), (4, 4)]:
            v = _mode(shape, k)
            qM = p.apply(v) / v
            xi2 = _xi2(shape, k)
            q = 1.0 / (omega ** 2 + 1j * omega * a - c ** 2 * xi2)
            cc = np.linspace(0.8, 1.2, 4001)
            bound = (nodes[1] - nodes[0]) ** 2 / 8 * np.abs(_d2q_paper(cc, omega, a, xi2)).max()
            assert np.abs(qM - q).max() <= bound * (1 + 1e-9) + 1e-15


# ---------------------------------------------------------------- Q_1 / homogeneous
def test_q1_inverts_stencil_with_discrete_symbol(orc):
    shape = (16, 16)
    c0 = 1.1
    omega = 2 * np.pi * 2.2
    p = orc.Problem(shape, omega, np.full(shape, c0), np.full(shape, 3.0), None, c0=c0, m_real=1,
                    symbol="discrete")
    rng = np.random.default_rng(9)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert rel(p.matvec(p.apply(v)), v) < 1e-12
    assert rel(p.apply(p.matvec(v)), v) < 1e-12


def test_error_paths(orc):
    shape = (8, 8)
    c = np.ones(shape)
    zeta = inputs.frame_layer(shape, 2, 0.1)
    c_bad = c.copy()
    c_bad[0, 3] = 1.05                                     # c != c_o inside the layer
    with pytest.raises(orc.OracleError) as e:
        orc.Problem(shape, 5.0, c_bad, None, zeta, m_real=3).apply(np.ones(shape))
    assert e.value.code == orc.E_LAYER
    c_nan = c.copy()
    c_nan[2, 2] = np.nan
    with pytest.raises(orc.OracleError) as e:
        orc.Problem(shape, 5.0, c_nan, m_real=3).apply(np.ones(shape))
    assert e.value.code == orc.E_MEDIA
    # a = 0 and no floor: omega = c |xi| exactly on the mode k = (1, 0) -> zero denominator
    with pytest.raises(orc.OracleError) as e:
        orc.Problem(shape, 2 * np.pi, c, None, None, m_real=1).apply(np.ones(shape))
    assert e.value.code == orc.E_MEDIA


def test_odd_lengths_rejected(orc):
    """Grid lengths must be even (the frequency range -N/2..N/2-1 of the transform)."""
    c = np.ones((15, 16))
    with pytest.raises(orc.OracleError):
        orc.Problem((15, 16), 10.0, c, None, None, m_real=2).setup()
    orc.Problem((18, 16), 10.0, np.ones((18, 16)), None, None, m_real=2, a_floor=1.0).setup()


# ---------------------------------------------------------------- higher-degree interpolation
@pytest.mark.parametrize("order", [2, 3])
def test_lagrange_weights_reproduce_polynomials(orc, order):
    """Degree-p piecewise Lagrange weights: node values are reproduced, every polynomial in
    Re gamma of degree <= p is reproduced exactly, the weights are continuous across the
    segment ends, and in the layer (Re gamma = c_o, a node) they equal the linear ones."""
    shape, c, zeta = _layer_medium()
    omega = 2 * np.pi * 4
    kw = dict(m_real=7, m_layer=3)
    p = orc.Problem(shape, omega, c, np.full(shape, 3.0), zeta, interp_order=order, **kw)
    lin = orc.Problem(shape, omega, c, np.full(shape, 3.0), zeta, **kw)
    st = p.setup()
    M, K, nodes = st["M"], st["K"], st["cnode"]
    for m, cn in enumerate(nodes):
        e = np.zeros(K)
        e[m] = 1
        assert np.abs(p.weights(cn, 0.0) - e).max() < 1e-14
    rng = np.random.default_rng(order)
    for cv in rng.uniform(st["cmin"], st["cmax"], 200):
        w = p.weights(cv, 0.0)[:M]
        assert np.count_nonzero(w) <= order + 1
        for deg in range(order + 1):
            assert abs(np.dot(w, nodes ** deg) - cv ** deg) < 1e-13 * max(1.0, cv ** deg), (deg, cv)
    for cn in nodes[1:-1]:
        d = np.abs(p.weights(cn - 1e-12, 0.0) - p.weights(cn + 1e-12, 0.0)).max()
        assert d < 1e-9, (cn, d)
    for zv in rng.uniform(0, st["zmax"], 20):
        assert np.abs(p.weights(1.0, zv) - lin.weights(1.0, zv)).max() < 1e-15


@pytest.mark.parametrize("order,lo,hi", [(2, 5.0, 11.0), (3, 10.0, 22.0)])
def test_lagrange_interpolation_error_rate(orc, order, lo, hi):
    """The interpolation error of Q_M against the exact operator Q falls by about 2^(p+1) per
    halving of the node spacing for degree-p pieces (Lemma 3's argument at higher degree)."""
    n = 32
    shape = (n, n)
    xs = inputs.mesh(shape)
    c = 1.0 + 0.3 * np.exp(-(xs[0] ** 2 + xs[1] ** 2) / 0.05)
    omega = 2 * np.pi * 4
    a = np.full(shape, 0.5 * omega)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    Qv = orc.Problem(shape, omega, c, a, m_real=2).exact_psdo(v)
    Ms = [5, 9, 17]
    err = [rel(orc.Problem(shape, omega, c, a, m_real=M, interp_order=order).apply(v), Qv) for M in Ms]
    ratios = np.array(err[:-1]) / np.array(err[1:])
    assert np.all(ratios > lo) and np.all(ratios < hi), (order, err, ratios)
