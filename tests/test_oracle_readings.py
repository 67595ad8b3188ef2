"""Pins of three set-up readings of the oracle, with the expected values written out
by hand in each test (not read back from the oracle's own set-up):

A6   real-node placement: two equidistant runs on [c_min, c_o] and [c_o, c_max]
     (Section 4.1 wants c_1 = c_min, c_M = c_max and equidistant nodes; Section 4.4
     wants c_o to be a node), with the split rounded half down, kept inside
     [1, M-2] and M raised to 3 when c_o is interior.
A11  symbol damping per node (Section 4 requires a = a(c)): a uniform a as is,
     otherwise the hat-weighted mean of a over the points each real node serves;
     layer nodes take the damping of c_o.
A12  the floor on the symbol damping where a = 0 (Section 3 assumes a_min > 0):
     only nodes of real speed are floored; layer nodes keep their damping.
"""
import numpy as np
import pytest

from paper_2409_16172_amd import inputs


def _framed(shape, width, interior, c0=1.0):
    """c = c0 on a frame of `width` cells (with zeta > 0 there), the given values inside."""
    e = inputs.boundary_distance_cells(shape)
    c = np.full(shape, c0)
    inner = e >= width
    vals = np.resize(np.asarray(interior, dtype=float), int(inner.sum()))
    c[inner] = vals
    zeta = np.where(e < width, 0.1 * (width - e) / width, 0.0)
    return c, zeta


# ---------------------------------------------------------------- A6
@pytest.mark.parametrize("cmin,c0,cmax,M,expect", [
    # interior c_o on the equidistant grid: split 2, both runs of 0.15
    (0.7, 1.0, 1.3, 5, [0.7, 0.85, 1.0, 1.15, 1.3]),
    # (c_o - c_min)/(c_max - c_min)(M - 1) = 1.5 exactly: the tie rounds down to 1
    (0.75, 1.0, 1.25, 4, [0.75, 1.0, 1.125, 1.25]),
    # M = 2 with an interior c_o is raised to 3
    (0.75, 1.0, 1.25, 2, [0.75, 1.0, 1.25]),
    # the split rounds to 0 and is kept at 1 so that both runs exist
    (0.99, 1.0, 1.5, 5, [0.99, 1.0, 1.0 + 0.5 / 3, 1.0 + 1.0 / 3, 1.5]),
    # ... and at the other end it rounds to M - 1 and is kept at M - 2
    (0.5, 1.0, 1.01, 5, [0.5, 0.5 + 0.5 / 3, 0.5 + 1.0 / 3, 1.0, 1.01]),
    # (0.3 / 0.8) * 7 = 2.625 rounds to 3: three intervals below c_o, four above
    (0.7, 1.0, 1.5, 8, [0.7, 0.8, 0.9, 1.0, 1.125, 1.25, 1.375, 1.5]),
])
def test_real_nodes_split_around_background(orc, cmin, c0, cmax, M, expect):
    shape = (16, 16)
    c, zeta = _framed(shape, 2, [cmin, cmax, c0, 0.5 * (cmin + cmax)], c0)
    st = orc.Problem(shape, 10.0, c, None, zeta, c0=c0, m_real=M, a_floor=1.0).setup()
    assert st["M"] == len(expect)
    assert np.abs(st["cnode"] - np.array(expect)).max() < 1e-15, st["cnode"]
    assert st["cnode"][st["mo"]] == c0


def test_real_nodes_with_background_at_an_end(orc):
    """c_o = c_min: no run below it (split 0), c_o is node 0; c_o = c_max: it is the last node."""
    shape = (16, 16)
    c, zeta = _framed(shape, 2, [1.0, 1.6, 1.3], 1.0)
    st = orc.Problem(shape, 10.0, c, None, zeta, m_real=4, a_floor=1.0).setup()
    assert np.abs(st["cnode"] - [1.0, 1.2, 1.4, 1.6]).max() < 1e-15 and st["mo"] == 0
    c, zeta = _framed(shape, 2, [0.4, 1.0, 0.7], 1.0)
    st = orc.Problem(shape, 10.0, c, None, zeta, m_real=4, a_floor=1.0).setup()
    assert np.abs(st["cnode"] - [0.4, 0.6, 0.8, 1.0]).max() < 1e-15 and st["mo"] == 3


def test_real_nodes_without_layer_are_equidistant(orc):
    shape = (8, 8)
    c = np.full(shape, 1.1)
    c[0, 0], c[3, 4] = 0.9, 1.5
    st = orc.Problem(shape, 10.0, c, None, None, m_real=4, a_floor=1.0).setup()
    assert np.abs(st["cnode"] - [0.9, 1.1, 1.3, 1.5]).max() < 1e-15


# ---------------------------------------------------------------- A11
def test_damping_mean_over_node_supports(orc):
    """4 x 4 grid, c on the nodes {1, 1.5, 2} and between them, a varying: each node's
    damping is sum_x w_m(x) a(x) / sum_x w_m(x) with the hat weights w_m."""
    c = np.array([[1.0, 1.25, 1.5, 1.75],
                  [2.0, 1.0, 1.125, 1.5],
                  [1.5, 1.5, 1.875, 2.0],
                  [1.0, 1.25, 1.75, 1.5]])
    a = np.array([[1.0, 2.0, 3.0, 4.0],
                  [5.0, 6.0, 7.0, 8.0],
                  [9.0, 10.0, 11.0, 12.0],
                  [13.0, 14.0, 15.0, 16.0]])
    # hat weights written out: a point between nodes m and m + 1 at fraction t gives
    # 1 - t to node m and t to node m + 1 (nodes 1.0, 1.5, 2.0)
    num = np.zeros(3)
    den = np.zeros(3)
    table = {1.0: {0: 1.0}, 1.125: {0: 0.75, 1: 0.25}, 1.25: {0: 0.5, 1: 0.5}, 1.5: {1: 1.0},
             1.75: {1: 0.5, 2: 0.5}, 1.875: {1: 0.25, 2: 0.75}, 2.0: {2: 1.0}}
    for cv, av in zip(c.ravel(), a.ravel()):
        for m, w in table[cv].items():
            num[m] += w * av
            den[m] += w
    expect = num / den
    # by hand: node 0 gets 1 (w 1), 6 (1), 13 (1), 2 (0.5), 14 (0.5), 7 (0.75)
    assert abs(expect[0] - (1 + 6 + 13 + 0.5 * 2 + 0.5 * 14 + 0.75 * 7) / 4.75) < 1e-15
    st = orc.Problem((4, 4), 10.0, c, a, None, m_real=3).setup()
    assert np.abs(st["cnode"] - [1.0, 1.5, 2.0]).max() == 0
    assert np.abs(st["ahat"] - expect).max() < 1e-14, (st["ahat"], expect)


def test_damping_mean_with_layer(orc):
    """With a layer, the points of the first layer segment (0 < zeta < zeta_1) give
    weight 1 - t to node c_o; points deeper in the layer give it none; every layer
    node takes the damping of c_o."""
    shape = (8, 8)
    e = inputs.boundary_distance_cells(shape)
    c = np.where(e >= 2, 1.5, 1.0)
    c[3, 3], c[4, 4] = 0.5, 1.5
    c[3, 4] = 1.0
    zeta = np.where(e == 0, 0.2, np.where(e == 1, 0.05, 0.0))
    a = np.arange(64, dtype=float).reshape(shape) + 1.0
    p = orc.Problem(shape, 10.0, c, a, zeta, m_real=3, m_layer=2)
    st = p.setup()
    # nodes: c_min 0.5, c_o 1.0, c_max 1.5 -> exactly the three real nodes; zeta nodes 0.1, 0.2
    assert np.abs(st["cnode"] - [0.5, 1.0, 1.5]).max() == 0
    assert np.abs(st["znode"] - [0.0, 0.1, 0.2]).max() < 1e-15
    num = np.zeros(3)
    den = np.zeros(3)
    for (i, j), cv in np.ndenumerate(c):
        z = zeta[i, j]
        if z > 0:
            if z < 0.1:                      # first layer segment, t = z / 0.1
                w = 1.0 - z / 0.1
                num[1] += w * a[i, j]
                den[1] += w
            continue
        m = {0.5: 0, 1.0: 1, 1.5: 2}[cv]
        num[m] += a[i, j]
        den[m] += 1.0
    expect = num / den
    K = st["K"]
    assert K == 5
    assert np.abs(st["ahat"][:3] - expect).max() < 1e-13, (st["ahat"], expect)
    assert np.all(st["ahat"][3:] == st["ahat"][1])


# ---------------------------------------------------------------- A12
def test_floor_applies_to_real_nodes_only(orc):
    """a = 0 with a floor F: every real node gets F, every layer node keeps 0."""
    shape = (16, 16)
    c, zeta = _framed(shape, 3, [0.8, 1.2, 1.05], 1.0)
    omega, F = 2 * np.pi * 3, 0.7
    p = orc.Problem(shape, omega, c, None, zeta, m_real=4, m_layer=3, a_floor=F)
    st = p.setup()
    M, K = st["M"], st["K"]
    assert (M, K) == (4, 7)
    assert np.all(st["ahat"][:M] == F) and np.all(st["ahat"][M:] == 0.0), st["ahat"]
    # and it is that damping the apply uses: one Fourier mode through the closed form,
    # with the symbol built here from the hand-set damping
    k = (2, -3)
    xs = inputs.mesh(shape)
    v = np.exp(1j * sum(2 * np.pi * kk * (x + 0.5) for kk, x in zip(k, xs)))
    xi2 = sum((2 * np.pi * kk) ** 2 for kk in k)
    ahat = np.array([F] * M + [0.0] * (K - M))
    qn = 1.0 / (omega ** 2 + 1j * omega * ahat - st["gamma"] ** 2 * xi2)
    ww = np.array([p.weights(cv, zv) for cv, zv in zip(c.ravel(), zeta.ravel())])
    expect = (ww @ qn).reshape(shape) * v
    assert np.abs(p.apply(v) - expect).max() < 1e-13 * np.abs(qn).max()


def test_floor_leaves_damped_nodes_and_layer_uses_background_damping(orc):
    """A uniform a above the floor is used as is everywhere; below it only the real
    nodes are raised, the layer nodes keep a."""
    shape = (16, 16)
    c, zeta = _framed(shape, 3, [0.8, 1.2, 1.05], 1.0)
    st = orc.Problem(shape, 10.0, c, np.full(shape, 2.0), zeta, m_real=4, a_floor=1.5).setup()
    assert np.all(st["ahat"] == 2.0)
    st = orc.Problem(shape, 10.0, c, np.full(shape, 0.5), zeta, m_real=4, a_floor=1.5).setup()
    assert np.all(st["ahat"][:4] == 1.5) and np.all(st["ahat"][4:] == 0.5)


def test_floor_in_the_tensor_schemes(orc):
    """Layer tensor: only the row Im gamma = 0 is floored.  Bivariate (c, a): every node
    has a real speed, so every damping node below the floor is raised."""
    shape = (16, 16)
    c, zeta = _framed(shape, 3, [0.8, 1.2, 1.05], 1.0)
    st = orc.Problem(shape, 10.0, c, None, zeta, m_real=3, m_layer=2, a_floor=0.9,
                     layer_tensor=True).setup()
    g = st["gamma"]
    assert st["K"] == 9
    assert np.all(st["ahat"][g.imag == 0] == 0.9) and np.all(st["ahat"][g.imag < 0] == 0.0)
    assert np.count_nonzero(g.imag == 0) == 3
    a = np.where(np.arange(256).reshape(shape) % 2 == 0, 0.2, 3.0)
    st = orc.Problem(shape, 10.0, c, a, None, m_real=3, m_damp=2, a_floor=0.9).setup()
    assert np.abs(st["ahat"] - [0.9, 0.9, 0.9, 3.0, 3.0, 3.0]).max() == 0


def test_layer_without_damping_has_no_symbol_zero(orc):
    """a = 0, no floor, with a layer: the layer nodes' denominators never vanish, so the
    failure is reported for the real nodes only (their zeros lie on the grid here)."""
    shape = (8, 8)
    c, zeta = _framed(shape, 2, [1.0], 1.0)
    # c = 1 everywhere: one real node, K = 1 + 2.  omega = 2 pi puts |xi| = omega on k = (1, 0)
    with pytest.raises(orc.OracleError) as e:
        orc.Problem(shape, 2 * np.pi, c, None, zeta, m_real=3, m_layer=2).apply(np.ones(shape))
    assert e.value.code == orc.E_MEDIA
    # off the grid's |xi| values the same plan is fine, and the layer nodes are undamped
    p = orc.Problem(shape, 2 * np.pi * 1.3, c, None, zeta, m_real=3, m_layer=2)
    st = p.setup()
    assert np.all(st["ahat"] == 0.0)
    p.apply(np.ones(shape))


def test_node_valued_media_with_floor_equal_exact_operator(orc):
    """a = 0 with a floor on media whose (c, zeta) take node values only: Q_M equals the
    exact operator of Eqn. Precond whose damping is floored where the speed is real
    (zeta = 0) and left at 0 in the layer -- a point-by-point brute force, independent
    of the node tables."""
    n = 16
    shape = (n, n)
    rng = np.random.default_rng(21)
    nodes = np.array([0.8, 0.9, 1.0, 1.15, 1.3])
    c = nodes[rng.integers(0, len(nodes), size=shape)]
    e = inputs.boundary_distance_cells(shape)
    znodes = np.array([0.05, 0.1, 0.2])
    zeta = np.where(e < 3, znodes[rng.integers(0, 3, size=shape)], 0.0)
    zeta[e == 0] = 0.2
    c[e < 3] = 1.0
    omega = 2 * np.pi * 2.5
    p = orc.Problem(shape, omega, c, None, zeta, nodes_real=nodes, nodes_zeta=znodes, a_floor=0.1 * omega)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    u, q = p.apply(v), p.exact_psdo(v)
    assert np.linalg.norm(u - q) / np.linalg.norm(q) < 1e-13
    # the layer points alone: with the floor wrongly applied there the operators differ
    pf = orc.Problem(shape, omega, c, np.zeros(shape), zeta, nodes_real=nodes, nodes_zeta=znodes,
                     a_floor=0.1 * omega)
    assert np.linalg.norm(pf.apply(v) - u) == 0.0
