"""Pins of the oracle's stencil P_N and restarted GMRES.

T7  constant coefficients: P_N exp(i xi.x) = (omega^2 + i omega a - gamma^2 lambda_h(k)) exp(i xi.x),
    the discrete analogue of the symbol of Eqn. 005; general media: the loops agree with an
    independent shifted-array form of the same centred differences (Section 5).
T8  on 16^2 grids GMRES to rtol 1e-13 agrees with a dense LU solve of P_N to 1e-10;
    check (b): constant media and the stencil's own symbol -> one iteration.
T9  Arnoldi invariants: A V_m = V_{m+1} H_m, V^H V = I; the residual GMRES reports is the
    true residual f - P_N x.
"""
import numpy as np
import pytest

from paper_2409_16172_amd import inputs
from tests.util import rel


def _roll_stencil(u, c, zeta, a, omega, length=1.0):
    g2 = (c * (1 - 1j * zeta)) ** 2
    lap = np.zeros_like(u)
    for ax in range(u.ndim):
        h = length / u.shape[ax]
        lap += (np.roll(u, -1, ax) - 2 * u + np.roll(u, 1, ax)) / h ** 2
    return g2 * lap + (omega ** 2 + 1j * omega * a) * u


def _media(n, seed=0, dim=2, width=3):
    shape = (n,) * dim
    c = inputs.gaussian_random_field(shape, 3.0, seed)
    c = inputs.blend_to_background(c, width, 1.0, taper=3)
    zeta = inputs.frame_layer(shape, width, 0.2)
    return shape, c, zeta


@pytest.mark.parametrize("dim", [2, 3])
def test_stencil_plane_wave_eigenrelation(orc, dim):
    n = 16 if dim == 2 else 8
    shape = (n,) * dim
    gam = 1.2 * (1 - 0.1j)
    omega, a = 7.0, 2.5
    # constant complex speed via c and zeta constant (no layer check in matvec)
    c = np.full(shape, 1.2)
    zeta = np.full(shape, 0.1)
    p = orc.Problem(shape, omega, c, np.full(shape, a), zeta, c0=1.2, m_real=1)
    k = (3, -2, 1)[:dim]
    xs = inputs.mesh(shape)
    v = np.exp(1j * sum(2 * np.pi * kk * (x + 0.5) for kk, x in zip(k, xs)))
    lam_h = sum(4 * n ** 2 * np.sin(np.pi * kk / n) ** 2 for kk in k)
    expect = (omega ** 2 + 1j * omega * a - gam ** 2 * lam_h) * v
    assert rel(p.matvec(v), expect) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_stencil_matches_shifted_arrays(orc, dim):
    shape, c, zeta = _media(16 if dim == 2 else 8, dim=dim, width=2)
    rng = np.random.default_rng(1)
    a = rng.uniform(0, 3, size=shape)
    u = rng.standard_normal((2,) + shape) + 1j * rng.standard_normal((2,) + shape)
    p = orc.Problem(shape, 9.0, c, a, zeta, m_real=4)
    y = p.matvec(u)
    for r in range(2):
        assert rel(y[r], _roll_stencil(u[r], c, zeta, a, 9.0)) < 1e-14


def _dense(p, shape):
    npt = int(np.prod(shape))
    A = np.zeros((npt, npt), complex)
    for j in range(npt):
        e = np.zeros(npt, complex)
        e[j] = 1
        A[:, j] = p.matvec(e.reshape(shape)).ravel()
    return A


@pytest.mark.parametrize("side", ["right", "left"])
def test_gmres_matches_dense_lu_16(orc, side):
    shape, c, zeta = _media(16)
    omega = 2 * np.pi * 2.0
    a = np.full(shape, 0.05 * omega)
    p = orc.Problem(shape, omega, c, a, zeta, m_real=4, a_floor=0.05 * omega)
    f = inputs.gaussian_source(shape, 2.0, (0.05, -0.1))
    x, info = p.gmres(f, rtol=1e-13, restart=30, side=side)
    # left: GMRES on Q P x = Q f stops on that system's residual (Eqn. MainDiscretePrecond)
    assert info["status"] == 0 and info["rel_prec_residual"] <= 1e-13
    assert info["rel_true_residual"] <= (1e-13 if side == "right" else 1e-11)
    xd = np.linalg.solve(_dense(p, shape), f.ravel()).reshape(shape)
    assert rel(x, xd) < 1e-10


def test_check_b_one_iteration_constant_media(orc):
    shape = (32, 32)
    omega = 2 * np.pi * 5
    p = orc.Problem(shape, omega, np.ones(shape), np.full(shape, 4.0), None, m_real=8,
                    symbol="discrete")
    f = inputs.gaussian_source(shape, 2.0, (0.1, 0.2))
    x, info = p.gmres(f, rtol=1e-8)
    assert info["iters"] == 1 and info["rel_true_residual"] < 1e-12


def test_arnoldi_invariants(orc):
    shape, c, zeta = _media(16, seed=4)
    omega = 2 * np.pi * 2.0
    p = orc.Problem(shape, omega, c, np.full(shape, 0.1 * omega), zeta, m_real=5,
                    a_floor=0.05 * omega)
    rng = np.random.default_rng(2)
    v0 = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    m = 12
    V, H, steps = p.arnoldi(v0, m, side="right")
    assert steps == m
    Vm = V.reshape(m + 1, -1).T
    AV = np.stack([p.matvec(p.apply(V[j])).ravel() for j in range(m)], axis=1)
    assert np.linalg.norm(AV - Vm @ H) < 1e-12 * np.linalg.norm(AV)
    assert np.abs(Vm.conj().T @ Vm - np.eye(m + 1)).max() < 1e-12


def test_reported_residual_is_true_residual(orc):
    shape, c, zeta = _media(32, seed=7)
    omega = 2 * np.pi * 4
    p = orc.Problem(shape, omega, c, np.full(shape, 0.05 * omega), zeta, m_real=6,
                    a_floor=0.05 * omega)
    f = inputs.gaussian_source(shape, 2.0, (0.0, 0.1))
    x, info = p.gmres(f, rtol=1e-9, restart=10)
    r = np.linalg.norm(f - p.matvec(x)) / np.linalg.norm(f)
    assert abs(r - info["rel_true_residual"]) < 1e-14 and r <= 1e-9
    # preconditioning helps: without it the same budget leaves a far larger residual
    _, info0 = p.gmres(f, rtol=1e-9, restart=10, side="none", max_cycles=info["cycles"])
    assert info0["rel_true_residual"] > 1e3 * info["rel_true_residual"]


def test_not_converged_status_and_resume(orc):
    shape, c, zeta = _media(32, seed=8)
    omega = 2 * np.pi * 4
    p = orc.Problem(shape, omega, c, np.full(shape, 0.05 * omega), zeta, m_real=6,
                    a_floor=0.05 * omega)
    f = inputs.gaussian_source(shape, 2.0, (0.0, 0.1))
    x1, info1 = p.gmres(f, rtol=1e-30, restart=5, max_cycles=1)
    assert info1["status"] == 8
    x2, info2 = p.gmres(f, x0=x1, rtol=1e-9, restart=30)
    assert info2["status"] == 0 and info2["rel_true_residual"] <= 1e-9
