"""Seeded synthetic inputs (media, absorbing layer, sources) shared by the tests,
the oracle checks and the benchmark.

This module holds no arithmetic of the preconditioner, the stencil or the
solver: it only draws and shapes input fields.  Both the HIP path and the CPU
oracle consume the arrays it returns.

Conventions (Section 5 of the paper, Example 1): the domain is a square/cube of
side L centred at the origin with periodic boundary conditions, discretised by
N points per axis at x_i = -L/2 + i*h, h = L/N.  Arrays are row-major with the
last axis contiguous.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_BASE = 20240916


def axis_coords(n: int, length: float = 1.0) -> np.ndarray:
    h = length / n
    return -0.5 * length + h * np.arange(n, dtype=np.float64)


def mesh(shape, length: float = 1.0):
    axes = [axis_coords(n, length) for n in shape]
    return np.meshgrid(*axes, indexing="ij")


def boundary_distance_cells(shape) -> np.ndarray:
    """e(x) = min over axes of the number of cells to the nearest domain edge."""
    e = None
    for ax, n in enumerate(shape):
        i = np.arange(n)
        d = np.minimum(i, n - 1 - i)
        sh = [1] * len(shape)
        sh[ax] = n
        d = d.reshape(sh)
        e = d if e is None else np.minimum(e, d)
    return np.broadcast_to(e, shape).astype(np.int64)


def frame_layer(shape, width: int, zeta_max: float = 0.133) -> np.ndarray:
    """Absorbing-layer profile zeta(x) >= 0 on a rectangular frame of `width`
    cells, rising linearly towards the edge (the linear ramp of the radial
    profile of Example 2, placed on a frame so that it fits any box)."""
    if width <= 0:
        return np.zeros(shape, dtype=np.float64)
    e = boundary_distance_cells(shape)
    z = np.where(e < width, zeta_max * (width - e) / width, 0.0)
    return z.astype(np.float64)


def blend_to_background(c: np.ndarray, width: int, c0: float = 1.0, taper: int = 8) -> np.ndarray:
    """Force c = c0 inside the layer (the layer assumption of Section 4.4) and
    blend smoothly back to c over `taper` cells just inside the layer's inner
    edge with a cosine ramp."""
    if width <= 0:
        return c.copy()
    e = boundary_distance_cells(c.shape).astype(np.float64)
    s = np.clip((e - width) / float(taper), 0.0, 1.0)
    ramp = 0.5 - 0.5 * np.cos(np.pi * s)
    out = c0 + (c - c0) * ramp
    out[e < width] = c0
    return out


def gaussian_random_field(shape, corr_cells: float, seed: int, lo: float = 0.8, hi: float = 1.2,
                          length: float = 1.0) -> np.ndarray:
    """White N(0,1) noise filtered by exp(-l^2 |xi|^2 / 2) (periodic, l = corr_cells*h),
    real part, then min-max mapped to [lo, hi]."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape)
    spec = np.fft.fftn(noise)
    ell = corr_cells * length / shape[0]
    xi2 = None
    for ax, n in enumerate(shape):
        k = np.fft.fftfreq(n, d=1.0 / n)
        xi = 2.0 * np.pi * k / length
        sh = [1] * len(shape)
        sh[ax] = n
        term = (xi ** 2).reshape(sh)
        xi2 = term if xi2 is None else xi2 + term
    g = np.real(np.fft.ifftn(spec * np.exp(-0.5 * ell * ell * xi2)))
    g = (g - g.min()) / (g.max() - g.min())
    return lo + (hi - lo) * g


def smooth_heaviside(s, eta):
    """H_eta(s) = 1/(1+exp(-s/eta)) (Example 1, the smoothed inclusion)."""
    return 0.5 * (1.0 + np.tanh(0.5 * np.asarray(s) / eta))


def periodic_sqdist(shape, centre, length: float = 1.0) -> np.ndarray:
    xs = mesh(shape, length)
    d2 = np.zeros(shape)
    for ax in range(len(shape)):
        d = xs[ax] - centre[ax]
        d = d - length * np.round(d / length)
        d2 = d2 + d * d
    return d2


def gaussian_source(shape, sigma_cells: float, centre, length: float = 1.0) -> np.ndarray:
    """Real Gaussian source exp(-|x - x_s|^2 / (2 sigma^2)), sigma = sigma_cells*h,
    with periodic distance."""
    h = length / shape[0]
    sig = sigma_cells * h
    return np.exp(-periodic_sqdist(shape, centre, length) / (2.0 * sig * sig)).astype(np.complex128)


def random_source_centres(shape, count: int, width: int, sigma_cells: float, seed: int,
                          length: float = 1.0):
    """Source positions drawn uniformly at least width + 3 sigma cells from the edge."""
    rng = np.random.default_rng(seed)
    n = shape[0]
    h = length / n
    margin = (width + 3.0 * sigma_cells) * h
    lo = -0.5 * length + margin
    hi = 0.5 * length - margin
    return [tuple(rng.uniform(lo, hi, size=len(shape))) for _ in range(count)]


def omega_for_wavelengths(n_lambda: float, c0: float = 1.0, length: float = 1.0) -> float:
    """omega giving n_lambda background wavelengths across the domain
    (points per wavelength = 2 pi c0 N / (L omega), Example 1)."""
    return 2.0 * math.pi * n_lambda * c0 / length


@dataclass
class Workload:
    name: str
    shape: tuple
    length: float
    omega: float
    c: np.ndarray
    a: np.ndarray
    zeta: np.ndarray
    f: np.ndarray             # [nrhs, *shape] complex128
    m_real: int
    m_layer: int
    c0: float = 1.0
    a_floor: float = 0.0
    precision: str = "fp64"
    restart: int = 30
    rtol: float = 1e-8
    info: dict = field(default_factory=dict)

    @property
    def dim(self):
        return len(self.shape)

    @property
    def npts(self):
        return int(np.prod(self.shape))


def _bump_2d(n: int, seed: int) -> Workload:
    shape = (n, n)
    omega = omega_for_wavelengths(n / 8.0)
    xs = mesh(shape)
    c = 1.0 + 0.3 * np.exp(-(xs[0] ** 2 + xs[1] ** 2) / 0.02)
    width = 8 if n >= 64 else max(2, n // 8)
    c = blend_to_background(c, width, 1.0, taper=min(8, n // 8))
    zeta = frame_layer(shape, width)
    a = np.zeros(shape)
    ctr = random_source_centres(shape, 1, width, 2.0, seed)[0]
    f = gaussian_source(shape, 2.0, ctr)[None]
    return Workload(f"2d_{n}_bump", shape, 1.0, omega, c, a, zeta, f, 8, 3,
                    a_floor=0.05 * omega, info={"seed": seed, "source": ctr, "layer_cells": width})


def _grf_2d(n: int, n_lambda: float, m_real: int, precision: str, seed: int,
            width: Optional[int] = None, nrhs: int = 1) -> Workload:
    shape = (n, n)
    omega = omega_for_wavelengths(n_lambda)
    width = 32 if width is None else width
    c = gaussian_random_field(shape, 20.0, seed)
    c = blend_to_background(c, width, 1.0)
    zeta = frame_layer(shape, width)
    a = np.full(shape, 0.05 * omega)
    ctrs = random_source_centres(shape, nrhs, width, 2.0, seed + 1)
    f = np.stack([gaussian_source(shape, 2.0, ct) for ct in ctrs])
    return Workload(f"2d_{n}_grf", shape, 1.0, omega, c, a, zeta, f, m_real, 3,
                    a_floor=0.05 * omega, precision=precision,
                    info={"seed": seed, "n_lambda": n_lambda, "layer_cells": width})


def _grf_3d(n: int, n_lambda: float, nrhs: int, seed: int, width: int = 24) -> Workload:
    shape = (n, n, n)
    omega = omega_for_wavelengths(n_lambda)
    c = gaussian_random_field(shape, 12.0 * n / 256.0, seed)
    r2 = periodic_sqdist(shape, (0.0, 0.0, 0.0))
    h = 1.0 / n
    c = c + (1.4 - c) * smooth_heaviside(0.1 - np.sqrt(r2), h)
    c = blend_to_background(c, width, 1.0)
    zeta = frame_layer(shape, width)
    a = np.full(shape, 0.05 * omega)
    ctrs = random_source_centres(shape, nrhs, width, 2.0, seed + 1)
    f = np.stack([gaussian_source(shape, 2.0, ct) for ct in ctrs])
    return Workload(f"3d_{n}_grf_sphere", shape, 1.0, omega, c, a, zeta, f, 16, 3,
                    a_floor=0.05 * omega, precision="mixed",
                    info={"seed": seed, "n_lambda": n_lambda, "layer_cells": width, "nrhs": nrhs})


def _inclusion_2d(n: int, ppw: float, delta: float, eta: float, a: float, m_real: int, precision: str,
                  restart: int) -> Workload:
    """Example 1 (Section 5.1): periodic unit square, background c_o = 1, a circular
    inclusion of radius 0.05 at the centre with c = c_o + delta H_eta(0.05 - r)
    (Eqn. WS), constant damping a, plane-wave source exp(i omega x_1 / c_o)
    (Eqn. Source), omega from the points per wavelength PPW = 2 pi c_o N / (L omega).
    No absorbing layer."""
    shape = (n, n)
    omega = 2.0 * math.pi * n / ppw
    xs = mesh(shape)
    r = np.sqrt(xs[0] ** 2 + xs[1] ** 2)
    c = 1.0 + delta * smooth_heaviside(0.05 - r, eta)
    f = np.exp(1j * omega * xs[0])[None]
    return Workload(f"2d_{n}_inclusion", shape, 1.0, omega, c, np.full(shape, float(a)), None, f, m_real, 0,
                    precision=precision, restart=restart,
                    info={"ppw": ppw, "delta": delta, "eta": eta, "a": a, "n_lambda": n / ppw})


def workload(name: str, **kw) -> Workload:
    """Named synthetic workloads.

    2d_64_bump        64^2, 8 wavelengths, Gaussian bump c = 1 + 0.3 exp(-|x|^2/0.02), a = 0,
                      8-cell layer, 8 + 3 nodes, FP64.
    2d_1024_grf       1024^2, 100 wavelengths, Gaussian random field in [0.8,1.2]
                      (correlation 20 cells), a = 0.05 omega, 32-cell layer, 16 + 3 nodes, FP64.
    2d_2048_grf       2048^2, 200 wavelengths, same recipe, 24 + 3 nodes, mixed precision.
    3d_256_grf        256^3, 25 wavelengths, 3-D random field (12 cells) plus a c = 1.4 sphere,
                      24-cell layer, 16 + 3 nodes, 16 right-hand sides, mixed precision.
    2d_inclusion      Example 1 of the paper: N^2 (default 2400^2 = 200 wavelengths at 12 points
                      per wavelength), circular inclusion with contrast delta = 1 and smoothness
                      eta = 1/800, a = 20, plane-wave source, 8 nodes, no layer, GMRES(10), FP64.
                      Overrides: n, ppw, delta, eta, a, m_real, precision, restart.
    Smaller variants take keyword overrides (n=..., n_lambda=..., nrhs=...).
    """
    if name == "2d_inclusion":
        return _inclusion_2d(kw.get("n", 2400), kw.get("ppw", 12.0), kw.get("delta", 1.0), kw.get("eta", 1.0 / 800),
                             kw.get("a", 20.0), kw.get("m_real", 8), kw.get("precision", "fp64"),
                             kw.get("restart", 10))
    idx = {"2d_64_bump": 0, "2d_1024_grf": 1, "2d_2048_grf": 2, "3d_256_grf": 3}
    if name not in idx:
        raise KeyError(name)
    seed = kw.pop("seed", SEED_BASE + idx[name])
    if name == "2d_64_bump":
        return _bump_2d(kw.get("n", 64), seed)
    if name == "2d_1024_grf":
        n = kw.get("n", 1024)
        return _grf_2d(n, kw.get("n_lambda", 100.0 * n / 1024), kw.get("m_real", 16),
                       kw.get("precision", "fp64"), seed, kw.get("width", max(8, 32 * n // 1024)),
                       kw.get("nrhs", 1))
    if name == "2d_2048_grf":
        n = kw.get("n", 2048)
        return _grf_2d(n, kw.get("n_lambda", 200.0 * n / 2048), kw.get("m_real", 24),
                       kw.get("precision", "mixed"), seed, kw.get("width", max(8, 32 * n // 2048)),
                       kw.get("nrhs", 1))
    n = kw.get("n", 256)
    return _grf_3d(n, kw.get("n_lambda", 25.0 * n / 256), kw.get("nrhs", 16), seed,
                   kw.get("width", max(4, 24 * n // 256)))
