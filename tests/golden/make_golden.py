"""Write the stored expected values under tests/golden/ from the CPU oracle.

The paper prints no worked example of the preconditioner apply or of a solve
(its tables are CPU timings and condition numbers of its own media), so the
stored values here are computed by the oracle alone, on small seeded inputs
from paper_2409_16172_amd.inputs, and each fixture names the passages that
define what it holds.  Run from the repository root:

    python tests/golden/make_golden.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2409_16172_amd import inputs  # noqa: E402


def cx(a):
    a = np.asarray(a).ravel()
    return [[float(v.real), float(v.imag)] for v in a]


def media(shape, seed, width):
    n = shape[0]
    c = inputs.gaussian_random_field(shape, max(2.0, n / 8), seed)
    c = inputs.blend_to_background(c, width, 1.0, taper=2)
    zeta = inputs.frame_layer(shape, width, 0.133)
    return c, zeta


def apply_fixture(name, shape, seed, width, n_lambda, m_real, symbol):
    c, zeta = media(shape, seed, width)
    omega = inputs.omega_for_wavelengths(n_lambda)
    a = np.full(shape, 0.05 * omega)
    p = oracle.Problem(shape, omega, c, a, zeta, m_real=m_real, m_layer=3, symbol=symbol, a_floor=0.05 * omega)
    st = p.setup()
    rng = np.random.default_rng(seed + 1)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    u = p.apply(v)
    return {
        "what": "u = Q_M v, the interpolated preconditioner with the absorbing layer",
        "cites": "Section 4.1 (Eqn. 105, 103), Section 4.4 (Eqn. Complex_wave_speed, 405, 403), Eqn. 021",
        "source": "tests/golden/make_golden.py, CPU FP64 oracle",
        "shape": list(shape), "length": 1.0, "omega": omega, "c0": 1.0, "m_real": m_real, "m_layer": 3,
        "symbol": symbol, "a_floor": 0.05 * omega,
        "c": c.ravel().tolist(), "a": a.ravel().tolist(), "zeta": zeta.ravel().tolist(),
        "K": st["K"], "cnode": st["cnode"].tolist(), "znode": st["znode"].tolist(),
        "ahat": st["ahat"].tolist(),
        "v": cx(v), "u": cx(u),
    }, name


def solve_fixture(name, shape, seed, width, n_lambda, m_real):
    c, zeta = media(shape, seed, width)
    omega = inputs.omega_for_wavelengths(n_lambda)
    a = np.full(shape, 0.05 * omega)
    p = oracle.Problem(shape, omega, c, a, zeta, m_real=m_real, m_layer=3, a_floor=0.05 * omega)
    f = inputs.gaussian_source(shape, 2.0, [0.1, -0.05][:len(shape)] + [0.0] * (len(shape) - 2))
    x, res = p.gmres(f, restart=30, rtol=1e-12)
    return {
        "what": "x with ||f - P_N x|| <= 1e-12 ||f||: right-preconditioned restarted GMRES(30) with Q_M",
        "cites": "Section 5 (Eqn. MainDiscrete, MainDiscretePrecond), Eqn. 003 with gamma (Section 4.4)",
        "source": "tests/golden/make_golden.py, CPU FP64 oracle",
        "shape": list(shape), "length": 1.0, "omega": omega, "c0": 1.0, "m_real": m_real, "m_layer": 3,
        "a_floor": 0.05 * omega,
        "c": c.ravel().tolist(), "a": a.ravel().tolist(), "zeta": zeta.ravel().tolist(),
        "f": cx(f), "x": cx(x), "rtol": 1e-12, "restart": 30,
        "iters": res["iters"], "cycles": res["cycles"], "rel_true_residual": res["rel_true_residual"],
    }, name


def main():
    oracle.build()
    fixtures = [
        apply_fixture("apply_2d_16x16.json", (16, 16), 7, 3, 3.0, 6, "continuous"),
        apply_fixture("apply_2d_16x32_discrete.json", (16, 32), 8, 3, 3.0, 5, "discrete"),
        apply_fixture("apply_3d_8x8x8.json", (8, 8, 8), 9, 2, 1.5, 4, "continuous"),
        solve_fixture("solve_2d_16x16.json", (16, 16), 10, 3, 2.0, 6),
    ]
    for data, name in fixtures:
        with open(os.path.join(HERE, name), "w") as fh:
            json.dump(data, fh, separators=(",", ":"))
            fh.write("\n")
        print(name, os.path.getsize(os.path.join(HERE, name)), "bytes")


if __name__ == "__main__":
    main()
