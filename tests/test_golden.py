"""Stored expected values (tests/golden/*.json, written by tests/golden/make_golden.py
from the CPU oracle alone; each fixture names the passages that define it).

CPU: the oracle still reproduces them (a change to the oracle's arithmetic shows up
here).  GPU: the HIP path, through the C ABI, reproduces the stored node tables,
applies and solution.
"""
import json
import os

import numpy as np
import pytest

from tests.util import rel

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
APPLY = ["apply_2d_16x16.json", "apply_2d_16x32_discrete.json", "apply_3d_8x8x8.json"]


def load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        d = json.load(fh)
    shape = tuple(d["shape"])
    out = dict(d)
    for k in ("c", "a", "zeta"):
        out[k] = np.array(d[k], dtype=np.float64).reshape(shape)
    for k in ("v", "u", "f", "x"):
        if k in d:
            arr = np.array(d[k], dtype=np.float64)
            out[k] = (arr[:, 0] + 1j * arr[:, 1]).reshape(shape)
    out["shape"] = shape
    return out


def oracle_problem(orc, g):
    return orc.Problem(g["shape"], g["omega"], g["c"], g["a"], g["zeta"], length=g["length"], c0=g["c0"],
                       m_real=g["m_real"], m_layer=g["m_layer"], symbol=g.get("symbol", "continuous"),
                       a_floor=g["a_floor"])


@pytest.mark.parametrize("name", APPLY)
def test_oracle_reproduces_golden_apply(orc, name):
    g = load(name)
    p = oracle_problem(orc, g)
    st = p.setup()
    assert st["K"] == g["K"]
    np.testing.assert_allclose(st["cnode"], g["cnode"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(st["znode"], g["znode"], rtol=0, atol=1e-15)
    assert rel(p.apply(g["v"]), g["u"]) <= 1e-14


def test_oracle_reproduces_golden_solve(orc):
    g = load("solve_2d_16x16.json")
    p = oracle_problem(orc, g)
    x, res = p.gmres(g["f"], restart=g["restart"], rtol=g["rtol"])
    assert (res["iters"], res["cycles"]) == (g["iters"], g["cycles"])
    assert rel(x, g["x"]) <= 1e-12
    assert rel(p.matvec(g["x"]), g["f"]) <= g["rtol"]


def _gpu_plan(g, precision="fp64"):
    from paper_2409_16172_amd import binding
    return binding.Plan(g["shape"], g["omega"], g["c"], g["a"], g["zeta"], length=g["length"], c0=g["c0"],
                        m_real=g["m_real"], m_layer=g["m_layer"], symbol=g.get("symbol", "continuous"),
                        a_floor=g["a_floor"], precision=precision)


@pytest.mark.gpu
@pytest.mark.parametrize("name", APPLY)
def test_gpu_reproduces_golden_apply(name):
    import torch
    g = load(name)
    print(f"[case] golden {name}", flush=True)
    plan = _gpu_plan(g)
    info = plan.info()
    assert info["K"] == g["K"]
    np.testing.assert_allclose(info["cnode"], g["cnode"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(info["znode"], g["znode"], rtol=0, atol=1e-15)
    u = plan.apply(torch.from_numpy(g["v"][None].copy()).to("cuda:0")).cpu().numpy()[0]
    assert rel(u, g["u"]) <= 1e-12
    plan32 = _gpu_plan(g, "mixed")
    u32 = plan32.apply(torch.from_numpy(g["v"][None].copy()).to("cuda:0").to(torch.complex64)).cpu().numpy()[0]
    assert rel(u32, g["u"]) <= 1e-5


@pytest.mark.gpu
def test_gpu_reproduces_golden_solve(orc):
    import torch
    g = load("solve_2d_16x16.json")
    print("[case] golden solve_2d_16x16", flush=True)
    plan = _gpu_plan(g)
    x, info = plan.solve(torch.from_numpy(g["f"][None].copy()).to("cuda:0"), rtol=g["rtol"], restart=g["restart"])
    xh = x.cpu().numpy()[0]
    assert info[0].status == 0
    assert rel(oracle_problem(orc, g).matvec(xh), g["f"]) <= g["rtol"] * 1.001
    assert rel(xh, g["x"]) <= 1e-8
