"""CPU-side checks of the C ABI: the library loads and exports every entry point
that include/helmpre.h declares (no GPU calls), and the host-only size queries."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "helmpre.h")).read()
    return sorted(set(re.findall(r"\b(hp_[a-z_]+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    names = _declared()
    for n in ("hp_plan_create", "hp_apply_precond", "hp_matvec", "hp_solve", "hp_plan_destroy"):
        assert n in names


def test_library_exports_all_declared_symbols():
    from paper_2409_16172_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libhelmpre.so not built")
    lib = binding.load_library()
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(binding.EXPORTED) == set(_declared())


def test_status_strings_and_workspace_queries():
    from paper_2409_16172_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libhelmpre.so not built")
    lib = binding.load_library()
    assert lib.hp_status_str(0) == b"ok"
    assert b"layer" in lib.hp_status_str(4)
    g = binding.HpGrid()
    g.dim = 2
    g.n[0], g.n[1] = 1024, 1024
    o = binding.HpPlanOpts()
    o.precision = 0
    o.max_nrhs = 1
    K = 19
    # t + K node fields (complex128) + per-point records and stencil coefficients
    assert lib.hp_plan_workspace_bytes(g, o, K) == (K + 1) * 1024 * 1024 * 16 + 1024 * 1024 * 40
    assert lib.hp_solve_workspace_bytes(g, 30, 2) > 2 * 33 * 1024 * 1024 * 16
