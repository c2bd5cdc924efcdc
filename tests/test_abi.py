"""The C-ABI library loads on the CPU and exports every entry point that
include/pot.h declares (no compute calls: there may be no GPU here)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pot.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\*?\s*(pot_[a-z_0-9]+)\s*\(", src, re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for required in ("pot_solve", "pot_solve_batched", "pot_workspace_bytes",
                     "pot_workspace_bytes_batched", "pot_status_string", "pot_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2601_17196_amd import pot
    if not os.path.exists(pot.lib_path()):
        pytest.skip("libpot.so not built (run __graft_entry__.build())")
    lib = ct.CDLL(pot.lib_path())
    for name in _declared():
        assert hasattr(lib, name), name


def test_host_only_calls():
    """Calls that touch no device: status strings, version, workspace sizing."""
    from paper_2601_17196_amd import pot
    if not os.path.exists(pot.lib_path()):
        pytest.skip("libpot.so not built")
    lib = pot.load()
    assert pot.status_string(0) == "ok"
    assert "invalid" in pot.status_string(1)
    assert lib.pot_version().decode().startswith("libpot")
    p = pot.Problem()
    p.n, p.m, p.kind, p.ldc = 4096, 4096, pot.COST_F32, 4096
    o = pot.make_options(1e-2)
    nb = pot.workspace_bytes(p, o)
    assert nb > 12 * 8 * 4096 * 2
    assert nb % 256 == 0
    p.n = 0
    assert pot.workspace_bytes(p, o) == 0
