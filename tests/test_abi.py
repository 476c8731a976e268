"""Host-side checks of the C ABI library (no GPU calls): it loads and exports
every function include/gp.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(gp_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("gp_sim_create", "gp_sim_step", "gp_sim_render", "gp_sim_step_render_graph",
              "gp_sim_destroy", "gp_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2606_19641_amd import gp
    if not os.path.exists(gp.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(gp.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(L, n)]
    assert not missing, missing
    assert set(gp.EXPORTS) <= _declared()


def test_last_error_is_callable_without_gpu():
    from paper_2606_19641_amd import gp
    if not os.path.exists(gp.LIB_PATH):
        pytest.skip("library not built")
    L = gp.lib()
    # a NULL config is rejected on the host before any device call
    assert L.gp_sim_required_bytes(None, None, 1) == -1
    assert b"cfg" in L.gp_last_error()
