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


def test_bad_obstacles_and_lights_are_rejected_on_the_host():
    """Input checks run before any device call (gp_sim_required_bytes)."""
    import numpy as np
    from paper_2606_19641_amd import gp, scenegen as g
    if not os.path.exists(gp.LIB_PATH):
        pytest.skip("library not built")
    cam, pal = g.camera_for(32), g.default_palette()
    sc = g.make_scene(0x5EED0002, 1, 6, 120, n_static=40, n_signals=30)
    base = gp.required_bytes([sc], cam, pal)
    plain = gp.required_bytes([g.make_scene(0x5EED0002, 1, 6, 120)], cam, pal)
    assert base > plain                          # obstacles and lights take workspace
    for field, idx, bad in (("static_xyp", (1, 0), np.inf), ("static_dims", (2, 1), np.nan),
                            ("signal_xyzr", (0, 3), 0.0), ("signal_xyzr", (1, 3), -0.2),
                            ("signal_xyzr", (2, 1), np.nan)):
        b = g.make_scene(0x5EED0002, 1, 6, 120, n_static=4, n_signals=3)
        getattr(b, field)[idx] = bad
        with pytest.raises(gp.GpError):
            gp.required_bytes([b], cam, pal)
    b = g.make_scene(0x5EED0002, 1, 6, 120, n_static=4)
    b.static_color = b.static_color[:2]          # shapes disagree: refused by the binding
    with pytest.raises(ValueError):
        gp.required_bytes([b], cam, pal)
