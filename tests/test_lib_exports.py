"""The C-ABI library loads and exports every symbol include/rt.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "rt.h")).read()
    return sorted(set(re.findall(r"^(?:rt_status|void|const char\*)\s+(rt_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("rt_scene_create", "rt_scene_build", "rt_trace", "rt_scene_destroy", "rt_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    import paper_2511_08498_amd as rt
    if not os.path.exists(rt.LIB_PATH):
        pytest.skip("librt.so not built")
    L = ctypes.CDLL(rt.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing
    assert set(rt.EXPORTS) == set(declared_symbols())
    L.rt_version.restype = ctypes.c_char_p
    assert b"gfx950" in L.rt_version()


def test_binding_refuses_without_library(tmp_path, monkeypatch):
    import paper_2511_08498_amd as rt
    monkeypatch.setattr(rt, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(rt, "_LIB", None)
    with pytest.raises(RuntimeError):
        rt.lib()
