"""The C-ABI library: it loads, exports every entry point include/ngravs.h
declares, and the Python binding refuses to run without it (no fallback)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ngravs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ngr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("ngr_tree_build", "ngr_compute_monopoles", "ngr_tree_force", "ngr_tree_free",
              "ngr_context_create", "ngr_context_destroy", "ngr_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    import paper_1502_07442_amd as ngr
    if not os.path.exists(ngr.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(ngr.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(ngr.EXPORTED) == declared_functions()


def test_binding_fails_loudly_without_library(monkeypatch):
    import paper_1502_07442_amd as ngr
    monkeypatch.setattr(ngr, "_lib", None)
    monkeypatch.setattr(ngr, "LIB_PATH", "/nonexistent/libngravs.so")
    with pytest.raises(RuntimeError, match="missing"):
        ngr.lib()


def test_context_create_rejects_bad_device_without_gpu():
    import paper_1502_07442_amd as ngr
    if not os.path.exists(ngr.LIB_PATH):
        pytest.skip("library not built")
    out = ctypes.c_void_p()
    assert ngr.lib().ngr_context_create(-1, None, ctypes.byref(out)) == ngr.EINVAL
    assert ngr.lib().ngr_tree_build(None, None, None, None) == ngr.EINVAL
    assert ngr.lib().ngr_tree_free(None, None) == ngr.OK


def test_short_range_grid_host_rule():
    """ngr_short_range_grid is host arithmetic: its period covers r_cut +
    12.5 r_s + 37 range and its last k is past the Gaussian's 1e-17 point;
    bad arguments are rejected."""
    import math
    import paper_1502_07442_amd as ngr
    if not os.path.exists(ngr.LIB_PATH):
        pytest.skip("library not built")
    for r_s, r_cut, rng in ((0.01, 0.045, 0.0), (0.0012, 0.0055, 0.03), (1.0, 4.5, 2.0)):
        nk, dk = ngr.short_range_grid(r_s, r_cut, rng)
        assert 2 * math.pi / dk >= r_cut + 12.5 * r_s + 37 * rng - 1e-12 * r_cut
        assert math.exp(-((nk - 1) * dk * r_s) ** 2) < 1e-17
        assert math.exp(-((nk - 2) * dk * r_s) ** 2) >= 1e-17 or nk == 2
    for bad in ((0.0, 0.045, 0.0), (0.01, -1.0, 0.0), (0.01, 0.045, -1.0), (1e-9, 0.045, 1e3)):
        with pytest.raises(ngr.NgravsError):
            ngr.short_range_grid(*bad)
