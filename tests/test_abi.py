"""The C ABI library loads and exports every entry point include/tetvol.h
declares; argument errors are reported without touching a GPU (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "tetvol.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_parses():
    names = declared_functions()
    for n in ["leb_build", "tet_render", "tet_grid_export", "tet_locate", "dda_render", "tet_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2506_11510_amd import _abi
    L = _abi.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert name in _abi.SIGNATURES, f"binding lacks {name}"
    # the shared object really exports them (dynamic symbol table)
    out = os.popen(f"nm -D --defined-only {_abi.SO_PATH}").read()
    for name in declared_functions():
        assert re.search(rf"\bT {name}$", out, flags=re.M), name


def test_defaults_and_argument_errors_without_gpu():
    from paper_2506_11510_amd import _abi
    L = _abi.lib()
    o = _abi.TetBuildOpts()
    L.tet_build_opts_defaults(ctypes.byref(o))
    assert o.max_tets > 0 and o.max_depth == 24
    r = _abi.TetRenderOpts()
    L.tet_render_opts_defaults(ctypes.byref(r))
    assert r.max_bounces >= 1 and r.max_steps_per_path > 0
    cam = _abi.make_camera(dict(pos=[0, 0, -1], look_at=[0, 0, 0], up=[0, 1, 0], fov_y_deg=40, width=8, height=8))
    # NULL output handle, NULL density, bad n: rejected before any device call
    assert L.leb_build(None, ctypes.byref(cam), 1.0, None, None, None) == _abi.TET_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert L.leb_build(None, ctypes.byref(cam), 1.0, None, None, ctypes.byref(h)) == _abi.TET_ERR_INVALID_ARG
    assert h.value is None
    assert b"density" in L.tet_last_error()
    d = _abi.TetDensity(ctypes.c_void_p(1), 6, 1, 1.0)
    assert L.leb_build(ctypes.byref(d), ctypes.byref(cam), 1.0, None, None, ctypes.byref(h)) == _abi.TET_ERR_INVALID_ARG
    bad = _abi.make_camera(dict(pos=[0, 0, 0], look_at=[0, 0, 0], up=[0, 1, 0], fov_y_deg=40, width=8, height=8))
    d = _abi.TetDensity(ctypes.c_void_p(1), 8, 1, 1.0)
    assert L.leb_build(ctypes.byref(d), ctypes.byref(bad), 1.0, None, None, ctypes.byref(h)) == _abi.TET_ERR_INVALID_ARG
    n = ctypes.c_int64()
    assert L.tet_grid_info(None, ctypes.byref(n), None, None) == _abi.TET_ERR_INVALID_ARG
    assert L.tet_render(None, ctypes.byref(cam), None, None, 1, 0, None, None, 1, None, None) != 0
    L.tet_grid_free(None)


def test_batch_and_cache_argument_errors_without_gpu():
    from paper_2506_11510_amd import _abi
    L = _abi.lib()
    h = ctypes.c_void_p()
    assert L.tet_render_batch(0, None, None, None, None, None, None, None, None, None, None) == _abi.TET_ERR_INVALID_ARG
    assert L.tet_batch_create(0, None, None, None, None, None, None, None, ctypes.byref(h)) == _abi.TET_ERR_INVALID_ARG
    assert h.value is None
    assert L.tet_batch_render(None, None, None, None) == _abi.TET_ERR_INVALID_ARG
    L.tet_batch_free(None)
    o = _abi.TetNrcOpts()
    L.tet_nrc_opts_defaults(ctypes.byref(o))
    assert (o.truncate_bounce, o.train_paths, o.train_vertices, o.train_steps) == (2, 16384, 4, 4)
    assert o.lr == pytest.approx(1e-3) and o.beta2 == pytest.approx(0.99) and o.ema == pytest.approx(0.95)
    o.train_vertices = 17
    assert L.tet_nrc_create(ctypes.byref(o), ctypes.byref(h)) == _abi.TET_ERR_INVALID_ARG and h.value is None
    assert L.tet_nrc_info(None, None, None) == _abi.TET_ERR_INVALID_ARG
    assert L.tet_nrc_export(None, None, 0, None) == _abi.TET_ERR_INVALID_ARG
    L.tet_nrc_free(None)


def test_product_never_imports_the_oracle():
    """The product package must not reach the oracle in any way."""
    pkg = os.path.join(ROOT, "paper_2506_11510_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "liboracle" not in txt, f
                assert "oracle.h" not in txt, f
