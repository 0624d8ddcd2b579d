"""The C-ABI libraries load and export every function their headers declare
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_1504_07499_amd as rh
from paper_1504_07499_amd import _build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header):
    with open(os.path.join(ROOT, "include", header)) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)
    skip = {"if", "sizeof", "defined"}
    return sorted({n for n in names if n not in skip and not n.startswith("__")})


@pytest.mark.parametrize("header,lib", [("rvehom.h", _build.hip_lib_path()),
                                        ("rvegeom.h", _build.geom_lib_path())])
def test_exports(header, lib):
    if not os.path.exists(lib):
        pytest.skip(f"{lib} not built")
    so = ctypes.CDLL(lib)
    names = declared_functions(header)
    assert len(names) >= 4
    for n in names:
        assert hasattr(so, n), f"{n} declared in {header} but not exported"


def test_supported_sizes_and_host_validation():
    if not os.path.exists(_build.hip_lib_path()):
        pytest.skip("HIP library not built")
    assert 128 in rh.rve_supported_n(0) and 32 in rh.rve_supported_n(1)
    with pytest.raises(rh.RveError) as ei:
        rh.rve_create(33, 8, 0.2, 0.1, 1)  # unsupported grid size: rejected before any GPU call
    assert ei.value.status == rh.RVE_ERR_ARG
    with pytest.raises(rh.RveError):
        rh.rve_create(32, 1, 0.9, 0.1, 1)  # sphere radius >= 0.5
    with pytest.raises(rh.RveError):
        rh.rve_create(32, 8, 0.2, 1.2, 1)


def test_tune_table_roundtrip(tmp_path):
    """The autotuner's table as text: import, export, save and load (no GPU
    call: the table is host state)."""
    if not os.path.exists(_build.hip_lib_path()):
        pytest.skip("HIP library not built")
    rh.rve_tune_import("gfx950 0 96 ztile 1\n\ngfx942 1 128 ztile 0\ngfx950 0 64 plane 1\n")
    out = rh.rve_tune_export().splitlines()
    assert "gfx950 0 96 ztile 1" in out and "gfx942 1 128 ztile 0" in out and "gfx950 0 64 plane 1" in out
    # a plane choice and a z-tile choice of one grid are separate entries
    rh.rve_tune_import("gfx950 0 64 ztile 0")
    out = rh.rve_tune_export().splitlines()
    assert "gfx950 0 64 plane 1" in out and "gfx950 0 64 ztile 0" in out
    for bad in ("gfx950 0 96 ztile 2", "gfx950 2 96 ztile 0", "gfx950 0 96 wtile 0",
                "gfx950 0 96 ztile 0 extra", "gfx950 0 ztile 0", "gfx950 0 96 plane 3"):
        with pytest.raises(rh.RveError) as ei:
            rh.rve_tune_import(bad)
        assert ei.value.status == rh.RVE_ERR_ARG
    path = str(tmp_path / "tune.txt")
    with open(path, "w") as f:
        f.write("gfx950 1 64 ztile 0\n")
    rh.rve_tune_save(path)  # merged with what the file held
    with open(path) as f:
        saved = f.read().splitlines()
    assert "gfx950 1 64 ztile 0" in saved and "gfx950 0 96 ztile 1" in saved
    assert rh.rve_tune_load(path) and not rh.rve_tune_load(str(tmp_path / "absent.txt"))
