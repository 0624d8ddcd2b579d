"""Seeded input generator (RSA spheres or aligned fibres + voxelization),
ctypes binding.

Wraps ``librvegeom.so`` (``geom/rve_geom.cpp``, declared in
``include/rvegeom.h``).  Paper: arXiv:1504.07499, Sec. 2 (RSA of identical
spheres, sphere list, voxelization with a coating of relative width l) and the
radius/coating relations behind Table "tab0" and Tables 1-3 of Sec. 5.

This module holds no homogenization arithmetic; the same phase images feed
both the GPU library and the FP64 oracle.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _build

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.geom_lib_path()
    if not os.path.exists(path):
        _build.build_geom()
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.rvegeom_radius.argtypes = [ctypes.c_int, ctypes.c_double]
    lib.rvegeom_radius.restype = ctypes.c_double
    lib.rvegeom_place.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_uint64, dp, ip]
    lib.rvegeom_place.restype = ctypes.c_int
    lib.rvegeom_voxelize.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_double,
                                     ctypes.c_double, u8p]
    lib.rvegeom_voxelize.restype = ctypes.c_int
    lib.rvegeom_generate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_uint64, u8p, dp, ip]
    lib.rvegeom_generate.restype = ctypes.c_int
    lib.rvegeom_fiber_radius.argtypes = [ctypes.c_int, ctypes.c_double]
    lib.rvegeom_fiber_radius.restype = ctypes.c_double
    lib.rvegeom_place_fibers.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_uint64, dp, ip]
    lib.rvegeom_place_fibers.restype = ctypes.c_int
    lib.rvegeom_voxelize_fibers.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_double,
                                            ctypes.c_double, u8p]
    lib.rvegeom_voxelize_fibers.restype = ctypes.c_int
    lib.rvegeom_generate_fibers.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_uint64, u8p, dp, ip]
    lib.rvegeom_generate_fibers.restype = ctypes.c_int
    lib.rvegeom_place_mixed.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_uint64, dp, dp, ip]
    lib.rvegeom_place_mixed.restype = ctypes.c_int
    lib.rvegeom_generate_mixed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_uint64, u8p]
    lib.rvegeom_generate_mixed.restype = ctypes.c_int
    _lib = lib
    return lib


MATRIX, INCLUSION, COATING = 0, 1, 2


def radius(n_spheres: int, volume_fraction: float) -> float:
    """r = (3 f / (4 pi n))^(1/3), coating included (Sec. 2)."""
    return float(_load().rvegeom_radius(int(n_spheres), float(volume_fraction)))


def place(n_spheres: int, volume_fraction: float, seed: int):
    """RSA centres (n, 3) and the method used (0 RSA, 1 RSA + MC shaking)."""
    lib = _load()
    c = np.zeros((int(n_spheres), 3))
    m = ctypes.c_int(-1)
    rc = lib.rvegeom_place(int(n_spheres), float(volume_fraction), int(seed),
                           c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(m))
    if rc == -2:
        raise RuntimeError("sphere placement exhausted its attempt budget (jammed)")
    if rc != 0:
        raise ValueError("invalid sphere placement arguments")
    return c, int(m.value)


def voxelize(n: int, centers: np.ndarray, r: float, layer: float) -> np.ndarray:
    """Phase image (n, n, n) uint8, [z][y][x]: 0 matrix, 1 inclusion, 2 coating."""
    lib = _load()
    c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((n, n, n), dtype=np.uint8)
    rc = lib.rvegeom_voxelize(int(n), int(c.shape[0]),
                              c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              float(r), float(layer),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc != 0:
        raise ValueError("invalid voxelization arguments")
    return out


def generate(n: int, n_spheres: int, volume_fraction: float, layer: float, seed: int):
    """RSA + voxelization.  Returns (phases (n,n,n) uint8, centers (n_sp,3), method)."""
    lib = _load()
    out = np.zeros((n, n, n), dtype=np.uint8)
    c = np.zeros((int(n_spheres), 3))
    m = ctypes.c_int(-1)
    rc = lib.rvegeom_generate(int(n), int(n_spheres), float(volume_fraction), float(layer),
                              int(seed), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                              c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(m))
    if rc == -2:
        raise RuntimeError("sphere placement exhausted its attempt budget (jammed)")
    if rc != 0:
        raise ValueError("invalid geometry arguments")
    return out, c, int(m.value)


def fiber_radius(n_fibers: int, volume_fraction: float) -> float:
    """r = (f / (pi n))^(1/2), coating included: aligned fibres along z."""
    return float(_load().rvegeom_fiber_radius(int(n_fibers), float(volume_fraction)))


def place_fibers(n_fibers: int, volume_fraction: float, seed: int):
    """RSA fibre axes (n, 2) in the unit square and the method used."""
    lib = _load()
    c = np.zeros((int(n_fibers), 2))
    m = ctypes.c_int(-1)
    rc = lib.rvegeom_place_fibers(int(n_fibers), float(volume_fraction), int(seed),
                                  c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(m))
    if rc == -2:
        raise RuntimeError("fibre placement exhausted its attempt budget (jammed)")
    if rc != 0:
        raise ValueError("invalid fibre placement arguments")
    return c, int(m.value)


def voxelize_fibers(n: int, centers: np.ndarray, r: float, layer: float) -> np.ndarray:
    """Phase image (n, n, n) uint8 of coated fibres along z."""
    lib = _load()
    c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 2)
    out = np.zeros((n, n, n), dtype=np.uint8)
    rc = lib.rvegeom_voxelize_fibers(int(n), int(c.shape[0]),
                                     c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     float(r), float(layer),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc != 0:
        raise ValueError("invalid fibre voxelization arguments")
    return out


def generate_fibers(n: int, n_fibers: int, volume_fraction: float, layer: float, seed: int):
    """Aligned coated fibres along z: (phases (n,n,n) uint8, axes (n_f, 2), method)."""
    lib = _load()
    out = np.zeros((n, n, n), dtype=np.uint8)
    c = np.zeros((int(n_fibers), 2))
    m = ctypes.c_int(-1)
    rc = lib.rvegeom_generate_fibers(int(n), int(n_fibers), float(volume_fraction), float(layer),
                                     int(seed), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                     c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(m))
    if rc == -2:
        raise RuntimeError("fibre placement exhausted its attempt budget (jammed)")
    if rc != 0:
        raise ValueError("invalid fibre geometry arguments")
    return out, c, int(m.value)


def place_mixed(n_spheres: int, f_spheres: float, n_fibers: int, f_fibers: float, seed: int):
    """Fibre axes (n_f, 2) and sphere centres (n_s, 3) of a mixed cell."""
    lib = _load()
    cs = np.zeros((int(n_spheres), 3))
    cf = np.zeros((int(n_fibers), 2))
    m = ctypes.c_int(-1)
    rc = lib.rvegeom_place_mixed(int(n_spheres), float(f_spheres), int(n_fibers), float(f_fibers), int(seed),
                                 cs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 cf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(m))
    if rc == -2:
        raise RuntimeError("mixed placement exhausted its attempt budget (jammed)")
    if rc != 0:
        raise ValueError("invalid mixed placement arguments")
    return cs, cf


def generate_mixed(n: int, n_spheres: int, f_spheres: float, n_fibers: int, f_fibers: float,
                   layer: float, seed: int) -> np.ndarray:
    """Coated spheres and coated fibres along z in one cell: phases (n,n,n) uint8."""
    lib = _load()
    out = np.zeros((n, n, n), dtype=np.uint8)
    rc = lib.rvegeom_generate_mixed(int(n), int(n_spheres), float(f_spheres), int(n_fibers),
                                    float(f_fibers), float(layer), int(seed),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc == -2:
        raise RuntimeError("mixed placement exhausted its attempt budget (jammed)")
    if rc != 0:
        raise ValueError("invalid mixed geometry arguments")
    return out


def random_phases(n: int, seed: int, probs=(0.5, 0.3, 0.2)) -> np.ndarray:
    """Seeded i.i.d. phase image, for tests that need arbitrary microstructures."""
    rng = np.random.default_rng(seed)
    return rng.choice(3, size=(n, n, n), p=list(probs)).astype(np.uint8)
