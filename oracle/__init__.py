"""FP64 CPU oracle for the accelerated FFT homogenization scheme.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (``paper_1504_07499_amd``) never imports it, and this package imports
nothing from the product path.

The numerics live in ``em_oracle.c`` (plain C99, own mixed-radix FFT,
OpenMP over pencils).  This module only marshals numpy arrays through ctypes.
Paper: arXiv:1504.07499, Sec. 3 (eq. (1), eq. (3), the Green operator, the
Algorithm of the accelerated scheme, L_hom from <phi>) and Sec. 5 (L0); the
elastic case that Sec. 6 names as the extension (``homogenize_elastic``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "em_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile em_oracle.c with gcc into liboracle.so (in place)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fcx-limited-range", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_fft3.argtypes = [ctypes.c_int, dp, ctypes.c_int]
    lib.orc_fft3.restype = None
    lib.orc_green_apply.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp]
    lib.orc_green_apply.restype = None
    lib.orc_homogenize.argtypes = [
        ctypes.c_int, ctypes.POINTER(ctypes.c_uint8), dp, ctypes.c_double,
        ctypes.c_int, ctypes.c_int, dp, dp, ip, ip, dp, dp, dp, ctypes.c_int, dp,
        ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.orc_homogenize.restype = ctypes.c_int
    lib.orc_homogenize_elastic.argtypes = [
        ctypes.c_int, ctypes.POINTER(ctypes.c_uint8), dp, ctypes.c_int, dp, ctypes.c_double,
        ctypes.c_int, dp, ip, ip, dp, dp, ctypes.c_int, dp]
    lib.orc_homogenize_elastic.restype = ctypes.c_int
    lib.orc_equilibrium_error.argtypes = [ctypes.c_int, dp, dp]
    lib.orc_equilibrium_error.restype = ctypes.c_double
    lib.orc_threads.argtypes = []
    lib.orc_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_set_threads.restype = None
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().orc_threads())


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


def fft3(a: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unnormalised full complex 3D DFT of an (n, n, n) array, [z][y][x]."""
    lib = _load()
    n = a.shape[0]
    assert a.shape == (n, n, n)
    buf = np.ascontiguousarray(a, dtype=np.complex128).copy()
    lib.orc_fft3(n, _dp(buf.view(np.float64)), int(sign))
    return buf


def green_apply(tau_hat: np.ndarray, k0: float, E) -> np.ndarray:
    """Step 4 of the Algorithm on three full spectra, shape (3, n, n, n)."""
    lib = _load()
    n = tau_hat.shape[1]
    assert tau_hat.shape == (3, n, n, n)
    t = np.ascontiguousarray(tau_hat, dtype=np.complex128)
    out = np.empty_like(t)
    Ev = np.ascontiguousarray(E, dtype=np.float64)
    lib.orc_green_apply(n, float(k0), _dp(Ev), _dp(t.view(np.float64)),
                        _dp(out.view(np.float64)))
    return out


def equilibrium_error(kvox: np.ndarray, field: np.ndarray) -> float:
    """eps_eq of step 1 (the scale-free reading) for one load case: kvox the
    (n, n, n) voxel conductivities, field the (3, n, n, n) gradient field."""
    lib = _load()
    k = np.ascontiguousarray(kvox, dtype=np.float64)
    n = k.shape[0]
    assert k.shape == (n, n, n)
    f = np.ascontiguousarray(field, dtype=np.float64)
    assert f.shape == (3, n, n, n)
    return float(lib.orc_equilibrium_error(n, _dp(k), _dp(f)))


@dataclass
class OracleResult:
    K: np.ndarray            # (3, 3), column j = load case e_j
    iters: np.ndarray        # (3,)
    status: np.ndarray       # (3,)
    final_residual: np.ndarray
    eps_eq: np.ndarray
    history: list            # per load case, eps_comp per iteration
    field: np.ndarray | None  # (3 lc, 3 comp, n, n, n) or None


def homogenize(phases: np.ndarray, k_phases, tol: float = 1e-6, max_iter: int = 10000,
               eq_check: bool = False, init_field: np.ndarray | None = None,
               want_field: bool = False, hist_cap: int | None = None,
               lc_mask: int = 7, scheme: int = 0, alpha: float = 2.0) -> OracleResult:
    """Run the Algorithm (Sec. 3) for E = e_1, e_2, e_3 on a phase image.
    scheme: 0 accelerated, 1 basic, 2 augmented Lagrangian, 3 dual,
    4 polarization (relaxation alpha)."""
    lib = _load()
    ph = np.ascontiguousarray(phases, dtype=np.uint8)
    n = ph.shape[0]
    assert ph.shape == (n, n, n)
    k = np.ascontiguousarray(k_phases, dtype=np.float64)
    assert k.shape == (3,)
    K = np.zeros(9)
    iters = np.zeros(3, dtype=np.int32)
    status = np.zeros(3, dtype=np.int32)
    res = np.zeros(3)
    eq = np.zeros(3)
    hc = int(max_iter if hist_cap is None else hist_cap)
    hist = np.zeros(3 * hc)
    init = None
    if init_field is not None:
        init = np.ascontiguousarray(init_field, dtype=np.float64)
        assert init.size == 9 * n ** 3
    field = np.zeros((3, 3, n, n, n)) if want_field else None
    rc = lib.orc_homogenize(
        n, ph.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _dp(k), float(tol),
        int(max_iter), int(bool(eq_check)), _dp(init) if init is not None else None,
        _dp(K), iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
        status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(res), _dp(eq),
        _dp(hist), hc, _dp(field) if field is not None else None, int(lc_mask), int(scheme),
        float(alpha))
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (code {rc})")
    h = hist.reshape(3, hc)
    history = [h[j, :min(int(iters[j]), hc)].copy() for j in range(3)]
    return OracleResult(K.reshape(3, 3), iters, status, res, eq, history, field)


# Tensor components of the elastic fields: 11, 22, 33, 23, 13, 12 (tensor,
# not engineering, shear components).
EL_COMPS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


@dataclass
class ElasticResult:
    S: np.ndarray            # (nlc, 6) mean stress per load case
    iters: np.ndarray
    status: np.ndarray
    final_residual: np.ndarray
    history: list
    field: np.ndarray | None  # (nlc, 6, n, n, n) or None


def homogenize_elastic(phases: np.ndarray, moduli, E, tol: float = 1e-6, max_iter: int = 10000,
                       want_field: bool = False, hist_cap: int | None = None) -> ElasticResult:
    """The accelerated scheme for isotropic elastic phases.  moduli: (3, 2)
    bulk and shear modulus per phase; E: (nlc, 6) imposed mean strains
    (components 11, 22, 33, 23, 13, 12 of the tensor)."""
    lib = _load()
    ph = np.ascontiguousarray(phases, dtype=np.uint8)
    n = ph.shape[0]
    assert ph.shape == (n, n, n)
    mod = np.ascontiguousarray(moduli, dtype=np.float64).reshape(6)
    Ev = np.ascontiguousarray(E, dtype=np.float64).reshape(-1, 6)
    nlc = Ev.shape[0]
    S = np.zeros((nlc, 6))
    iters = np.zeros(nlc, dtype=np.int32)
    status = np.zeros(nlc, dtype=np.int32)
    res = np.zeros(nlc)
    hc = int(max_iter if hist_cap is None else hist_cap)
    hist = np.zeros(nlc * hc)
    field = np.zeros((nlc, 6, n, n, n)) if want_field else None
    rc = lib.orc_homogenize_elastic(
        n, ph.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _dp(mod), nlc, _dp(Ev), float(tol),
        int(max_iter), _dp(S), iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
        status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(res), _dp(hist), hc,
        _dp(field) if field is not None else None)
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (code {rc})")
    h = hist.reshape(nlc, hc)
    history = [h[j, :min(int(iters[j]), hc)].copy() for j in range(nlc)]
    return ElasticResult(S, iters, status, res, history, field)
