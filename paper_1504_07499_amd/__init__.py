"""MI355X-native accelerated FFT homogenization of three-phase voxel RVEs.

Thin Python binding of the C ABI in ``include/rvehom.h`` (``librvehom.so``,
built in-tree for gfx950).  Every step of the solve runs in the library's HIP
kernels; this module only marshals arguments.  There is no CPU fallback:
the first call raises ImportError if the native library is missing.

Paper: S. Lemaitre, V. Salnikov, D. Choi, P. Karamian, "Computation of thermal
properties via 3D homogenization of multiphase materials using FFT-based
accelerated scheme", arXiv:1504.07499 -- Sec. 2 (RVE generation), Sec. 3
(the Algorithm of the accelerated scheme and L_hom from <phi>), Sec. 5 (L0).

PyTorch is optional and only used for device memory and streams: pass
``stream=torch.cuda.current_stream()`` and/or a ``workspace`` CUDA uint8
tensor of at least ``rve_workspace_size(rve, precision)`` bytes.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import _build

__all__ = [
    "RveError", "RVE", "HomResult", "rve_supported_n", "rve_create", "rve_create_from_phases",
    "rve_get_phases", "rve_get_spheres", "rve_workspace_size", "homogenize", "homogenize_batch", "homogenize_no_alloc",
    "rve_get_kernel_times", "rve_server_create", "rve_server_submit", "rve_server_poll",
    "rve_server_drain", "rve_server_get_stats", "rve_server_destroy", "rve_destroy", "rve_last_error", "library_path",
    "RVE_OK", "RVE_NOT_CONVERGED", "RVE_STALLED", "RVE_PENDING", "RVE_ERR_ARG", "RVE_ERR_JAMMED",
    "RVE_ERR_OOM", "RVE_ERR_DEVICE", "RVE_ERR_NONFINITE",
]

RVE_OK, RVE_NOT_CONVERGED, RVE_STALLED, RVE_PENDING = 0, 1, 2, 3
RVE_ERR_ARG, RVE_ERR_JAMMED, RVE_ERR_OOM, RVE_ERR_DEVICE, RVE_ERR_NONFINITE = -1, -2, -3, -4, -5


class _Geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("n_spheres", ctypes.c_int),
                ("volume_fraction", ctypes.c_double), ("layer", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class _Opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("precision", ctypes.c_int),
                ("equilibrium_check", ctypes.c_int), ("stall_window", ctypes.c_int),
                ("lc_mask", ctypes.c_int), ("timing", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("init_field", ctypes.POINTER(ctypes.c_double)),
                ("out_field", ctypes.POINTER(ctypes.c_double)), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("scheme", ctypes.c_int),
                ("fp32_refine", ctypes.c_int), ("path_flags", ctypes.c_int),
                ("alpha", ctypes.c_double)]


class _Result(ctypes.Structure):
    _fields_ = [("K", ctypes.c_double * 9), ("iters", ctypes.c_int * 3),
                ("status", ctypes.c_int * 3), ("final_residual", ctypes.c_double * 3),
                ("eps_eq", ctypes.c_double * 3), ("solve_ms", ctypes.c_double),
                ("refine_iters", ctypes.c_int * 3)]


class _ElResult(ctypes.Structure):
    _fields_ = [("C", ctypes.c_double * 36), ("C_basis", ctypes.c_double * 36),
                ("iters", ctypes.c_int * 6), ("status", ctypes.c_int * 6),
                ("final_residual", ctypes.c_double * 6), ("solve_ms", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
                ("resident_peak", ctypes.c_int), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("refined", ctypes.c_uint64),
                ("graph_hits", ctypes.c_uint64), ("graph_misses", ctypes.c_uint64)]


class _KTimes(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p * 4), ("total_ms", ctypes.c_double * 4),
                ("launches", ctypes.c_int * 4), ("total_bytes", ctypes.c_double * 4)]


def library_path() -> str:
    return _build.hip_lib_path()


def _load_library():
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first (__graft_entry__.build()); "
            "there is no CPU fallback")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    c_int, c_double, c_size_t, c_vp = ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
    sig = {
        "rve_supported_n": (c_int, [c_int, P(c_int), c_int, P(c_int)]),
        "rve_tune_export": (c_size_t, [ctypes.c_char_p, c_size_t]),
        "rve_tune_import": (c_int, [ctypes.c_char_p]),
        "rve_create": (c_int, [P(_Geom), P(c_vp)]),
        "rve_create_from_phases": (c_int, [c_int, P(ctypes.c_uint8), P(c_vp)]),
        "rve_get_phases": (c_int, [c_vp, P(ctypes.c_uint8), c_size_t]),
        "rve_get_spheres": (c_int, [c_vp, P(c_double), c_int, P(c_int), P(c_double)]),
        "rve_n": (c_int, [c_vp]),
        "rve_workspace_size": (c_size_t, [c_vp, c_int]),
        "homogenize": (c_int, [c_vp, P(c_double), c_double, P(_Opts), P(_Result), P(c_double), c_int]),
        "homogenize_batch": (c_int, [c_int, P(c_vp), P(c_double), P(c_double), P(_Opts), P(_Result)]),
        "homogenize_no_alloc": (c_int, [c_vp, P(c_double), c_double, P(_Opts), P(_Result), P(c_double), c_int]),
        "rve_get_kernel_times": (c_int, [c_vp, P(_KTimes)]),
        "homogenize_elastic": (c_int, [c_vp, P(c_double), c_double, P(_Opts), P(_ElResult), P(c_double), c_int]),
        "rve_supported_n_elastic": (c_int, [c_int, P(c_int), c_int, P(c_int)]),
        "rve_server_create": (c_int, [c_size_t, c_int, c_int, P(c_vp)]),
        "rve_server_submit": (c_int, [c_vp, P(_Geom), P(c_double), c_double, P(ctypes.c_uint64)]),
        "rve_server_poll": (c_int, [c_vp, ctypes.c_uint64, P(_Result), P(c_double)]),
        "rve_server_drain": (c_int, [c_vp]),
        "rve_server_get_stats": (c_int, [c_vp, P(_ServerStats)]),
        "rve_server_destroy": (None, [c_vp]),
        "rve_destroy": (None, [c_vp]),
        "rve_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class _LazyLib:
    """Loads librvehom.so on first use, so that importing the input generator
    (``paper_1504_07499_amd.geom``) does not touch the GPU library."""

    _lib = None

    def __getattr__(self, name):
        if _LazyLib._lib is None:
            _LazyLib._lib = _load_library()
        return getattr(_LazyLib._lib, name)


_lib = _LazyLib()


class RveError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


def rve_last_error() -> str:
    return (_lib.rve_last_error() or b"").decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise RveError(rc, rve_last_error())
    return rc


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


class RVE:
    """Owning wrapper of an ``rve_t`` handle."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        if not self._h:
            raise RveError(RVE_ERR_ARG, "RVE handle already destroyed")
        return self._h

    @property
    def n(self) -> int:
        return int(_lib.rve_n(self.handle))

    def close(self):
        if self._h:
            _lib.rve_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def rve_supported_n(precision: int = 0) -> list:
    out = (ctypes.c_int * 64)()
    cnt = ctypes.c_int(0)
    _check(_lib.rve_supported_n(int(precision), out, 64, ctypes.byref(cnt)))
    return [int(out[i]) for i in range(min(cnt.value, 64))]


def rve_tune_export() -> str:
    """The autotuner's choices of this process, as text lines
    "<gfx arch> <precision> <n> ztile <0|1>" (z-pass tile width) and
    "<gfx arch> <precision> <n> plane <0|1>" (fused plane pass threads)."""
    need = int(_lib.rve_tune_export(None, 0))
    buf = ctypes.create_string_buffer(need)
    _lib.rve_tune_export(buf, need)
    return buf.value.decode()


def rve_tune_import(text: str) -> None:
    """Adds autotuner choices (text of rve_tune_export); they replace the
    timing for their (architecture, precision, N)."""
    _check(_lib.rve_tune_import(text.encode()))


def rve_tune_save(path: str) -> None:
    """Writes this process's autotuner choices to path (merged with the
    choices already there for other grids or architectures)."""
    lines = {}
    if os.path.exists(path):
        with open(path) as f:
            for ln in f:
                if ln.strip():
                    lines[tuple(ln.split()[:4])] = ln.strip()
    for ln in rve_tune_export().splitlines():
        if ln.strip():
            lines[tuple(ln.split()[:4])] = ln.strip()
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("".join(v + "\n" for v in sorted(lines.values())))
    os.replace(tmp, path)


def rve_tune_load(path: str) -> bool:
    """Imports the autotuner choices saved at path; False if there is no file."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        rve_tune_import(f.read())
    return True


def rve_create(n: int, n_spheres: int, volume_fraction: float, layer: float, seed: int) -> RVE:
    """RSA + voxelization (Sec. 2) of an N^3 RVE, uploaded to the device."""
    g = _Geom(int(n), int(n_spheres), float(volume_fraction), float(layer), int(seed))
    h = ctypes.c_void_p()
    _check(_lib.rve_create(ctypes.byref(g), ctypes.byref(h)))
    return RVE(h.value)


def rve_create_from_phases(phases: np.ndarray) -> RVE:
    ph = np.ascontiguousarray(phases, dtype=np.uint8)
    n = ph.shape[0]
    if ph.shape != (n, n, n):
        raise RveError(RVE_ERR_ARG, f"phase image must be (n, n, n), got {ph.shape}")
    h = ctypes.c_void_p()
    _check(_lib.rve_create_from_phases(n, ph.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                       ctypes.byref(h)))
    return RVE(h.value)


def rve_get_phases(rve: RVE) -> np.ndarray:
    n = rve.n
    out = np.empty((n, n, n), dtype=np.uint8)
    _check(_lib.rve_get_phases(rve.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                               out.size))
    return out


def rve_get_spheres(rve: RVE):
    """(xyzr (count, 4), layer)."""
    cnt = ctypes.c_int(0)
    layer = ctypes.c_double(0.0)
    _check(_lib.rve_get_spheres(rve.handle, None, 0, ctypes.byref(cnt), ctypes.byref(layer)))
    out = np.zeros((cnt.value, 4))
    if cnt.value:
        _check(_lib.rve_get_spheres(rve.handle, _dptr(out), cnt.value, ctypes.byref(cnt),
                                    ctypes.byref(layer)))
    return out, float(layer.value)


def rve_workspace_size(rve: RVE, precision: int = 0) -> int:
    return int(_lib.rve_workspace_size(rve.handle, int(precision)))


@dataclass
class HomResult:
    status: int
    K: np.ndarray
    iters: np.ndarray
    lc_status: np.ndarray
    final_residual: np.ndarray
    eps_eq: np.ndarray
    solve_ms: float
    history: list = field(default_factory=list)
    field: np.ndarray | None = None
    refine_iters: np.ndarray | None = None  # FP64 iterations past the FP32 floor


def _to_result(rc: int, r: _Result, hist=None, hist_cap=0, fld=None) -> HomResult:
    iters = np.array(r.iters[:], dtype=np.int64)
    history = []
    if hist is not None:
        h = hist.reshape(3, hist_cap)
        history = [h[j, :min(int(iters[j]), hist_cap)].copy() for j in range(3)]
    return HomResult(rc, np.array(r.K[:]).reshape(3, 3), iters, np.array(r.status[:]),
                     np.array(r.final_residual[:]), np.array(r.eps_eq[:]), float(r.solve_ms),
                     history, fld, np.array(r.refine_iters[:], dtype=np.int64))


SCHEMES = {"accelerated": 0, "basic": 1, "augmented_lagrangian": 2, "dual": 3, "polarization": 4}

# measurement switches of rve_opts.path_flags (results do not depend on them)
PATH_NO_GRAPHS, PATH_NO_FUSED, PATH_NO_MERGE, PATH_NO_CHAINS = 1, 2, 4, 8
PATH_ZTILE_DEFAULT, PATH_ZTILE_ALT = 16, 32
PATH_PLANE_DEFAULT, PATH_PLANE_ALT = 64, 128


def _opts(max_iter=0, precision=0, equilibrium_check=False, stall_window=-1, lc_mask=7,
          timing=False, stream=None, init_field=None, out_field=None, workspace=None,
          scheme="accelerated", fp32_refine=True, path_flags=0, alpha=0.0):
    o = _Opts()
    o.alpha = float(alpha)
    o.fp32_refine = 0 if fp32_refine else -1
    o.path_flags = int(path_flags)
    o.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    o.max_iter = int(max_iter)
    o.precision = int(precision)
    o.equilibrium_check = int(bool(equilibrium_check))
    o.stall_window = int(stall_window)
    o.lc_mask = int(lc_mask)
    # timing: True = all four kernels, or a bitmask (1 fwd_plane, 2 zgreen,
    # 4 inv_plane, 8 reduce; + 16 = time one batch of iterations in four)
    o.timing = 15 if timing is True else int(timing)
    o.stream = _stream_handle(stream)
    o.init_field = _dptr(init_field) if init_field is not None else None
    o.out_field = _dptr(out_field) if out_field is not None else None
    if workspace is not None:
        o.workspace = int(workspace.data_ptr())
        o.workspace_bytes = int(workspace.numel() * workspace.element_size())
    return o


def homogenize(rve: RVE, k_phases, tol: float = 1e-6, *, max_iter: int = 0, precision: int = 0,
               equilibrium_check: bool = False, stall_window: int = -1, lc_mask: int = 7,
               timing=False, stream=None, init_field: np.ndarray | None = None,
               want_field: bool = False, workspace=None, hist_cap: int = 0,
               scheme="accelerated", fp32_refine: bool = True, path_flags: int = 0,
               alpha: float = 0.0) -> HomResult:
    """The Algorithm of Sec. 3 for E = e_1, e_2, e_3 on the device.

    scheme: "accelerated" (Eyre-Milton, the paper's choice), "basic" (the
    basic scheme the paper names as an alternative: e+ = c, k0 = mean of the
    extreme conductivities) or "augmented_lagrangian" (also named there; k0
    of Sec. 5; the field returned is its state lam - k0 d; no equilibrium
    check), "dual" (the flux-based dual scheme, k0 the harmonic mean of the
    extremes; no start field) or "polarization" (relaxation alpha in (0, 2],
    0 = 2).  fp32_refine (precision 0): continue load cases stopped by the
    FP32 rounding floor in FP64 until eps_comp < tol.  path_flags: the
    PATH_* measurement switches."""
    k = np.ascontiguousarray(k_phases, dtype=np.float64)
    if k.shape != (3,):
        raise RveError(RVE_ERR_ARG, "k_phases must hold 3 conductivities")
    n = rve.n
    init = None
    if init_field is not None:
        init = np.ascontiguousarray(init_field, dtype=np.float64)
        if init.size != 9 * n ** 3:
            raise RveError(RVE_ERR_ARG, "init_field must hold 9 n^3 values")
    fld = np.zeros((3, 3, n, n, n)) if want_field else None
    o = _opts(max_iter, precision, equilibrium_check, stall_window, lc_mask, timing, stream, init,
              fld, workspace, scheme, fp32_refine, path_flags, alpha)
    res = _Result()
    hist = np.zeros(3 * hist_cap) if hist_cap > 0 else None
    rc = _check(_lib.homogenize(rve.handle, _dptr(k), float(tol), ctypes.byref(o), ctypes.byref(res),
                                _dptr(hist) if hist is not None else None, int(hist_cap)))
    return _to_result(rc, res, hist, hist_cap, fld)


def homogenize_no_alloc(rve: RVE, k_phases, tol: float = 1e-6, *, max_iter: int = 0, precision: int = 0,
                        stall_window: int = -1, lc_mask: int = 7, stream=None, hist_cap: int = 0,
                        scheme="accelerated", fp32_refine: bool = True, path_flags: int = 0,
                        alpha: float = 0.0) -> HomResult:
    """homogenize without any allocation: the library's fixed device array
    (64 MiB per GPU) holds the workspaces, so N <= 64."""
    k = np.ascontiguousarray(k_phases, dtype=np.float64)
    if k.shape != (3,):
        raise RveError(RVE_ERR_ARG, "k_phases must hold 3 conductivities")
    o = _opts(max_iter, precision, False, stall_window, lc_mask, False, stream, None, None, None, scheme,
              fp32_refine, path_flags, alpha)
    res = _Result()
    hist = np.zeros(3 * hist_cap) if hist_cap > 0 else None
    rc = _check(_lib.homogenize_no_alloc(rve.handle, _dptr(k), float(tol), ctypes.byref(o), ctypes.byref(res),
                                         _dptr(hist) if hist is not None else None, int(hist_cap)))
    return _to_result(rc, res, hist, hist_cap)


@dataclass
class ElasticResult:
    status: int
    C: np.ndarray          # (6, 6) Voigt stiffness (11, 22, 33, 23, 13, 12; engineering shear)
    C_basis: np.ndarray    # (6, 6) in the orthonormal basis B_0..B_5 of the kernels
    iters: np.ndarray
    lc_status: np.ndarray
    final_residual: np.ndarray
    solve_ms: float
    history: list = field(default_factory=list)
    field: np.ndarray | None = None  # (6 load cases, 6 components, n, n, n), basis components


# Orthonormal basis of symmetric tensors of the elastic case (load case j
# imposes E = B[j]; field components are e : B[k]).
def _sym_unit(i, j):
    a = np.zeros((3, 3))
    a[i, j] = a[j, i] = 1.0
    return a / np.sqrt(2.0)


ELASTIC_BASIS = np.array([
    np.eye(3) / np.sqrt(3.0),
    np.diag([1.0, -1.0, 0.0]) / np.sqrt(2.0),
    np.diag([1.0, 1.0, -2.0]) / np.sqrt(6.0),
    _sym_unit(1, 2),
    _sym_unit(0, 2),
    _sym_unit(0, 1),
])


def moduli_from_young_poisson(young, poisson):
    """(kappa, mu) per phase from Young's moduli and Poisson ratios."""
    E = np.asarray(young, dtype=np.float64)
    nu = np.asarray(poisson, dtype=np.float64)
    return np.stack([E / (3.0 * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))], axis=-1)


def homogenize_elastic(rve: RVE, moduli, tol: float = 1e-6, *, max_iter: int = 0, precision: int = 0,
                       stall_window: int = -1, stream=None, init_field: np.ndarray | None = None,
                       want_field: bool = False, hist_cap: int = 0, path_flags: int = 0) -> ElasticResult:
    """The accelerated scheme for isotropic elastic phases (the elastic case
    Sec. 6 names as the extension): moduli (3, 2) = (bulk, shear) of matrix,
    inclusion, coating; six load cases E = B_j."""
    m = np.ascontiguousarray(moduli, dtype=np.float64).reshape(-1)
    if m.shape != (6,):
        raise RveError(RVE_ERR_ARG, "moduli must hold (kappa, mu) of 3 phases")
    n = rve.n
    init = None
    if init_field is not None:
        init = np.ascontiguousarray(init_field, dtype=np.float64)
        if init.size != 36 * n ** 3:
            raise RveError(RVE_ERR_ARG, "init_field must hold 36 n^3 values")
    fld = np.zeros((6, 6, n, n, n)) if want_field else None
    o = _opts(max_iter, precision, False, stall_window, 0, False, stream, init, fld, None, path_flags=path_flags)
    res = _ElResult()
    hist = np.zeros(6 * hist_cap) if hist_cap > 0 else None
    rc = _check(_lib.homogenize_elastic(rve.handle, _dptr(m), float(tol), ctypes.byref(o), ctypes.byref(res),
                                        _dptr(hist) if hist is not None else None, int(hist_cap)))
    iters = np.array(res.iters[:], dtype=np.int64)
    history = []
    if hist is not None:
        h = hist.reshape(6, hist_cap)
        history = [h[j, :min(int(iters[j]), hist_cap)].copy() for j in range(6)]
    return ElasticResult(rc, np.array(res.C[:]).reshape(6, 6), np.array(res.C_basis[:]).reshape(6, 6), iters,
                         np.array(res.status[:]), np.array(res.final_residual[:]), float(res.solve_ms),
                         history, fld)


def rve_supported_n_elastic(precision: int = 0) -> list:
    """Grid sizes of the elastic case for a precision."""
    buf = (ctypes.c_int * 64)()
    cnt = ctypes.c_int(0)
    _check(_lib.rve_supported_n_elastic(int(precision), buf, 64, ctypes.byref(cnt)))
    return list(buf[:cnt.value])


def homogenize_batch(rves, k_phases, tol, *, max_iter: int = 0, precision: int = 0,
                     stall_window: int = -1, equilibrium_check: bool = False,
                     scheme="accelerated", fp32_refine: bool = True, alpha: float = 0.0) -> list:
    """Several RVEs (mixed N) solved concurrently; returns one HomResult each."""
    count = len(rves)
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k_phases, dtype=np.float64), (count, 3)))
    t = np.ascontiguousarray(np.broadcast_to(np.asarray(tol, dtype=np.float64), (count,)))
    hs = (ctypes.c_void_p * max(count, 1))(*[r.handle.value for r in rves])
    o = _opts(max_iter, precision, equilibrium_check, stall_window, scheme=scheme, fp32_refine=fp32_refine,
              alpha=alpha)
    out = (_Result * max(count, 1))()
    rc = _check(_lib.homogenize_batch(count, hs, _dptr(k), _dptr(t), ctypes.byref(o), out))
    res = []
    for i in range(count):
        r = _to_result(0, out[i])
        st = [int(s) for s in r.lc_status]
        r.status = min(st) if min(st) < 0 else max(st)
        res.append(r)
    _ = rc
    return res


def rve_get_kernel_times(rve: RVE) -> dict:
    kt = _KTimes()
    _check(_lib.rve_get_kernel_times(rve.handle, ctypes.byref(kt)))
    out = {}
    for i in range(4):
        name = kt.name[i].decode() if kt.name[i] else f"k{i}"
        out[name] = {"total_ms": float(kt.total_ms[i]), "launches": int(kt.launches[i]),
                     "total_bytes": float(kt.total_bytes[i])}
    return out


def rve_destroy(rve: RVE) -> None:
    rve.close()


# ---------------------------------------------------------------- serving
def rve_server_create(hbm_budget_bytes: int, max_slots: int, precision: int = 0):
    h = ctypes.c_void_p()
    _check(_lib.rve_server_create(int(hbm_budget_bytes), int(max_slots), int(precision),
                                  ctypes.byref(h)))
    return h


def rve_server_submit(server, n, n_spheres, volume_fraction, layer, seed, k_phases, tol) -> int:
    g = _Geom(int(n), int(n_spheres), float(volume_fraction), float(layer), int(seed))
    k = np.ascontiguousarray(k_phases, dtype=np.float64)
    t = ctypes.c_uint64(0)
    _check(_lib.rve_server_submit(server, ctypes.byref(g), _dptr(k), float(tol), ctypes.byref(t)))
    return int(t.value)


def rve_server_poll(server, ticket: int):
    """None while pending, else (HomResult, latency_s)."""
    res = _Result()
    lat = ctypes.c_double(0.0)
    rc = _lib.rve_server_poll(server, ctypes.c_uint64(int(ticket)), ctypes.byref(res),
                              ctypes.byref(lat))
    if rc == RVE_PENDING:
        return None
    if rc in (RVE_ERR_ARG, RVE_ERR_DEVICE):
        raise RveError(rc, rve_last_error())
    return _to_result(rc, res), float(lat.value)


def rve_server_drain(server) -> None:
    _check(_lib.rve_server_drain(server))


def rve_server_get_stats(server) -> dict:
    st = _ServerStats()
    _check(_lib.rve_server_get_stats(server, ctypes.byref(st)))
    return {name: int(getattr(st, name)) for name, _ in _ServerStats._fields_}


def rve_server_destroy(server) -> None:
    _lib.rve_server_destroy(server)
