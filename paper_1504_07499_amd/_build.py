"""In-tree build of the native libraries (no JIT cache, no site-packages).

* ``librvegeom.so``  -- seeded input generator (g++), ``geom/rve_geom.cpp``.
* ``librvehom.so``   -- HIP kernels for gfx950 + the C ABI of
  ``include/rvehom.h`` (hipcc), ``csrc/*.hip`` plus the generator source.
"""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def geom_lib_path() -> str:
    return os.path.join(PKG, "librvegeom.so")


def hip_lib_path() -> str:
    return os.path.join(PKG, "librvehom.so")


def _run(cmd):
    subprocess.run(cmd, check=True)


def build_geom() -> str:
    out = geom_lib_path()
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", INCLUDE, "-o", out + ".tmp",
          os.path.join(PKG, "geom", "rve_geom.cpp")])
    os.replace(out + ".tmp", out)
    return out


def hip_sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def kernel_source_hash() -> str:
    """Short hash of the sources that define the kernels and their launch
    shapes (csrc/*.hip and *.hpp except the host-side rvehom_* files):
    counter summaries record it, so that figures taken on other kernels are
    not reused."""
    h = hashlib.sha256()
    csrc = os.path.join(PKG, "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")) and not name.startswith("rvehom_"):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def hip_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            # packed FP32 instructions stay off (see the design notes)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", os.path.join(PKG, "csrc"),
            "-Wno-unused-command-line-argument"]


def build_hip(jobs: int = 8) -> str:
    """Compile every csrc/*.hip to an object for gfx950, then link the C ABI."""
    out = hip_lib_path()
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    srcs = hip_sources()
    for src in srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *hip_flags(), "-c", src, "-o", obj]))
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError("hipcc failed")
    gobj = os.path.join(objdir, "rve_geom.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-c", "-I", INCLUDE,
          os.path.join(PKG, "geom", "rve_geom.cpp"), "-o", gobj])
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", out + ".tmp", *objs, gobj])
    os.replace(out + ".tmp", out)
    return out


def build_all() -> None:
    build_geom()
    build_hip()
