"""The paper's stochastic study on the GPU path (arXiv:1504.07499, Sec. 5).

For each (resolution, number of spheres, layer) the paper generates 10 RSA
samples at sphere volume fraction 0.30, computes the conductivity tensor with
the accelerated scheme and averages the mean of its diagonal (the composite is
close to isotropic) over the samples.  Conductivities: matrix 1, inclusion 0.2,
coating 400.  This module runs that sweep through ``homogenize_batch`` (all
samples of one set in one batched solve) and returns mean and standard
deviation of the isotropic value per set.

Command line (GPU):  python -m paper_1504_07499_amd.study --res 64 128 --samples 10
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import homogenize_batch, rve_create

PAPER_K = (1.0, 0.2, 400.0)  # matrix, inclusion, coating (Sec. 5)
PAPER_RES = (64, 128, 256)
PAPER_NSP = (30, 40, 50, 60, 70, 80, 90, 100)
PAPER_LAYERS = (0.02, 0.04, 0.06, 0.08, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9)


def isotropic_value(K: np.ndarray) -> float:
    """Mean of the diagonal of the tensor (Sec. 5)."""
    return float(np.trace(K) / 3.0)


def sample_seed(res: int, nsp: int, layer: float, i: int) -> int:
    """Seed of sample i of a set; the same centres are reused across layers
    so that curves versus l compare identical sphere arrangements."""
    return 1_000_003 * res + 1009 * nsp + i


def run_set(res, nsp, layer, samples, k=PAPER_K, f=0.3, tol=1e-5, precision=0):
    rves = [rve_create(res, nsp, f, layer, sample_seed(res, nsp, layer, i)) for i in range(samples)]
    try:
        out = homogenize_batch(rves, k, tol, precision=precision)
    finally:
        for r in rves:
            r.close()
    vals = np.array([isotropic_value(o.K) for o in out])
    iters = np.array([o.iters.max() for o in out])
    return {"res": res, "n_sp": nsp, "layer": layer, "samples": samples,
            "k_iso_mean": float(vals.mean()), "k_iso_std": float(vals.std(ddof=1)) if samples > 1 else 0.0,
            "iters_mean": float(iters.mean()), "status": [int(o.status) for o in out],
            "seeds": [sample_seed(res, nsp, layer, i) for i in range(samples)],
            "K": [o.K.tolist() for o in out]}


def sweep(res_list=PAPER_RES, nsp_list=PAPER_NSP, layers=PAPER_LAYERS, samples=10, **kw):
    rows = []
    for res in res_list:
        for nsp in nsp_list:
            for layer in layers:
                t0 = time.perf_counter()
                row = run_set(res, nsp, layer, samples, **kw)
                row["seconds"] = time.perf_counter() - t0
                rows.append(row)
                print(json.dumps(row), flush=True)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--res", type=int, nargs="+", default=list(PAPER_RES))
    ap.add_argument("--nsp", type=int, nargs="+", default=list(PAPER_NSP))
    ap.add_argument("--layers", type=float, nargs="+", default=list(PAPER_LAYERS))
    ap.add_argument("--samples", type=int, default=10)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--precision", type=int, default=0)
    a = ap.parse_args(argv)
    sweep(a.res, a.nsp, a.layers, a.samples, tol=a.tol, precision=a.precision)


if __name__ == "__main__":
    sys.exit(main())
