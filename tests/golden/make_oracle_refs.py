"""Write oracle reference tensors for the full-size parity tests.

Calls only the FP64 oracle (``oracle/``) and the seeded input generator; no
value here comes from the GPU path.  Output: ``oracle_refs.json`` beside this
script.  Run from the repository root:  python tests/golden/make_oracle_refs.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1504_07499_amd import geom  # noqa: E402

K_CFG = [0.2, 0.3, 400.0]

# name: (n, n_spheres, volume fraction, layer, seed, k, tol, max_iter, lc_mask)
CASES = {
    # 32^3, 8 spheres, f = 0.2, l = 0.1, seed 1, tol 1e-6 (full solve)
    "rve32_8sph_f0.20_l0.10_seed1": (32, 8, 0.2, 0.1, 1, K_CFG, 1e-6, 10000, 7),
    # 128^3, 50 spheres, f = 0.3, l = 0.2, seed 2, tol 1e-6 (full solve)
    "rve128_50sph_f0.30_l0.20_seed2": (128, 50, 0.3, 0.2, 2, K_CFG, 1e-6, 10000, 7),
    # 256^3, 100 spheres, f = 0.4 (RSA, then the Monte Carlo fallback), seed 3,
    # the same centres for every layer; k_coating = 0.2 c for contrast c
    "rve256_100sph_f0.40_l0.10_c1e3_seed3": (256, 100, 0.4, 0.1, 3, [0.2, 0.3, 200.0], 1e-6, 10000, 7),
    "rve256_100sph_f0.40_l0.20_c1e2_seed3": (256, 100, 0.4, 0.2, 3, [0.2, 0.3, 20.0], 1e-6, 10000, 7),
    "rve256_100sph_f0.40_l0.05_c1e4_seed3": (256, 100, 0.4, 0.05, 3, [0.2, 0.3, 2000.0], 1e-6, 10000, 7),
}


def main():
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_refs.json")
    refs = {}
    if os.path.exists(out_path):
        with open(out_path) as f:
            refs = json.load(f)
    only = sys.argv[1:]
    for name, (n, nsp, f, layer, seed, k, tol, max_iter, mask) in CASES.items():
        if only and name not in only:
            continue
        ph, _, method = geom.generate(n, nsp, f, layer, seed)
        t0 = time.time()
        r = oracle.homogenize(ph, k, tol=tol, max_iter=max_iter, lc_mask=mask)
        dt = time.time() - t0
        refs[name] = {
            "geometry": {"n": n, "n_spheres": nsp, "volume_fraction": f, "layer": layer,
                         "seed": seed, "placement_method": method},
            "phase_fractions": (np.bincount(ph.ravel(), minlength=3) / ph.size).tolist(),
            "k_phases": k, "tol": tol, "max_iter": max_iter, "lc_mask": mask,
            "K": r.K.tolist(), "iters": r.iters.tolist(), "status": r.status.tolist(),
            "final_residual": r.final_residual.tolist(), "eps_eq": r.eps_eq.tolist(),
            "oracle_seconds": dt, "oracle_threads": oracle.threads(),
        }
        print(name, r.iters.tolist(), f"{dt:.1f}s", flush=True)
        with open(out_path, "w") as fh:
            json.dump(refs, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
