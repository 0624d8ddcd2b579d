"""Seeded synthetic workloads beyond the single-RVE benchmark, run through the
C ABI: the batched realizations, the serving trace and the 256^3 contrast
sweep.  All parameters are drawn from seeded generators; the RVE geometry
follows Sec. 2 of arXiv:1504.07499 (RSA spheres, coating layer l), the solve
follows the Algorithm of Sec. 3.

Command line (GPU):
  python -m paper_1504_07499_amd.workloads batch  [--count 64]
  python -m paper_1504_07499_amd.workloads serve  [--rate 200 --requests 2000]
  python -m paper_1504_07499_amd.workloads sweep256
  python -m paper_1504_07499_amd.workloads rates  [--requests 200 --rate 200]
  python -m paper_1504_07499_amd.workloads run512
  python -m paper_1504_07499_amd.workloads schemes [--precision 1]
  python -m paper_1504_07499_amd.workloads fibers
  python -m paper_1504_07499_amd.workloads elastic
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import threading
import time

import numpy as np

from . import (homogenize, homogenize_batch, rve_create, rve_create_from_phases, rve_server_create,
               rve_server_destroy, rve_server_drain, rve_server_poll, rve_server_submit)
from .geom import generate_fibers

K_BENCH = (0.2, 0.3, 400.0)  # matrix, inclusion, coating


# --------------------------------------------------------------------------- batch
def batch_specs(count=64, seed=4):
    """count RVEs: N uniform on {64, 96, 128}, 20-100 spheres, volume fraction
    U[0.10, 0.40], layer U[0.05, 0.30]; RVE seeds 1000 + i."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        specs.append((int(rng.choice([64, 96, 128])), int(rng.integers(20, 101)),
                      float(rng.uniform(0.10, 0.40)), float(rng.uniform(0.05, 0.30)), 1000 + i))
    return specs


def run_batch(count=64, seed=4, precision=0, tol=1e-6, check_alone=4):
    specs = batch_specs(count, seed)
    rves = [rve_create(*s) for s in specs]
    try:
        homogenize_batch(rves[:2], K_BENCH, tol, precision=precision)  # warm-up (graphs, workspaces)
        t0 = time.perf_counter()
        res = homogenize_batch(rves, K_BENCH, tol, precision=precision)
        wall = time.perf_counter() - t0
        Ks = np.array([r.K for r in res])
        vox = sum(s[0] ** 3 * int(r.iters.sum()) for s, r in zip(specs, res))
        same = True
        for i in range(min(check_alone, count)):
            a = homogenize(rves[i], K_BENCH, tol, precision=precision)
            same &= bool(np.array_equal(a.K, res[i].K))
        # the same solves one after another, each timed: the rate each grid
        # size reaches alone bounds what any batching can gain
        per_n = {}
        t1 = time.perf_counter()
        for s_, r in zip(specs, rves):
            ta = time.perf_counter()
            a = homogenize(r, K_BENCH, tol, precision=precision)
            d = per_n.setdefault(s_[0], {"solves": 0, "seconds": 0.0, "voxel_iters": 0})
            d["solves"] += 1
            d["seconds"] += time.perf_counter() - ta
            d["voxel_iters"] += s_[0] ** 3 * int(a.iters.sum())
        seq = time.perf_counter() - t1
    finally:
        for r in rves:
            r.close()
    for d in per_n.values():
        d["voxel_iters_per_s_per_lc"] = d["voxel_iters"] / d["seconds"]
    best = max(d["voxel_iters_per_s_per_lc"] for d in per_n.values())
    return {"workload": f"batch of {count} RVEs, N in {{64,96,128}}, seed {seed}",
            "precision": "fp32" if precision == 0 else "fp64", "tol": tol,
            "wall_s": wall, "solves_per_s": count / wall, "voxel_iters_per_s_per_lc": vox / wall,
            "sequential_wall_s": seq, "batch_speedup_vs_sequential": seq / wall,
            "sequential_by_n": {str(n_): d for n_, d in sorted(per_n.items())},
            # batched rate over the best rate of one grid size solved alone:
            # the ceiling a persistent multi-RVE kernel could at most approach
            "batch_rate_over_best_alone": (vox / wall) / best,
            "K_mean": Ks.mean(0).tolist(), "K_var": Ks.var(0, ddof=1).tolist(),
            "k_iso_mean": float(np.mean([np.trace(k) / 3 for k in Ks])),
            "status_counts": {str(s): int(sum(1 for r in res if r.status == s)) for s in set(r.status for r in res)},
            "alone_equals_batched": same}


# --------------------------------------------------------------------------- serve
def serve_trace(requests=2000, rate=200.0, seed=5):
    """Poisson arrivals at `rate` per second; N uniform on {32, 64, 128, 256};
    10-100 spheres; contrast log-uniform in [10, 1e4] (coating 0.2 c);
    volume fraction U[0.10, 0.30]; layer U[0.05, 0.30]."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=requests))
    out = []
    for i in range(requests):
        c = 10.0 ** rng.uniform(1.0, 4.0)
        out.append({"t": float(t[i]), "n": int(rng.choice([32, 64, 128, 256])),
                    "n_spheres": int(rng.integers(10, 101)), "f": float(rng.uniform(0.10, 0.30)),
                    "layer": float(rng.uniform(0.05, 0.30)), "seed": 5000 + i,
                    "k": (0.2, 0.3, 0.2 * c), "contrast": c})
    return out


def _pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def run_serve(trace, precision=0, tol=1e-6, budget_bytes=64 << 30, slots=16):
    """Continuous batching: submit each request at its arrival time; the
    library admits requests by footprint and slot while others iterate."""
    srv = rve_server_create(budget_bytes, slots, precision)
    tickets = [None] * len(trace)
    t0 = time.perf_counter()

    def submitter():
        for i, r in enumerate(trace):
            dt = t0 + r["t"] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            tickets[i] = rve_server_submit(srv, r["n"], r["n_spheres"], r["f"], r["layer"], r["seed"],
                                           r["k"], tol)
            if (i + 1) % 100 == 0:
                print(f"[serve] {i + 1} of {len(trace)} submitted at {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    rve_server_drain(srv)
    makespan = time.perf_counter() - t0
    lat, results = [], []
    for tk in tickets:
        res, l = rve_server_poll(srv, tk)
        lat.append(l)
        results.append(res)
    rve_server_destroy(srv)
    return {"mode": "served (continuous batching)", "precision": "fp32" if precision == 0 else "fp64",
            "requests": len(trace), "makespan_s": makespan, "solves_per_s": len(trace) / makespan,
            "p50_latency_s": _pct(lat, 50), "p99_latency_s": _pct(lat, 99),
            "status_counts": {str(s): int(sum(1 for r in results if r.status == s))
                              for s in set(r.status for r in results)}}, results


def run_sequential(trace, precision=1, tol=1e-6):
    """The plain single-RVE path: one request at a time, in arrival order."""
    t0 = time.perf_counter()
    lat, results = [], []
    for r in trace:
        now = time.perf_counter() - t0
        if now < r["t"]:
            time.sleep(r["t"] - now)
        with rve_create(r["n"], r["n_spheres"], r["f"], r["layer"], r["seed"]) as h:
            res = homogenize(h, r["k"], tol, precision=precision)
        lat.append(time.perf_counter() - t0 - r["t"])
        results.append(res)
        if len(results) % 100 == 0:
            print(f"[sequential] {len(results)} of {len(trace)} done at {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    makespan = time.perf_counter() - t0
    return {"mode": "sequential single-RVE", "precision": "fp32" if precision == 0 else "fp64",
            "requests": len(trace), "makespan_s": makespan, "solves_per_s": len(trace) / makespan,
            "p50_latency_s": _pct(lat, 50), "p99_latency_s": _pct(lat, 99)}, results


def tensor_err(K, Kref):
    return float(np.abs(K - Kref).max() / np.abs(Kref).max())


# --------------------------------------------------------------------------- sweep
def run_sweep256(layers=(0.05, 0.1, 0.2), contrasts=(1e2, 1e3, 1e4), n_spheres=100, f=0.40, seed=3,
                 tol=1e-6):
    """256^3, the same sphere centres for every (l, c); FP32 against FP64:
    iteration counts and per-entry tensor error."""
    rows = []
    for layer in layers:
        with rve_create(256, n_spheres, f, layer, seed) as h:
            for c in contrasts:
                k = (0.2, 0.3, 0.2 * c)
                r64 = homogenize(h, k, tol, precision=1)
                r32 = homogenize(h, k, tol, precision=0)
                rows.append({"layer": layer, "contrast": c, "iters_fp64": r64.iters.tolist(),
                             "iters_fp32": r32.iters.tolist(), "refine_iters_fp32": r32.refine_iters.tolist(),
                             "status_fp32": r32.lc_status.tolist(),
                             "ms_fp64": r64.solve_ms, "ms_fp32": r32.solve_ms,
                             "k_iso_fp64": float(np.trace(r64.K) / 3),
                             "err_fp32_vs_fp64": tensor_err(r32.K, r64.K)})
                print(json.dumps(rows[-1]), flush=True)
    return rows


def run_rate_sweep(requests=200, overload_rate=200.0, fractions=(0.5, 0.8), slots=16, check=20, seed=5):
    """Serving capacity and latency: the trace at an overload rate gives the
    capacity (served solves/s); the same request mix is then replayed at the
    given fractions of that capacity.  The first `check` requests of the
    overload run are also solved alone in FP64 and compared."""
    rows = []
    trace = serve_trace(requests, overload_rate, seed)
    out, served = run_serve(trace, slots=slots)
    cap = out["solves_per_s"]
    out.update({"rate": overload_rate, "fraction_of_capacity": overload_rate / cap})
    if check:
        errs = []
        for r, x in zip(trace[:check], served[:check]):
            with rve_create(r["n"], r["n_spheres"], r["f"], r["layer"], r["seed"]) as h:
                ref = homogenize(h, r["k"], 1e-6, precision=1)
            errs.append(tensor_err(x.K, ref.K))
        out["max_err_vs_fp64_first_%d" % check] = max(errs)
    rows.append(out)
    print(json.dumps(out), flush=True)
    for frac in fractions:
        rate = frac * cap
        tr = serve_trace(requests, rate, seed)
        o, _ = run_serve(tr, slots=slots)
        o.update({"rate": rate, "fraction_of_capacity": frac})
        rows.append(o)
        print(json.dumps(o), flush=True)
    return rows


def run_512(n_spheres=100, f=0.30, layer=0.2, seed=7, k=K_BENCH, tol=1e-6):
    """One 512^3 RVE on one GPU in both precisions (the paper needed a
    cluster for 512^3, Sec. 4): iterations, solve time, FP32 against FP64."""
    t0 = time.perf_counter()
    with rve_create(512, n_spheres, f, layer, seed) as h:
        setup = time.perf_counter() - t0
        r32 = homogenize(h, k, tol, precision=0)
        r64 = homogenize(h, k, tol, precision=1)
    out = {"n": 512, "n_spheres": n_spheres, "f": f, "layer": layer, "seed": seed, "setup_s": setup,
           "iters_fp32": r32.iters.tolist(), "refine_iters_fp32": r32.refine_iters.tolist(),
           "iters_fp64": r64.iters.tolist(),
           "status_fp32": r32.lc_status.tolist(), "ms_fp32": r32.solve_ms, "ms_fp64": r64.solve_ms,
           "voxel_iters_per_s_per_lc_fp32": 512 ** 3 * int(r32.iters.sum()) / (r32.solve_ms * 1e-3),
           "voxel_iters_per_s_per_lc_fp64": 512 ** 3 * int(r64.iters.sum()) / (r64.solve_ms * 1e-3),
           "k_iso_fp64": float(np.trace(r64.K) / 3), "err_fp32_vs_fp64": tensor_err(r32.K, r64.K)}
    print(json.dumps(out), flush=True)
    return out


# ---------------------------------------------------------------------- solve
def run_solve(n=256, n_spheres=100, f=0.40, layer=0.2, seed=3, k=K_BENCH, tol=1e-6, precision=0, repeat=2,
              max_iter=0, path_flags=0, fp32_refine=True):
    """Repeated solves of one seeded RVE (RSA spheres, Sec. 2): iterations,
    time and tensor of each, e.g. to profile one grid size (path_flags: the
    PATH_* measurement switches, e.g. 8 for one stream)."""
    rows = []
    with rve_create(n, n_spheres, f, layer, seed) as h:
        for _ in range(repeat):
            r = homogenize(h, k, tol, precision=precision, max_iter=max_iter, path_flags=path_flags,
                           fp32_refine=fp32_refine)
            row = {"n": n, "n_spheres": n_spheres, "f": f, "layer": layer, "seed": seed, "k": list(k),
                   "precision": "fp32" if precision == 0 else "fp64", "iters": r.iters.tolist(),
                   "refine_iters": r.refine_iters.tolist(),
                   "status": r.lc_status.tolist(), "ms": r.solve_ms,
                   "voxel_iters_per_s_per_lc": n ** 3 * int(r.iters.sum()) / (r.solve_ms * 1e-3),
                   "K": r.K.tolist()}
            rows.append(row)
            print(json.dumps(row), flush=True)
    return rows


# -------------------------------------------------------------------- schemes
def run_schemes(coatings=(1.0, 4.0, 20.0, 80.0, 400.0), n=128, n_spheres=50, f=0.30, layer=0.2, seed=2,
                tol=1e-6, precision=1, max_iter=20000):
    """Iterations against contrast for the schemes Sec. 3 names (accelerated,
    augmented Lagrangian, polarization at relaxation 1.5, dual, basic) on
    one RVE: matrix 1, inclusion 0.2, coating from 1 to 400 (contrast 5 to
    2000, the range of Sec. 3), with the contraction bound of each scheme
    and the iterations it predicts."""
    rows = []
    alpha = 1.5
    with rve_create(n, n_spheres, f, layer, seed) as h:
        for kc in coatings:
            k = (1.0, 0.2, kc)
            c = max(k) / min(k)
            rho = (math.sqrt(c) - 1) / (math.sqrt(c) + 1)
            bounds = {"accelerated": rho, "augmented_lagrangian": 0.5 * (1 + rho),
                      "polarization": abs(1 - alpha / 2) + alpha / 2 * rho,
                      "dual": (c - 1) / (c + 1), "basic": (c - 1) / (c + 1)}
            ref = None
            for sch in ("accelerated", "augmented_lagrangian", "polarization", "dual", "basic"):
                r = homogenize(h, k, tol, precision=precision, scheme=sch, max_iter=max_iter,
                               alpha=alpha if sch == "polarization" else 0.0)
                if ref is None:
                    ref = r
                row = {"contrast": c, "scheme": sch, "iters": r.iters.tolist(),
                       "status": r.lc_status.tolist(), "ms": r.solve_ms,
                       "ms_per_iter": r.solve_ms / max(1, int(r.iters.max())),
                       "rate_bound": bounds[sch],
                       "iters_bound": math.ceil(math.log(tol) / math.log(bounds[sch])),
                       "k_iso": float(np.trace(r.K) / 3), "err_vs_accelerated": tensor_err(r.K, ref.K)}
                rows.append(row)
                print(json.dumps(row), flush=True)
    return rows


# --------------------------------------------------------------------- fibres
def run_fibers(layers=(0.02, 0.05, 0.1, 0.2, 0.4, 0.8), n=128, n_fibers=40, f=0.40, seeds=(1, 2, 3),
               k=(1.0, 0.2, 400.0), tol=1e-6, precision=0):
    """Aligned coated fibres along z (the cylindrical inclusions Sec. 6 names
    next), the paper's conductivities: transverse and axial conductivity
    against the coating layer l, over a few seeded realizations."""
    rows = []
    for layer in layers:
        for seed in seeds:
            ph, _, _ = generate_fibers(n, n_fibers, f, layer, seed)
            with rve_create_from_phases(ph) as h:
                r = homogenize(h, k, tol, precision=precision)
            kv = np.asarray(k)[ph]
            row = {"layer": layer, "seed": seed, "iters": r.iters.tolist(), "status": r.lc_status.tolist(),
                   "ms": r.solve_ms, "k_transverse": float(0.5 * (r.K[0, 0] + r.K[1, 1])),
                   "k_axial": float(r.K[2, 2]), "k_mean": float(kv.mean()),
                   "k_harmonic": float(1.0 / (1.0 / kv).mean())}
            rows.append(row)
            print(json.dumps(row), flush=True)
    return rows


# -------------------------------------------------------------------- elastic
def run_elastic(sizes=((128, 0), (128, 1), (256, 0), (256, 1), (512, 0), (512, 1)),
                moduli=((4.0, 1.5), (40.0, 30.0), (150.0, 100.0)),
                n_spheres=50, f=0.30, layer=0.2, seed=2, tol=1e-6, reps=3):
    """The elastic case (Sec. 6) on coated-sphere RVEs: six load cases,
    iterations, solve time, voxel-iterations/s per load case, the
    algorithmic HBM rate of the path (bytes per iteration of the passes
    times iterations over the solve time) and the isotropic moduli of
    C_hom."""
    from . import homogenize_elastic
    rows = []
    for n, prec in sizes:
        with rve_create(n, n_spheres, f, layer, seed) as h:
            r = homogenize_elastic(h, moduli, tol, precision=prec)
            best = r
            for _ in range(reps if n <= 256 else 1):
                g = homogenize_elastic(h, moduli, tol, precision=prec)
                if g.solve_ms < best.solve_ms:
                    best = g
        M = n ** 3
        b = 4 if prec == 0 else 8
        # fused: whole planes (not FP32 96^3) and the FP32 256^3 split planes
        fused = not (n == 96 and prec == 0) and (n <= 128 or (prec == 0 and n <= 256))
        five = (prec == 1 and n >= 256) or n >= 512
        # per iteration of all six load cases (the phase image read once per
        # pass): z pass 2 C; fused plane pass 2 C + 2 * 36 M b + M; separate
        # plane passes 2 C + 3 * 36 M b + 2 M; the five-pass form adds the two
        # column passes, 4 C
        C = 36 * n * n * (n // 2 + 1) * 2 * b
        per_it = 2 * C + (2 * C + 72 * M * b + M if fused else 2 * C + 108 * M * b + 2 * M) + (4 * C if five else 0)
        its = float(best.iters.mean())
        Cm = best.C_basis
        row = {"n": n, "precision": "fp32" if prec == 0 else "fp64", "iters": best.iters.tolist(),
               "status": best.lc_status.tolist(), "ms": best.solve_ms,
               "voxel_iters_per_s_per_lc": M * int(best.iters.sum()) / (best.solve_ms * 1e-3),
               "algorithmic_GBps": per_it * its / (best.solve_ms * 1e-3) / 1e9,
               "kappa_eff": float(Cm[0, 0] / 3.0), "mu_eff": float(np.trace(Cm[1:, 1:]) / 10.0),
               "max_asym": float(np.abs(best.C - best.C.T).max() / np.abs(best.C).max())}
        rows.append(row)
        print(json.dumps(row), flush=True)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("batch")
    b.add_argument("--count", type=int, default=64)
    b.add_argument("--precision", type=int, default=0)
    s = sub.add_parser("serve")
    s.add_argument("--requests", type=int, default=2000)
    s.add_argument("--rate", type=float, default=200.0)
    s.add_argument("--slots", type=int, default=16)
    s.add_argument("--baseline", type=int, default=0, help="also run the sequential FP64 path")
    sub.add_parser("sweep256")
    sub.add_parser("run512")
    so = sub.add_parser("solve")
    so.add_argument("--n", type=int, default=256)
    so.add_argument("--spheres", type=int, default=100)
    so.add_argument("--f", type=float, default=0.40)
    so.add_argument("--layer", type=float, default=0.2)
    so.add_argument("--seed", type=int, default=3)
    so.add_argument("--precision", type=int, default=0)
    so.add_argument("--repeat", type=int, default=2)
    so.add_argument("--kc", type=float, default=K_BENCH[2], help="coating conductivity (matrix 0.2, inclusion 0.3)")
    so.add_argument("--tol", type=float, default=1e-6)
    so.add_argument("--max-iter", type=int, default=0)
    so.add_argument("--path-flags", type=int, default=0)
    so.add_argument("--no-refine", action="store_true")
    sub.add_parser("fibers")
    el = sub.add_parser("elastic")
    el.add_argument("--n", type=int, nargs="*", default=None, help="grid sizes (default 128, 256, 512)")
    el.add_argument("--precision", type=int, nargs="*", default=None, help="precisions (default 0 and 1)")
    el.add_argument("--reps", type=int, default=3)
    sc = sub.add_parser("schemes")
    sc.add_argument("--precision", type=int, default=1)
    rs = sub.add_parser("rates")
    rs.add_argument("--requests", type=int, default=200)
    rs.add_argument("--rate", type=float, default=200.0)
    a = ap.parse_args(argv)
    if a.cmd == "batch":
        print(json.dumps(run_batch(a.count, precision=a.precision)), flush=True)
    elif a.cmd == "serve":
        tr = serve_trace(a.requests, a.rate)
        out, served = run_serve(tr, slots=a.slots)
        print(json.dumps(out), flush=True)
        if a.baseline:
            seq, ref = run_sequential(tr, precision=1)
            seq["max_err_served_fp32_vs_fp64"] = max(tensor_err(x.K, y.K) for x, y in zip(served, ref))
            print(json.dumps(seq), flush=True)
    elif a.cmd == "run512":
        run_512()
    elif a.cmd == "solve":
        run_solve(a.n, a.spheres, a.f, a.layer, a.seed, k=(K_BENCH[0], K_BENCH[1], a.kc), tol=a.tol,
                  precision=a.precision, repeat=a.repeat, max_iter=a.max_iter, path_flags=a.path_flags,
                  fp32_refine=not a.no_refine)
    elif a.cmd == "fibers":
        run_fibers()
    elif a.cmd == "elastic":
        if a.n or a.precision:
            sizes = [(n, p) for n in (a.n or [128, 256, 512]) for p in (a.precision if a.precision else [0, 1])]
            run_elastic(sizes=sizes, reps=a.reps)
        else:
            run_elastic(reps=a.reps)
    elif a.cmd == "schemes":
        run_schemes(precision=a.precision)
    elif a.cmd == "rates":
        run_rate_sweep(a.requests, a.rate)
    else:
        run_sweep256()


if __name__ == "__main__":
    sys.exit(main())
