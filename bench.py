#!/usr/bin/env python3
"""Throughput of the accelerated FFT homogenization solve on one MI355X.

Workload (one "step" = one full solve, all three unit load cases, until every
load case has eps_comp < 1e-6): a 256^3 periodic RVE with 100 spheres at
volume fraction 0.40 (coating included; RSA, then the Monte Carlo fallback
of the generator), coating layer l = 0.1, seed 3; conductivities matrix 0.2,
inclusion 0.3, coating 200 (contrast 1e3); FP32 FFT/update with FP64
reductions, and an FP64 continuation of load cases the FP32 rounding floor
stops above tol.  The phase image is generated and uploaded before the timed
region; the timed region holds exactly --steps solves.

metric: voxel-iterations per second per load case, i.e. sum over load cases
of N^3 * iterations, divided by the wall time of the solves.

Also reported: the roofline of the dominant kernel (algorithmic bytes per
launch over its HIP-event-timed launch duration, against 8 TB/s, taken in the
first timed solve, which runs on a single stream; the others run the three
load cases as concurrent chains, and the whole path's bytes over the wall
time are given beside it); the 128^3 benchmark RVE as a secondary figure; a
bounded serving leg (a Poisson trace of mixed requests through the
continuous-batching server: solves/s, p50 and p99 latency, tensor error
against the FP64 single-RVE path); and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1504_07499_amd._build import kernel_source_hash  # noqa: E402

METRIC = "voxel-iters/s per load case; RVE solves/s + p50/p99 at 1e-4 tensor err"
HBM_PEAK_GBS = 8000.0
PRECISION = "fp32 fft/update, fp64 reductions; fp64 continuation past the fp32 rounding floor"
# 256^3, 100 spheres at f = 0.40, l = 0.1, contrast 1e3 (k_coating = 0.2 c), seed 3
WORKLOAD = {"workload": "rve256_100sph_f0.40_l0.10_c1e3_seed3", "n": 256, "n_spheres": 100,
            "volume_fraction": 0.40, "layer": 0.1, "seed": 3, "k_phases": [0.2, 0.3, 200.0],
            "contrast": 1000.0, "tol": 1e-6, "precision": PRECISION, "load_cases": 3}
# the 128^3 RVE (50 spheres, f = 0.30, l = 0.2, seed 2, contrast 2000), a secondary figure
SECONDARY = {"workload": "rve128_50sph_f0.30_l0.20_seed2", "n": 128, "n_spheres": 50,
             "volume_fraction": 0.30, "layer": 0.2, "seed": 2, "k_phases": [0.2, 0.3, 400.0],
             "contrast": 2000.0, "tol": 1e-6, "precision": PRECISION, "load_cases": 3}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rve256_fp32.txt")


def measured_traffic(kernel: str, launches_bytes: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash():  # counters of other kernel sources
        return None
    key = f"{kernel}_hbm_bytes_per_launch"
    return float(vals[key]) if key in vals else None


def cpu_baseline(phases, k, sample_iters: int, single_iters: int):
    """The FP64 oracle on the host: sample_iters iterations of load case e_1
    on all host threads, and single_iters on one thread."""
    import oracle

    m = phases.size
    cores = oracle.threads()
    t0 = time.perf_counter()
    r = oracle.homogenize(phases, k, tol=0.0, max_iter=sample_iters, lc_mask=1)
    dt = time.perf_counter() - t0
    out = {"value": m * int(r.iters[0]) / dt, "unit": "voxel-iters/s per load case",
           "cores": cores, "kind": "oracle",
           "sample": f"{sample_iters} iterations of load case e_1 on the same {phases.shape[0]}^3 "
                     f"RVE (FP64, own FFT, OpenMP), {dt:.1f} s"}
    if single_iters > 0:
        oracle.set_threads(1)
        try:
            t0 = time.perf_counter()
            r1 = oracle.homogenize(phases, k, tol=0.0, max_iter=single_iters, lc_mask=1)
            d1 = time.perf_counter() - t0
        finally:
            oracle.set_threads(cores)
        out["single_thread"] = {"value": m * int(r1.iters[0]) / d1, "cores": 1,
                                "sample": f"{single_iters} iterations of load case e_1, {d1:.1f} s"}
    return out


def calibrate_copy(mib: int = 512, reps: int = 4) -> None:
    """Device-to-device copies of a known size (the runtime's blit kernel),
    run under rocprofv3 --pmc to scale FETCH_SIZE / WRITE_SIZE readings."""
    import ctypes

    import paper_1504_07499_amd as rh

    rh.rve_supported_n(0)  # loads librvehom.so and with it the HIP runtime
    hip = ctypes.CDLL("libamdhip64.so.7")
    n = mib << 20
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(a), ctypes.c_size_t(n)) == 0
    assert hip.hipMalloc(ctypes.byref(b), ctypes.c_size_t(n)) == 0
    for _ in range(reps):
        assert hip.hipMemcpy(b, a, ctypes.c_size_t(n), 3) == 0  # device to device
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(a)
    hip.hipFree(b)
    print(json.dumps({"copy_bytes": n, "reps": reps}), flush=True)


def copy_bandwidth_gbs(mib: int = 1024, reps: int = 5) -> float:
    """Achieved HBM bandwidth of a plain device-to-device copy (the runtime's
    blit kernel; buffers four times the 256 MB last-level cache), read plus
    written bytes over HIP-event time: the practical ceiling next to the
    nominal peak."""
    import ctypes

    hip = ctypes.CDLL("libamdhip64.so.7")
    n = mib << 20
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    e0, e1 = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(a), ctypes.c_size_t(n)) == 0
    assert hip.hipMalloc(ctypes.byref(b), ctypes.c_size_t(n)) == 0
    assert hip.hipEventCreate(ctypes.byref(e0)) == 0 and hip.hipEventCreate(ctypes.byref(e1)) == 0
    assert hip.hipMemcpyAsync(b, a, ctypes.c_size_t(n), 3, None) == 0  # warm-up
    assert hip.hipEventRecord(e0, None) == 0
    for _ in range(reps):
        assert hip.hipMemcpyAsync(b, a, ctypes.c_size_t(n), 3, None) == 0
    assert hip.hipEventRecord(e1, None) == 0
    assert hip.hipEventSynchronize(e1) == 0
    ms = ctypes.c_float()
    assert hip.hipEventElapsedTime(ctypes.byref(ms), e0, e1) == 0
    hip.hipEventDestroy(e0)
    hip.hipEventDestroy(e1)
    hip.hipFree(a)
    hip.hipFree(b)
    return 2.0 * n * reps / (ms.value * 1e-3) / 1e9


def oracle_ref(name):
    path = os.path.join(ROOT, "tests", "golden", "oracle_refs.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f).get(name)


def tensor_err(K, Kref):
    import numpy as np

    Kref = np.asarray(Kref)
    return float(np.abs(np.asarray(K) - Kref).max() / np.abs(Kref).max())


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def secondary_leg(rh, steps=5):
    """The 128^3 RVE: warm-up, then `steps` solves (three concurrent chains)."""
    import numpy as np

    w = SECONDARY
    k = np.array(w["k_phases"])
    with rh.rve_create(w["n"], w["n_spheres"], w["volume_fraction"], w["layer"], w["seed"]) as r:
        rh.homogenize(r, k, w["tol"], precision=0)
        t0 = time.perf_counter()
        res = [rh.homogenize(r, k, w["tol"], precision=0) for _ in range(steps)]
        wall = time.perf_counter() - t0
    last = res[-1]
    vox = sum(w["n"] ** 3 * int(x.iters.sum()) for x in res)
    ref = oracle_ref(w["workload"])
    return {"workload": w["workload"], "value": vox / wall, "unit": "voxel-iters/s per load case",
            "ms_per_solve": 1e3 * wall / steps, "iters_per_load_case": [int(i) for i in last.iters],
            "fp64_refine_iters": [int(i) for i in last.refine_iters],
            "lc_status": [int(s) for s in last.lc_status],
            "tensor_err_vs_oracle": tensor_err(last.K, ref["K"]) if ref else None}


def serving_leg(rh, requests, rate, budget_gib=48, slots=16):
    """A Poisson trace of mixed requests (N uniform on {32, 64, 128, 256},
    10-100 spheres, contrast log-uniform in [10, 1e4]) through the
    continuous-batching server; served tensors of the N <= 128 requests
    checked against the FP64 single-RVE path."""
    from paper_1504_07499_amd import workloads

    trace = workloads.serve_trace(requests=requests, rate=rate, seed=5)
    out, results = workloads.run_serve(trace, precision=0, budget_bytes=budget_gib << 30, slots=slots)
    errs = []
    for r, res in zip(trace, results):
        if r["n"] <= 128:
            with rh.rve_create(r["n"], r["n_spheres"], r["f"], r["layer"], r["seed"]) as h:
                ref = rh.homogenize(h, r["k"], 1e-6, precision=1)
            errs.append(tensor_err(res.K, ref.K))
    out["trace"] = (f"{requests} requests, Poisson rate {rate}/s (trace seed 5), N uniform on "
                    "{32, 64, 128, 256}, contrast log-uniform in [10, 1e4]")
    out["tensor_err_vs_fp64_max"] = max(errs) if errs else None
    out["tensor_err_checked"] = len(errs)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-iters", type=int, default=10)
    ap.add_argument("--cpu-iters-single", type=int, default=1,
                    help="oracle iterations timed on one host thread (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=100,
                    help="requests of the serving leg (0 = skip it)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--no-secondary", action="store_true", help="skip the 128^3 leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="skip the per-launch HIP events (no roofline)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run device-to-device copies of known size (counter scaling)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solve of one RVE runs on one device and "
              "independent RVEs need no communication; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import paper_1504_07499_amd as rh

    w = WORKLOAD
    n = w["n"]
    k = np.array(w["k_phases"])
    single = rh.PATH_NO_CHAINS
    progress(f"generating {w['workload']}")
    rve = rh.rve_create(n, w["n_spheres"], w["volume_fraction"], w["layer"], w["seed"])
    for _ in range(args.warmup):
        rh.homogenize(rve, k, w["tol"], precision=0)
    progress("warm-up done")
    timing = not args.no_timing
    mask = 0
    if timing:
        # one solve outside the timed region, on a single stream with every
        # kernel timed: picks the dominant kernel and gives the algorithmic
        # bytes per load-case iteration of the FP32 path
        probe = rh.homogenize(rve, k, w["tol"], precision=0, timing=15, path_flags=single)
        kt = rh.rve_get_kernel_times(rve)
        names = list(kt)
        cand = [kk for kk in names if kk != "reduce" and kt[kk]["launches"] > 0]
        dom = max(cand, key=lambda kk: kt[kk]["total_ms"])
        mask = 1 << names.index(dom)
        fp32_iters = int(probe.iters.sum() - probe.refine_iters.sum())
        bytes_per_lc_iter = sum(kt[kk]["total_bytes"] for kk in names) / max(fp32_iters, 1)
        progress(f"probe solve: dominant kernel {dom}")
    totals = {}
    step_iters, step_refine, step_ms, results = [], [], [], []
    t0 = time.perf_counter()
    for step in range(args.steps):
        # the first timed solve runs on a single stream with events around the
        # dominant kernel (its launches then cover all three load cases and do
        # not overlap other kernels, so event time is kernel time); the others
        # run as three concurrent load-case chains without events
        measure = timing and step == 0
        res = rh.homogenize(rve, k, w["tol"], precision=0, timing=mask if measure else 0,
                            path_flags=single if measure else 0)
        results.append(res)
        if measure:
            for name, v in rh.rve_get_kernel_times(rve).items():
                t = totals.setdefault(name, {"total_ms": 0.0, "launches": 0, "total_bytes": 0.0})
                for key in t:
                    t[key] += v[key]
    wall = time.perf_counter() - t0
    progress(f"{args.steps} timed solves in {wall:.2f} s")
    for res in results:
        step_iters.append([int(i) for i in res.iters])
        step_refine.append([int(i) for i in res.refine_iters])
        step_ms.append(res.solve_ms)
    m = n ** 3
    voxel_iters = sum(m * sum(it) for it in step_iters)
    value = voxel_iters / wall
    last = results[-1]

    roofline = None
    if timing and totals and totals.get(dom, {}).get("launches"):
        d = totals[dom]
        avg_ms = d["total_ms"] / d["launches"]
        bytes_per_launch = d["total_bytes"] / d["launches"]
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        tr = measured_traffic(dom, bytes_per_launch)
        fp32_total = sum(sum(it) - sum(rf) for it, rf in zip(step_iters, step_refine))
        path_bytes = bytes_per_lc_iter * fp32_total
        path_achieved = path_bytes / wall / 1e9
        copy_gbs = copy_bandwidth_gbs()
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
                    "kernel": dom, "avg_launch_ms": round(avg_ms, 5), "launches": d["launches"],
                    "algorithmic_bytes_per_launch": bytes_per_launch,
                    "measured_in": "the first timed solve (single stream, launches of all three load cases)",
                    # the whole path: the FP32 kernels' algorithmic bytes over
                    # the wall time of all timed solves (three concurrent
                    # chains; the FP64 continuation's time included, its bytes not)
                    "path": {"algorithmic_bytes_per_load_case_iteration": bytes_per_lc_iter,
                             "achieved": round(path_achieved, 1),
                             "frac": round(path_achieved / HBM_PEAK_GBS, 4)},
                    # a plain device-to-device copy, timed after the solves
                    "copy": {"achieved": round(copy_gbs, 1), "frac": round(copy_gbs / HBM_PEAK_GBS, 4),
                             "kernel_frac_of_copy": round(achieved / copy_gbs, 4)},
                    "per_kernel_avg_ms_probe": {
                        kk: round(kt[kk]["total_ms"] / max(kt[kk]["launches"], 1), 5)
                        for kk in names if kt[kk]["launches"]}}
    rve.close()

    ref = oracle_ref(w["workload"])
    err = tensor_err(last.K, ref["K"]) if ref else None

    secondary = None if args.no_secondary else secondary_leg(rh)
    progress("secondary leg done")
    serving = None
    if args.serve_requests > 0:
        serving = serving_leg(rh, args.serve_requests, args.serve_rate)
        progress("serving leg done")

    cpu = None
    if not args.no_cpu_baseline:
        from paper_1504_07499_amd import geom

        ph, _, _ = geom.generate(n, w["n_spheres"], w["volume_fraction"], w["layer"], w["seed"])
        cpu = cpu_baseline(ph, k, args.cpu_iters, args.cpu_iters_single)
        progress("cpu baseline done")

    line = {
        "metric": METRIC, "value": value, "unit": "voxel-iters/s per load case", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded RSA RVE)", "config": w,
        "iters_per_load_case": step_iters[-1], "fp64_refine_iters": step_refine[-1],
        "solves_per_s": args.steps / wall,
        "device_solve_ms_median": float(np.median(step_ms)),
        "tensor_err_vs_oracle": err, "lc_status": [int(s) for s in last.lc_status],
        "roofline": roofline, "secondary": secondary, "serving": serving, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
