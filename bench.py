#!/usr/bin/env python3
"""Throughput of the accelerated FFT homogenization solve on one MI355X.

Workload (one "step" = one full solve, all three unit load cases, until every
load case has eps_comp < 1e-6): a 128^3 periodic RVE with 50 RSA spheres at
volume fraction 0.30 (coating included), coating layer l = 0.2, seed 2;
conductivities matrix 0.2, inclusion 0.3, coating 400; FP32 FFT/update with
FP64 reductions.  The phase image is generated and uploaded before the timed
region; the timed region holds exactly --steps solves.

metric: voxel-iterations per second per load case, i.e. sum over load cases
of N^3 * iterations, divided by the wall time of the solves.

Also reported: the roofline of the dominant kernel (algorithmic bytes per
launch over its HIP-event-timed launch duration, against 8 TB/s, taken in the
first timed solve, which runs on a single stream; the others run the three
load cases as concurrent chains, and the whole path's bytes over the wall
time are given beside it), and the FP64 CPU oracle timed on a bounded sample
of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-iters/s per load case; RVE solves/s + p50/p99 at 1e-4 tensor err"
HBM_PEAK_GBS = 8000.0
WORKLOAD = {"workload": "rve128_50sph_f0.30_l0.20_seed2", "n": 128, "n_spheres": 50,
            "volume_fraction": 0.30, "layer": 0.2, "seed": 2, "k_phases": [0.2, 0.3, 400.0],
            "tol": 1e-6, "precision": "fp32 fft/update, fp64 reductions",
            "load_cases": 3}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rve128_fp32.txt")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1504_07499_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


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
    if vals.get("source_hash") != kernel_source_hash():
        return None
    key = f"{kernel}_hbm_bytes_per_launch"
    return float(vals[key]) if key in vals else None


def cpu_baseline(phases, k, sample_iters: int):
    import oracle

    t0 = time.perf_counter()
    r = oracle.homogenize(phases, k, tol=0.0, max_iter=sample_iters, lc_mask=1)
    dt = time.perf_counter() - t0
    m = phases.size
    return {"value": m * int(r.iters[0]) / dt, "unit": "voxel-iters/s per load case",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{sample_iters} iterations of load case e_1 on the same 128^3 RVE "
                      f"(FP64, own FFT, OpenMP), {dt:.1f} s"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-iters", type=int, default=30)
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
    rve = rh.rve_create(n, w["n_spheres"], w["volume_fraction"], w["layer"], w["seed"])
    for _ in range(args.warmup):
        rh.homogenize(rve, k, w["tol"], precision=0)
    timing = not args.no_timing
    mask = 0
    if timing:
        # one solve outside the timed region, on a single stream with every
        # kernel timed: picks the dominant kernel and gives the algorithmic
        # bytes per load-case iteration of the whole path
        os.environ["RVEHOM_CHAINS"] = "0"
        try:
            probe = rh.homogenize(rve, k, w["tol"], precision=0, timing=15)
        finally:
            os.environ.pop("RVEHOM_CHAINS", None)
        kt = rh.rve_get_kernel_times(rve)
        names = list(kt)
        cand = [kk for kk in names if kk != "reduce" and kt[kk]["launches"] > 0]
        dom = max(cand, key=lambda kk: kt[kk]["total_ms"])
        mask = 1 << names.index(dom)
        bytes_per_lc_iter = sum(kt[kk]["total_bytes"] for kk in names) / max(int(probe.iters.sum()), 1)
    totals = {}
    step_iters, step_ms, results = [], [], []
    t0 = time.perf_counter()
    for step in range(args.steps):
        # the first timed solve runs on a single stream with events around the
        # dominant kernel (its launches then cover all three load cases and do
        # not overlap other kernels, so event time is kernel time); the others
        # run as three concurrent load-case chains without events
        measure = timing and step == 0
        if measure:
            os.environ["RVEHOM_CHAINS"] = "0"
        try:
            res = rh.homogenize(rve, k, w["tol"], precision=0, timing=mask if measure else 0)
        finally:
            if measure:
                os.environ.pop("RVEHOM_CHAINS", None)
        results.append(res)
        if measure:
            for name, v in rh.rve_get_kernel_times(rve).items():
                t = totals.setdefault(name, {"total_ms": 0.0, "launches": 0, "total_bytes": 0.0})
                for key in t:
                    t[key] += v[key]
    wall = time.perf_counter() - t0
    for res in results:
        step_iters.append([int(i) for i in res.iters])
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
        path_bytes = bytes_per_lc_iter * sum(sum(it) for it in step_iters)
        path_achieved = path_bytes / wall / 1e9
        copy_gbs = copy_bandwidth_gbs()
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
                    "kernel": dom, "avg_launch_ms": round(avg_ms, 5), "launches": d["launches"],
                    "algorithmic_bytes_per_launch": bytes_per_launch,
                    "measured_in": "the first timed solve (single stream, launches of all three load cases)",
                    # the whole path: every kernel's algorithmic bytes over the
                    # wall time of all timed solves (three concurrent chains)
                    "path": {"algorithmic_bytes_per_load_case_iteration": bytes_per_lc_iter,
                             "achieved": round(path_achieved, 1),
                             "frac": round(path_achieved / HBM_PEAK_GBS, 4)},
                    # a plain device-to-device copy, timed after the solves
                    "copy": {"achieved": round(copy_gbs, 1), "frac": round(copy_gbs / HBM_PEAK_GBS, 4),
                             "kernel_frac_of_copy": round(achieved / copy_gbs, 4)},
                    "per_kernel_avg_ms_probe": {
                        kk: round(kt[kk]["total_ms"] / max(kt[kk]["launches"], 1), 5)
                        for kk in names if kt[kk]["launches"]}}

    err = None
    refs_path = os.path.join(ROOT, "tests", "golden", "oracle_refs.json")
    if os.path.exists(refs_path):
        with open(refs_path) as f:
            refs = json.load(f)
        ref = refs.get(w["workload"])
        if ref:
            Kr = np.array(ref["K"])
            err = float(np.abs(last.K - Kr).max() / np.abs(Kr).max())

    cpu = None
    if not args.no_cpu_baseline:
        from paper_1504_07499_amd import geom

        ph, _, _ = geom.generate(n, w["n_spheres"], w["volume_fraction"], w["layer"], w["seed"])
        cpu = cpu_baseline(ph, k, args.cpu_iters)

    line = {
        "metric": METRIC, "value": value, "unit": "voxel-iters/s per load case", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded RSA RVE)", "config": w,
        "iters_per_load_case": step_iters[-1], "solves_per_s": args.steps / wall,
        "device_solve_ms_median": float(np.median(step_ms)),
        "tensor_err_vs_oracle": err, "lc_status": [int(s) for s in last.lc_status],
        "roofline": roofline, "cpu_baseline": cpu,
    }
    rve.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
