"""Per-kernel summaries of rocprofv3 result databases for the solver's kernels.

rocprofv3 (ROCm 7) writes its results as an SQLite database
(``<dir>/<name>_results.db``).  This module reads the kernel trace
(``kernels`` view) and the counter collections (``counters_collection``
view) of such databases and prints one table per run:

* trace: calls, average duration of the launches that did the whole pass
  (early exits after convergence left out and counted), grid, workgroup,
  LDS bytes and VGPRs per kernel, and -- for the solver's passes in the
  trace's precision
  (--real-bytes) -- the algorithmic HBM bytes per launch (all three load
  cases: each pass reads and writes its fields once, the phase image once)
  and the rate they imply;
* counters: the average per dispatch of every collected counter, plus, for
  FETCH_SIZE / WRITE_SIZE, the HBM bytes per launch scaled by the reading of
  a device-to-device copy of known size (``bench.py --calibrate-copy``), and
  for the SQ counters the derived VALU busy, LDS share and occupancy.

Command line:
  python -m paper_1504_07499_amd.profile_summary trace DB --n 256 --real-bytes 4
  python -m paper_1504_07499_amd.profile_summary traffic FETCH_DB WRITE_DB COPY_FETCH_DB COPY_WRITE_DB --n 256 [--source-hash]
  python -m paper_1504_07499_amd.profile_summary sq DB [DB ...]
"""
from __future__ import annotations

import argparse
import collections
import sqlite3
import sys

CUS = 256  # compute units of an MI355X
SIMDS = 4 * CUS
XCDS = 8


def short_name(name: str) -> str:
    """Kernel name without the argument list."""
    depth, out = 0, []
    for ch in name:
        if ch == "(" and depth == 0:
            break
        out.append(ch)
        depth += ch == "<"
        depth -= ch == ">"
    return "".join(out).replace("void ", "").replace("rvehom::", "")


def algorithmic_bytes(name: str, n: int, rb: int) -> float | None:
    """HBM bytes per launch of a solver pass over all load cases: for the
    conductivity case (9 channels) e is 9 n^3 reals, the half spectrum
    9 n^2 (n/2 + 1) complex values, the phase image n^3 bytes; the elastic
    case (template argument NC = 6, and k_zgreen_el) has 36 channels.  rb:
    bytes per real of FP32 kernels (FP64 kernels, first template argument
    double, take 8).  The plane passes, the z pass and the five-pass form's
    passes (k_fwd_rows, k_cols, k_inv_rows)."""
    s = short_name(name)
    args = s.split("<", 1)[1].rstrip(">").split(", ") if "<" in s else []
    if args and args[0] == "double":
        rb = 8
    # components per load case: <T, N, S, NT, FWD, UPD, NC, ...> for
    # k_inv_plane, <T, N, S, NT, PHI, NC, ...> for k_fwd_plane, the last
    # argument of the five-pass kernels
    nc = 3
    if s.startswith("k_zgreen_el"):
        nc = 6
    elif s.startswith("k_inv_plane") and len(args) > 6:
        nc = int(args[6])
    elif s.startswith("k_fwd_plane") and len(args) > 5:
        nc = int(args[5])
    elif s.startswith(("k_fwd_rows", "k_cols", "k_inv_rows")) and args:
        nc = int(args[-1])
    ch = nc * nc
    m = n ** 3
    field = ch * m * rb
    spec = ch * n * n * (n // 2 + 1) * 2 * rb
    phase = float(m)
    if s.startswith("k_inv_plane"):
        fused = len(args) > 4 and args[4] == "true"  # <T, N, S, NT, FWD, ...>
        return 2 * spec + 2 * field + phase if fused else spec + 2 * field + phase
    if s.startswith("k_fwd_plane"):
        return field + spec + phase
    if s.startswith("k_zgreen"):
        return 2 * spec
    # the five-pass form: rows forward e -> spectrum, a column pass in
    # place, rows inverse
    if s.startswith("k_fwd_rows"):
        return field + spec + phase
    if s.startswith("k_cols"):
        return 2 * spec
    if s.startswith("k_inv_rows"):
        return spec + 2 * field + phase
    return None


def _connect(db):
    return sqlite3.connect(f"file:{db}?mode=ro", uri=True)


def full_launches(durations):
    """The launches that did the pass's work: the solver launches whole
    batches of iterations, and a launch after every load case has converged
    exits at once (as does one whose load cases are partly frozen, with
    less work); those under 0.8 of the median duration are left out of the
    average."""
    v = sorted(durations)
    med = v[len(v) // 2]
    return [d for d in durations if d >= 0.8 * med]


def trace(db: str, n: int, rb: int) -> str:
    """calls: all launches; short: those left out of avg_us (full_launches);
    avg_us and the rate: the launches that did the whole pass."""
    con = _connect(db)
    groups = collections.OrderedDict()
    for name, dur, grid, wg, lds, vgpr in con.execute(
            "select name, duration, grid_x, workgroup_x, lds_size, vgpr_count from kernels"):
        g = groups.setdefault((name, grid), {"d": [], "wg": wg, "lds": lds, "vgpr": vgpr})
        g["d"].append(dur)
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]["d"]))
    out = [f"{'kernel':58s} {'grid':>8s} {'wg':>5s} {'lds':>7s} {'vgpr':>5s} {'calls':>6s} {'short':>5s} "
           f"{'avg_us':>9s} {'alg_MB':>9s} {'TB/s':>6s} {'frac8':>6s}"]
    for (name, grid), g in rows:
        wg, lds, vgpr = g["wg"], g["lds"], g["vgpr"]
        full = full_launches(g["d"])
        avg = sum(full) / len(full)
        ab = algorithmic_bytes(name, n, rb)
        # kernels of the other precision (an FP64 continuation in an FP32
        # trace runs on the load cases still active): no byte count
        s_args = short_name(name).split("<", 1)[1].split(", ") if "<" in short_name(name) else []
        if s_args and s_args[0] in ("float", "double") and (8 if s_args[0] == "double" else 4) != rb:
            ab = None
        us = avg / 1e3
        rate = ab / (avg * 1e-9) / 1e12 if ab else None
        out.append(f"{short_name(name)[:58]:58s} {grid // max(wg, 1):8d} {wg:5d} {lds:7d} {vgpr:5d} "
                   f"{len(g['d']):6d} {len(g['d']) - len(full):5d} "
                   f"{us:9.1f} " + (f"{ab / 1e6:9.1f} {rate:6.2f} {rate / 8.0:6.3f}" if ab else
                                    f"{'':>9s} {'':>6s} {'':>6s}"))
    return "\n".join(out)


def counters(db: str) -> dict:
    """{kernel name: {counter: average value per dispatch}}."""
    con = _connect(db)
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for name, ctr, val in con.execute("select kernel_name, counter_name, value from counters_collection"):
        acc[name][ctr].append(val)
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}


def copy_factor(db: str, ctr: str, copy_bytes: float) -> float:
    """Bytes per counter unit from the copy kernel's reading (FETCH_SIZE and
    WRITE_SIZE are in KiB; the copy reads and writes copy_bytes)."""
    c = counters(db)
    vals = [v[ctr] for k, v in c.items() if "copyBuffer" in k and ctr in v]
    big = max(vals)
    return copy_bytes / (big * 1024.0)


def timing_name(name: str) -> str | None:
    """The pass name under which the library's per-launch timing reports a
    kernel (rve_get_kernel_times), for the three passes of an iteration."""
    s = short_name(name)
    args = s.split("<", 1)[1].rstrip(">").split(", ") if "<" in s else []
    if s.startswith("k_inv_plane"):
        return "inv_fwd_plane" if len(args) > 4 and args[4] == "true" else "inv_plane"
    if s.startswith("k_fwd_plane") and len(args) > 4 and args[4] == "false":
        return "fwd_plane"
    if s.startswith("k_zgreen"):
        return "zgreen"
    return None


def traffic(fetch_db, write_db, copy_fetch_db, copy_write_db, n, rb, copy_bytes=512 << 20,
            source_hash=None) -> str:
    """Counter table, plus (with source_hash) "key = value" lines of HBM bytes
    per launch for each pass (the largest-traffic kernel of each name)."""
    ff = copy_factor(copy_fetch_db, "FETCH_SIZE", copy_bytes)
    fw = copy_factor(copy_write_db, "WRITE_SIZE", copy_bytes)
    fc, wc = counters(fetch_db), counters(write_db)
    out = [f"counter scaling by a {copy_bytes >> 20} MiB device-to-device copy: FETCH_SIZE x {ff:.4f}, "
           f"WRITE_SIZE x {fw:.4f}",
           f"{'kernel':58s} {'fetch_MB':>9s} {'write_MB':>9s} {'hbm_MB':>9s} {'alg_MB':>9s} {'hbm/alg':>8s}"]
    keys = {}
    for name in sorted(fc, key=lambda k: -fc[k].get("FETCH_SIZE", 0)):
        if name not in wc:
            continue
        f = fc[name]["FETCH_SIZE"] * 1024.0 * ff
        w = wc[name]["WRITE_SIZE"] * 1024.0 * fw
        ab = algorithmic_bytes(name, n, rb)
        if ab is None:
            continue
        out.append(f"{short_name(name)[:58]:58s} {f / 1e6:9.1f} {w / 1e6:9.1f} {(f + w) / 1e6:9.1f} "
                   f"{ab / 1e6:9.1f} {(f + w) / ab:8.3f}")
        tn = timing_name(name)
        # the pass as the solve loop runs it: the parity-layout z pass where
        # there is one (template argument 5), else the largest traffic
        targs = short_name(name).split("<", 1)[1].rstrip(">").split(", ") if "<" in short_name(name) else []
        par = len(targs) > 4 and targs[4] == "true"
        if tn and (tn not in keys or (tn == "zgreen" and par)):
            keys[tn] = (f, w)
    if source_hash:
        out.append("")
        out.append(f"source_hash = {source_hash}")
        for tn, (f, w) in sorted(keys.items()):
            out.append(f"{tn}_fetch_bytes_per_launch = {f:.6e}")
            out.append(f"{tn}_write_bytes_per_launch = {w:.6e}")
            out.append(f"{tn}_hbm_bytes_per_launch = {f + w:.6e}")
    return "\n".join(out)


def sq(dbs) -> str:
    merged = collections.defaultdict(dict)
    for db in dbs:
        for k, v in counters(db).items():
            merged[k].update(v)
    out = []
    for name, c in sorted(merged.items(), key=lambda kv: -kv[1].get("GRBM_GUI_ACTIVE", 0)):
        if not short_name(name).startswith(("k_inv_plane", "k_fwd_plane", "k_zgreen")):
            continue
        out.append(short_name(name))
        cyc = c.get("GRBM_GUI_ACTIVE", 0) / XCDS  # GPU-busy cycles (summed over the XCDs)
        for key in sorted(c):
            out.append(f"    {key:24s} {c[key]:16.0f}")
        if cyc:
            if "SQ_ACTIVE_INST_VALU" in c:
                # one wave64 VALU instruction occupies a SIMD for 4 cycles
                out.append(f"    VALU busy                {4 * c['SQ_ACTIVE_INST_VALU'] / SIMDS / cyc:16.3f}")
            if "SQ_ACTIVE_INST_LDS" in c:
                out.append(f"    LDS issue busy           {4 * c['SQ_ACTIVE_INST_LDS'] / SIMDS / cyc:16.3f}")
            if "SQ_LDS_BANK_CONFLICT" in c and "SQ_ACTIVE_INST_LDS" in c and c["SQ_ACTIVE_INST_LDS"]:
                out.append(f"    LDS bank-conflict cycles / LDS active {c['SQ_LDS_BANK_CONFLICT'] / c['SQ_ACTIVE_INST_LDS']:8.3f}")
            if "SQ_WAVE_CYCLES" in c:
                # SQ_WAVE_CYCLES counts wave-cycles in units of 4 cycles, summed over the GPU
                out.append(f"    waves per SIMD (mean)    {4 * c['SQ_WAVE_CYCLES'] / SIMDS / cyc:16.2f}")
            if "SQ_WAIT_INST_LDS" in c and "SQ_WAVE_CYCLES" in c:
                out.append(f"    wave time waiting on LDS issue {c['SQ_WAIT_INST_LDS'] / c['SQ_WAVE_CYCLES']:10.3f}")
            if "SQ_WAIT_ANY" in c and "SQ_WAVE_CYCLES" in c:
                out.append(f"    wave time waiting (any)  {c['SQ_WAIT_ANY'] / c['SQ_WAVE_CYCLES']:16.3f}")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--n", type=int, default=256)
    t.add_argument("--real-bytes", type=int, default=4)
    tr = sub.add_parser("traffic")
    tr.add_argument("fetch_db")
    tr.add_argument("write_db")
    tr.add_argument("copy_fetch_db")
    tr.add_argument("copy_write_db")
    tr.add_argument("--n", type=int, default=256)
    tr.add_argument("--real-bytes", type=int, default=4)
    tr.add_argument("--source-hash", action="store_true",
                    help="append the per-launch bytes with the hash of the kernel sources of this tree")
    s = sub.add_parser("sq")
    s.add_argument("dbs", nargs="+")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace(a.db, a.n, a.real_bytes))
    elif a.cmd == "traffic":
        from ._build import kernel_source_hash
        print(traffic(a.fetch_db, a.write_db, a.copy_fetch_db, a.copy_write_db, a.n, a.real_bytes,
                      source_hash=kernel_source_hash() if a.source_hash else None))
    else:
        print(sq(a.dbs))


if __name__ == "__main__":
    sys.exit(main())
