"""The per-kernel summaries of rocprofv3 databases (no GPU: small SQLite
files written here stand in for the profiler's output).  Checks the
algorithmic byte counts against the sizes they are defined from, the
precision filter of the trace table, and the counter scaling by the copy
kernel's reading."""
import sqlite3

import pytest

from paper_1504_07499_amd import profile_summary as ps

MB = 1e6


def sizes(n, rb):
    """e (9 channels of n^3 reals), the half spectrum with its kx = n/2
    column (9 n^2 (n/2 + 1) complex values) and the phase image (n^3 B)."""
    m = n ** 3
    return 9.0 * m * rb, 9.0 * n * n * (n // 2 + 1) * 2 * rb, float(m)


@pytest.mark.parametrize("n", [128, 256])
def test_algorithmic_bytes_of_each_pass(n):
    field, spec, phase = sizes(n, 4)
    f64, s64, _ = sizes(n, 8)
    ab = ps.algorithmic_bytes
    # fused inverse + forward pass: spectrum in and out, e in and out, phases once
    assert ab(f"k_inv_plane<float, {n}, 2, 1024, true, 0, 3, 16, 2>", n, 4) == 2 * spec + 2 * field + phase
    # separate inverse pass and first forward pass
    assert ab(f"k_inv_plane<float, {n}, 1, 512, false, 0>", n, 4) == spec + 2 * field + phase
    assert ab(f"k_fwd_plane<float, {n}, 2, 1024, false, 3, true, 16>", n, 4) == field + spec + phase
    # z pass: the spectrum in and out
    assert ab(f"k_zgreen<float, {n}, 8, 256, true, 2>", n, 4) == 2 * spec
    # FP64 kernels take 8 bytes per real whatever the trace's precision
    assert ab(f"k_zgreen<double, {n}, 4, 256, true, 4>", n, 4) == 2 * s64
    # the five-pass form of the conductivity case (last argument NC = 3)
    assert ab(f"k_fwd_rows<double, {n}, 16, 256, false, 3>", n, 8) == f64 + s64 + phase
    assert ab(f"k_cols<double, {n}, 16, 256, true, false, 3>", n, 8) == 2 * s64
    assert ab(f"k_inv_rows<double, {n}, 16, 256, 0, 3>", n, 8) == s64 + 2 * f64 + phase
    # the elastic case (six components per load case: 36 channels)
    assert ab(f"k_inv_rows<float, {n}, 16, 256, 0, 6>", n, 4) == 4 * (spec + 2 * field) + phase
    assert ab(f"k_inv_plane<float, {n}, 2, 1024, true, 0, 6, 16, 2>", n, 4) == 4 * (2 * spec + 2 * field) + phase
    assert ab(f"k_fwd_plane<float, {n}, 2, 1024, false, 6, true, 16>", n, 4) == 4 * (field + spec) + phase
    assert ab(f"k_zgreen_el<float, {n}, 8, 1024, true>", n, 4) == 4 * 2 * spec
    # other kernels are not counted
    assert ab("k_reduce", n, 4) is None
    # the 256^3 FP32 figures quoted with the profiles
    if n == 256:
        assert round(ab("k_inv_plane<float, 256, 2, 1024, true, 0, 3, 16, 2>", n, 4) / MB, 1) == 2442.1
        assert round(ab("k_zgreen<float, 256, 8, 256, true, 2>", n, 4) / MB, 1) == 1217.4


def test_names():
    assert ps.short_name("void rvehom::k_zgreen<float, 256, 8, 256, true, 2>(Cx<float>*, int)") == \
        "k_zgreen<float, 256, 8, 256, true, 2>"
    assert ps.timing_name("k_inv_plane<float, 256, 2, 1024, true, 0, 3, 16, 2>") == "inv_fwd_plane"
    assert ps.timing_name("k_inv_plane<float, 256, 2, 1024, false, 0, 3, 2, 2>") == "inv_plane"
    assert ps.timing_name("k_fwd_plane<float, 256, 2, 1024, false, 3, true, 16>") == "fwd_plane"
    assert ps.timing_name("k_zgreen<float, 256, 8, 256, true, 2>") == "zgreen"
    assert ps.timing_name("k_cols<float, 512, 16, 256, true, false, 3>") is None


def _db(path, kernels=(), counters=()):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, duration real, grid_x int, workgroup_x int, lds_size int, "
                "vgpr_count int, accum_vgpr_count int)")
    con.executemany("insert into kernels values (?, ?, ?, ?, ?, ?, ?)", kernels)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", counters)
    con.commit()
    con.close()
    return str(path)


def test_trace_rates_and_precision_filter(tmp_path):
    fused = "k_inv_plane<float, 256, 2, 1024, true, 0, 3, 16, 2>"
    fp64 = "k_inv_plane<double, 256, 4, 512, true, 0, 3, 1, 16>"
    # two full launches and one that exited at once (every load case frozen)
    db = _db(tmp_path / "t.db", kernels=[(fused, 600e3, 4608 * 1024, 1024, 134552, 64, 0),
                                         (fused, 620e3, 4608 * 1024, 1024, 134552, 64, 0),
                                         (fused, 8e3, 4608 * 1024, 1024, 134552, 64, 0),
                                         (fp64, 450e3, 9216 * 512, 512, 136432, 112, 0)])
    rows = {ln.split()[0]: ln.split() for ln in ps.trace(db, 256, 4).splitlines()[1:]}
    r = rows["k_inv_plane<float,"]
    # grid in workgroups, calls, short launches, average duration of the
    # full ones, bytes, rate and fraction of 8 TB/s
    cols = r[len(fused.split()):]
    assert cols[0] == "4608" and cols[4] == "3" and cols[5] == "1"
    assert float(cols[6]) == pytest.approx(610.0)
    alg = ps.algorithmic_bytes(fused, 256, 4)
    assert float(cols[7]) == pytest.approx(alg / MB, abs=0.05)
    assert float(cols[8]) == pytest.approx(alg / 610e-6 / 1e12, abs=0.005)
    assert float(cols[9]) == pytest.approx(alg / 610e-6 / 8e12, abs=0.0005)
    # an FP64 kernel in an FP32 trace (a continuation on fewer load cases): no byte count
    assert len(rows["k_inv_plane<double,"]) == len(fp64.split()) + 7


def test_traffic_scaled_by_the_copy(tmp_path):
    fused = "k_inv_plane<float, 256, 2, 1024, true, 0, 3, 16, 2>"
    copy = "__amd_rocclr_copyBuffer"
    copy_bytes = 512 << 20
    # FETCH_SIZE reads half the copy's bytes (factor 2), WRITE_SIZE all of them
    fc = _db(tmp_path / "fc.db", counters=[(copy, "FETCH_SIZE", copy_bytes / 2 / 1024)])
    wc = _db(tmp_path / "wc.db", counters=[(copy, "WRITE_SIZE", copy_bytes / 1024)])
    f = _db(tmp_path / "f.db", counters=[(fused, "FETCH_SIZE", 620e6 / 1024), (fused, "FETCH_SIZE", 620e6 / 1024)])
    w = _db(tmp_path / "w.db", counters=[(fused, "WRITE_SIZE", 1213e6 / 1024)])
    out = ps.traffic(f, w, fc, wc, 256, 4, source_hash="abc")
    assert "FETCH_SIZE x 2.0000, WRITE_SIZE x 1.0000" in out
    keys = dict(ln.split(" = ") for ln in out.splitlines() if " = " in ln)
    assert keys["source_hash"] == "abc"
    assert float(keys["inv_fwd_plane_fetch_bytes_per_launch"]) == pytest.approx(1240e6, rel=1e-6)
    assert float(keys["inv_fwd_plane_write_bytes_per_launch"]) == pytest.approx(1213e6, rel=1e-6)
    assert float(keys["inv_fwd_plane_hbm_bytes_per_launch"]) == pytest.approx(2453e6, rel=1e-6)


def test_committed_traffic_summary_matches_the_kernel_sources():
    """The bench reports the counter traffic of its dominant kernel only from
    a summary taken on the kernel sources in the tree: the committed one must
    carry their hash and the three passes' bytes per launch."""
    import bench

    for k in ("inv_fwd_plane", "zgreen", "fwd_plane"):
        v = bench.measured_traffic(k, 0)
        assert v is not None and v > 1e9, k
    # within a few per cent of the algorithmic bytes (no re-reads to speak of)
    alg = ps.algorithmic_bytes("k_inv_plane<float, 256, 2, 1024, true, 0, 3, 16, 2>", 256, 4)
    assert 1.0 <= bench.measured_traffic("inv_fwd_plane", 0) / alg <= 1.1
