"""GPU tests of the C ABI beyond numerics: error paths, workspaces and
streams from PyTorch, batched solves and the serving loop."""
import numpy as np
import pytest

import oracle
import paper_1504_07499_amd as rh
from paper_1504_07499_amd import geom

pytestmark = pytest.mark.gpu

K3 = np.array([0.2, 0.3, 400.0])


def test_argument_errors():
    print("\n[case] argument errors", flush=True)
    ph = geom.random_phases(16, 1)
    with rh.rve_create_from_phases(ph) as r:
        for bad_k in ([0.0, 1.0, 2.0], [1.0, -1.0, 2.0], [1.0, np.nan, 2.0], [np.inf, 1, 1]):
            with pytest.raises(rh.RveError) as ei:
                rh.homogenize(r, bad_k, 1e-6)
            assert ei.value.status == rh.RVE_ERR_ARG
        with pytest.raises(rh.RveError):
            rh.homogenize(r, K3, -1.0)
        with pytest.raises(rh.RveError):
            rh.homogenize(r, K3, 1e-6, precision=2)
        g = rh.homogenize(r, K3, 1e-12, max_iter=1, precision=1)
        assert g.status == rh.RVE_NOT_CONVERGED and list(g.iters) == [1, 1, 1]
    bad = ph.copy()
    bad[3, 2, 1] = 3
    with pytest.raises(rh.RveError):
        rh.rve_create_from_phases(bad)
    with pytest.raises(rh.RveError):
        rh.rve_create_from_phases(np.zeros((10, 10, 10), np.uint8))  # unsupported N


def test_fp32_stall_detection():
    """tol below the FP32 floor: without the FP64 continuation the solve stops
    as STALLED, not after max_iter; with it (the default) the stalled load
    cases continue in FP64 from their FP32 fields down to tol, and the tensor
    is the FP64 solve's."""
    print("\n[case] stall", flush=True)
    ph, _, _ = geom.generate(32, 8, 0.2, 0.1, 1)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K3, 1e-14, precision=0, max_iter=3000, fp32_refine=False)
        assert g.status == rh.RVE_STALLED
        assert g.iters.max() < 3000 and g.refine_iters.max() == 0
        ref = rh.homogenize(r, K3, 1e-14, precision=0, max_iter=3000, hist_cap=3000)
        f64 = rh.homogenize(r, K3, 1e-14, precision=1, max_iter=3000)
    assert ref.status == rh.RVE_OK
    assert np.all(ref.refine_iters > 0) and np.all(ref.iters > ref.refine_iters)
    assert np.all(ref.final_residual < 1e-14)
    for j in range(3):
        h = ref.history[j]
        assert len(h) == ref.iters[j] and h[-1] == ref.final_residual[j]
    assert np.abs(ref.K - f64.K).max() <= 1e-12 * np.abs(f64.K).max()


_TORCH_CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import torch
torch.cuda.init()
import paper_1504_07499_amd as rh
from paper_1504_07499_amd import geom
K3 = np.array([0.2, 0.3, 400.0])
ph, _, _ = geom.generate(32, 8, 0.2, 0.1, 1)
with rh.rve_create_from_phases(ph) as r:
    own = rh.homogenize(r, K3, 1e-6, precision=0)
    nbytes = rh.rve_workspace_size(r, 0)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ext = rh.homogenize(r, K3, 1e-6, precision=0, workspace=ws,
                            stream=torch.cuda.current_stream())
    small = torch.empty(nbytes // 2, dtype=torch.uint8, device="cuda")
    try:
        rh.homogenize(r, K3, 1e-6, precision=0, workspace=small)
        raise SystemExit("undersized workspace accepted")
    except rh.RveError:
        pass
assert np.array_equal(own.K, ext.K) and np.array_equal(own.iters, ext.iters)
print("torch interop ok", list(ext.iters), flush=True)
"""


_SHARED_WS_CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import torch
torch.cuda.init()
import paper_1504_07499_amd as rh
from paper_1504_07499_amd import geom
K3 = np.array([0.2, 0.3, 400.0])
pa, _, _ = geom.generate(32, 8, 0.2, 0.1, 1)
pb, _, _ = geom.generate(48, 10, 0.3, 0.2, 4)
with rh.rve_create_from_phases(pa) as a, rh.rve_create_from_phases(pb) as b:
    ws = torch.empty(max(rh.rve_workspace_size(a, 1), rh.rve_workspace_size(b, 1)), dtype=torch.uint8,
                     device="cuda")
    for prec in (1, 0):
        a1 = rh.homogenize(a, K3, 1e-6, precision=prec, workspace=ws)
        b1 = rh.homogenize(b, K3, 1e-6, precision=prec, workspace=ws)  # overwrites a's data in ws
        a2 = rh.homogenize(a, K3, 1e-6, precision=prec, workspace=ws)
        b2 = rh.homogenize(b, K3, 1e-6, precision=prec)
        assert np.array_equal(a1.K, a2.K) and np.array_equal(a1.iters, a2.iters), prec
        assert np.array_equal(b1.K, b2.K), prec
print("shared workspace ok", flush=True)
"""


def test_workspace_shared_between_handles():
    """One caller workspace used by two RVE handles of different N in turn:
    each solve rebuilds what it needs in it (the twiddle table included),
    so a handle's second solve equals its first bit for bit.  Child process
    with torch, as test_torch_workspace_and_stream."""
    import os
    import subprocess
    import sys

    pytest.importorskip("torch")
    print("\n[case] shared workspace (child process)", flush=True)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", _SHARED_WS_CHILD, root], capture_output=True,
                         text=True, timeout=300)
    print(out.stdout[-2000:], out.stderr[-2000:])
    assert out.returncode == 0
    assert "shared workspace ok" in out.stdout


def test_torch_workspace_and_stream():
    """Device memory and the stream may come from PyTorch; the result is the
    same as with the library's own workspace.  Runs in a child process that
    imports torch before the library, so both use torch's HIP runtime (a
    process can hold only one)."""
    import os
    import subprocess
    import sys

    pytest.importorskip("torch")
    print("\n[case] torch workspace (child process)", flush=True)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", _TORCH_CHILD, root], capture_output=True,
                         text=True, timeout=300)
    print(out.stdout[-2000:], out.stderr[-2000:])
    assert out.returncode == 0
    assert "torch interop ok" in out.stdout


@pytest.mark.parametrize("precision,scheme", [(0, "accelerated"), (1, "accelerated"),
                                              (0, "augmented_lagrangian")])
def test_batch_equals_alone(precision, scheme):
    """Mixed grid sizes in one batched solve: each result is bitwise the
    result of solving that RVE alone."""
    print(f"\n[case] batch precision={precision} scheme={scheme}", flush=True)
    specs = [(16, 3, 0.2, 0.2, 1), (24, 5, 0.25, 0.1, 2), (32, 8, 0.2, 0.1, 3),
             (48, 10, 0.3, 0.2, 4), (32, 4, 0.1, 0.3, 5)]
    rves = [rh.rve_create(*s) for s in specs]
    ks = np.array([K3, [1.0, 0.2, 400.0], K3, [0.2, 0.3, 20.0], K3])
    tols = np.array([1e-6, 1e-6, 1e-5, 1e-6, 1e-6])
    alone = [rh.homogenize(r, kk, t, precision=precision, scheme=scheme)
             for r, kk, t in zip(rves, ks, tols)]
    mixed = rh.homogenize_batch(rves, ks, tols, precision=precision, scheme=scheme)
    for a, b in zip(alone, mixed):
        assert np.array_equal(a.K, b.K)
        assert np.array_equal(a.iters, b.iters)
    # and each batched tensor against the FP64 oracle on the same phases
    sch = rh.SCHEMES[scheme]
    for r, kk, t, b in zip(rves, ks, tols, mixed):
        ref = oracle.homogenize(rh.rve_get_phases(r), kk, tol=t, scheme=sch)
        err = np.abs(b.K - ref.K).max() / np.abs(ref.K).max()
        assert err <= (1e-9 if precision else 1e-4), err
        if precision:
            assert list(b.iters) == list(ref.iters)
    for r in rves:
        r.close()


def test_server_results_match_alone():
    """Continuous batching: requests of different sizes and contrasts admitted
    while others run; every served tensor equals the alone solve."""
    print("\n[case] server", flush=True)
    reqs = [(32, 8, 0.2, 0.1, 11, [0.2, 0.3, 400.0], 1e-6),
            (16, 4, 0.2, 0.2, 12, [0.2, 0.3, 20.0], 1e-6),
            (64, 20, 0.2, 0.2, 13, [0.2, 0.3, 2000.0], 1e-6),
            (32, 10, 0.3, 0.1, 14, [0.2, 0.3, 2.0], 1e-6),
            (48, 12, 0.25, 0.3, 15, [0.2, 0.3, 200.0], 1e-6),
            (16, 2, 0.1, 0.3, 16, [0.2, 0.3, 400.0], 1e-6)]
    srv = rh.rve_server_create(1 << 30, 3, 0)
    tickets = [rh.rve_server_submit(srv, *q[:5], q[5], q[6]) for q in reqs]
    rh.rve_server_drain(srv)
    served = []
    for t in tickets:
        got = rh.rve_server_poll(srv, t)
        assert got is not None
        served.append(got)
    rh.rve_server_destroy(srv)
    for q, (res, lat) in zip(reqs, served):
        assert lat > 0
        with rh.rve_create(*q[:5]) as r:
            alone = rh.homogenize(r, q[5], q[6], precision=0)
            ph = rh.rve_get_phases(r)
        assert np.array_equal(res.K, alone.K)
        assert np.array_equal(res.iters, alone.iters)
        assert res.status == rh.RVE_OK
        ref = oracle.homogenize(ph, q[5], tol=q[6])
        assert np.abs(res.K - ref.K).max() / np.abs(ref.K).max() <= 1e-4


def _footprint(n, precision):
    """Device block of one served request: phase image, workspace and (FP32)
    the FP64 continuation's workspace, each rounded up to 256 bytes."""
    up = lambda b: (b + 255) // 256 * 256  # noqa: E731
    with rh.rve_create_from_phases(np.zeros((n, n, n), np.uint8)) as r:
        b = up(n ** 3) + up(rh.rve_workspace_size(r, precision))
        if precision == 0:
            b += up(rh.rve_workspace_size(r, 1))
    return b


def test_server_budget_admission_and_graph_reuse():
    """A budget of 1.5 request footprints keeps one request resident at a
    time, even when a backlog arrives while the server is idle; requests of
    one grid size reuse the instantiated iteration graphs; results equal the
    alone solves."""
    print("\n[case] server budget", flush=True)
    fp = _footprint(32, 0)
    srv = rh.rve_server_create(int(1.5 * fp), 4, 0)
    reqs = [(32, 8, 0.2, 0.1, 40 + i, [0.2, 0.3, 40.0 * (i + 1)], 1e-6) for i in range(5)]
    tickets = [rh.rve_server_submit(srv, *q[:5], q[5], q[6]) for q in reqs]
    rh.rve_server_drain(srv)
    served = [rh.rve_server_poll(srv, t) for t in tickets]
    st = rh.rve_server_get_stats(srv)
    rh.rve_server_destroy(srv)
    print(st, flush=True)
    assert st["resident_peak"] == 1
    assert st["peak_bytes"] <= st["arena_bytes"] and st["peak_bytes"] == fp
    assert st["admitted"] == 5 and st["completed"] == 5
    assert st["graph_hits"] > 0
    for q, (res, _) in zip(reqs, served):
        with rh.rve_create(*q[:5]) as r:
            alone = rh.homogenize(r, q[5], q[6], precision=0)
        assert np.array_equal(res.K, alone.K) and np.array_equal(res.iters, alone.iters)
    # a request larger than the budget is refused at submission
    srv = rh.rve_server_create(int(1.5 * fp), 2, 0)
    with pytest.raises(rh.RveError) as ei:
        rh.rve_server_submit(srv, 64, 8, 0.2, 0.1, 1, [0.2, 0.3, 400.0], 1e-6)
    assert ei.value.status == rh.RVE_ERR_OOM
    rh.rve_server_destroy(srv)


def test_kernel_timing_does_not_change_results():
    """Events recorded inside the replayed graphs: same tensor, one timed
    launch per working iteration (single stream), positive durations; with
    the three load-case chains each chain times its own launches."""

    print("\n[case] kernel timing", flush=True)
    ph, _, _ = geom.generate(48, 10, 0.25, 0.2, 8)
    with rh.rve_create_from_phases(ph) as r:
        one = rh.PATH_NO_CHAINS
        plain = rh.homogenize(r, K3, 1e-6, precision=0, path_flags=one)
        timed = rh.homogenize(r, K3, 1e-6, precision=0, timing=True, path_flags=one)
        kt = rh.rve_get_kernel_times(r)
        only = rh.homogenize(r, K3, 1e-6, precision=0, timing=4, path_flags=one)
        kt4 = rh.rve_get_kernel_times(r)
        sampled = rh.homogenize(r, K3, 1e-6, precision=0, timing=4 | 16, path_flags=one)
        kts = rh.rve_get_kernel_times(r)
        chained = rh.homogenize(r, K3, 1e-6, precision=0, timing=True)
        ktc = rh.rve_get_kernel_times(r)
    assert np.array_equal(plain.K, timed.K) and np.array_equal(plain.K, only.K)
    assert np.array_equal(plain.K, sampled.K) and np.array_equal(plain.K, chained.K)
    # the kernel times cover the FP32 iterations (not the FP64 continuation)
    it32 = plain.iters - plain.refine_iters
    # sampled: one batch of iterations in four carries events
    assert 0 < kts[list(kts)[2]]["launches"] < int(it32.max())
    assert kts[list(kts)[2]]["total_ms"] > 0
    names = list(kt)
    assert names[1] == "zgreen" and names[3] == "reduce"
    for name in names[1:]:
        assert kt[name]["launches"] == int(it32.max())
        assert kt[name]["total_ms"] > 0
        # chains: every load case launches its own kernels
        assert ktc[name]["launches"] == int(it32.sum())
        assert ktc[name]["total_ms"] > 0
    assert kt4[names[2]]["launches"] == int(it32.max())
    assert kt4["zgreen"]["launches"] == 0


def test_fused_pass_matches_separate_passes():
    """The fused inverse + next forward pass gives the separate passes'
    result (identical arithmetic, different kernel boundaries)."""

    print("\n[case] fused vs separate", flush=True)
    ph, _, _ = geom.generate(64, 12, 0.3, 0.2, 21)
    with rh.rve_create_from_phases(ph) as r:
        fused = rh.homogenize(r, K3, 1e-6, precision=1)
        sep = rh.homogenize(r, K3, 1e-6, precision=1, path_flags=rh.PATH_NO_FUSED)
    assert np.array_equal(fused.iters, sep.iters)
    assert np.abs(fused.K - sep.K).max() <= 1e-12 * np.abs(sep.K).max()


@pytest.mark.parametrize("precision", [0, 1])
def test_load_case_chains_match_single_stream(precision):
    """A full solve runs as three concurrent single-load-case solves (own
    streams and graphs); tensor, iteration counts and histories equal those
    of the single-stream solve of all three load cases."""

    print(f"\n[case] chains vs single stream precision={precision}", flush=True)
    ph, _, _ = geom.generate(64, 12, 0.3, 0.2, 23)
    with rh.rve_create_from_phases(ph) as r:
        chained = rh.homogenize(r, K3, 1e-6, precision=precision, hist_cap=512)
        single = rh.homogenize(r, K3, 1e-6, precision=precision, hist_cap=512,
                               path_flags=rh.PATH_NO_CHAINS)
        one = rh.homogenize(r, K3, 1e-6, precision=precision, lc_mask=2)
    assert np.array_equal(chained.K, single.K)
    assert np.array_equal(chained.iters, single.iters)
    assert np.array_equal(chained.lc_status, single.lc_status)
    for j in range(3):
        n = int(single.iters[j])
        np.testing.assert_array_equal(chained.history[j][:n], single.history[j][:n])
    # a single load case (its own grid) gives that column exactly
    assert np.array_equal(one.K[:, 1], single.K[:, 1]) and int(one.iters[1]) == int(single.iters[1])


@pytest.mark.parametrize("n,precision", [(64, 0), (128, 0), (64, 1)])
def test_z_tile_widths_give_identical_results(n, precision):
    """The autotuner picks one of two z-tile widths per grid size; both give
    bitwise the same result (the z transform of a pencil does not depend on
    how many pencils a tile holds)."""

    print(f"\n[case] z tile widths n={n} precision={precision}", flush=True)
    ph, _, _ = geom.generate(n, 12, 0.3, 0.2, 31)
    out = []
    with rh.rve_create_from_phases(ph) as r:
        for v in (rh.PATH_ZTILE_DEFAULT, rh.PATH_ZTILE_ALT):
            out.append(rh.homogenize(r, K3, 1e-6, precision=precision, max_iter=60, path_flags=v))
    assert np.array_equal(out[0].K, out[1].K)
    assert np.array_equal(out[0].iters, out[1].iters)


@pytest.mark.parametrize("n,precision", [(32, 1), (64, 0), (128, 0), (48, 1)])
def test_plane_thread_counts_agree(n, precision):
    """The autotuner picks one of two thread counts per workgroup for the
    fused plane pass.  Both run the same arithmetic per voxel (up to the
    compiler's instruction choice for each shape) and group the FP64
    partial sums (residual, flux) differently.  The fields after a fixed
    number of iterations match the oracle's at either count (FP64 within
    1e-9, FP32 within 3e-5 of the largest value), and the forced
    alternative converges like the oracle (FP64: the same iteration counts,
    tensor within 1e-9)."""
    print(f"\n[case] plane thread counts n={n} precision={precision}", flush=True)
    ph, _, _ = geom.generate(n, 12, 0.3, 0.2, 31)
    ref20 = oracle.homogenize(ph, K3, tol=0.0, max_iter=20, want_field=True)
    scale = np.max(np.abs(ref20.field))
    bar = 1e-9 if precision == 1 else 3e-5
    with rh.rve_create_from_phases(ph) as r:
        for v in (rh.PATH_PLANE_DEFAULT, rh.PATH_PLANE_ALT):
            g = rh.homogenize(r, K3, 0.0, precision=precision, max_iter=20, want_field=True, path_flags=v)
            assert np.max(np.abs(g.field - ref20.field)) <= bar * scale
            assert np.max(np.abs(g.K - ref20.K)) <= bar * np.max(np.abs(ref20.K))
        if n <= 32 and precision == 1:
            ref = oracle.homogenize(ph, K3, tol=1e-6)
            g = rh.homogenize(r, K3, 1e-6, precision=1, path_flags=rh.PATH_PLANE_ALT)
            assert np.array_equal(g.iters, ref.iters)
            assert np.max(np.abs(g.K - ref.K)) <= 1e-9 * np.max(np.abs(ref.K))
        # the autotuned solve leaves a plane choice for this grid in the table
        rh.homogenize(r, K3, 1e-6, precision=precision, max_iter=5)
    assert any(ln.split()[1:4] == [str(precision), str(n), "plane"] for ln in rh.rve_tune_export().splitlines())


@pytest.mark.parametrize("precision", [1, 0])
def test_nonfinite_start_field_is_reported(precision):
    """A NaN in the start field of load case e_2 makes its residual
    non-finite: the solve reports NONFINITE (as the oracle does for that load
    case, after one iteration); the other load cases, solved from the same
    start field, converge as without it."""
    print(f"\n[case] non-finite start field precision={precision}", flush=True)
    import oracle

    ph = geom.random_phases(16, 21)
    init = np.zeros((3, 3, 16, 16, 16))
    for j in range(3):
        init[j, j] = 1.0
    init[1, 0, 3, 4, 5] = np.nan
    ref = oracle.homogenize(ph, K3, tol=1e-6, init_field=init)
    assert ref.status[1] == rh.RVE_ERR_NONFINITE and int(ref.iters[1]) == 1
    with rh.rve_create_from_phases(ph) as r:
        with pytest.raises(rh.RveError) as err:
            rh.homogenize(r, K3, 1e-6, precision=precision, init_field=init)
        assert err.value.status == rh.RVE_ERR_NONFINITE
        g = rh.homogenize(r, K3, 1e-6, precision=precision, init_field=init, lc_mask=5)
        clean = rh.homogenize(r, K3, 1e-6, precision=precision, lc_mask=5)
    for j in (0, 2):
        assert int(g.lc_status[j]) == int(clean.lc_status[j])
        np.testing.assert_allclose(g.K[:, j], clean.K[:, j], rtol=1e-12, atol=0)
