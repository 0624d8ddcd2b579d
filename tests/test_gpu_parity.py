"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Inputs are seeded phase images from the input generator; the oracle and the
HIP path share nothing else.  Bars: FP64 mode 1e-9 per tensor entry
(relative to the largest entry), FP32 mode 1e-4 (the two tolerances the
build targets); fields compared element by element after a fixed number of
iterations.
"""
import numpy as np
import pytest

import oracle
import paper_1504_07499_amd as rh
from paper_1504_07499_amd import geom

pytestmark = pytest.mark.gpu

K_PAPER_CFG = np.array([0.2, 0.3, 400.0])  # matrix, inclusion, coating


def tensor_err(K, Kref):
    return float(np.abs(K - Kref).max() / np.abs(Kref).max())


def field_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48, 64, 96, 128])
def test_field_after_fixed_iterations(n, precision):
    """Three iterations from E on an i.i.d. phase image: every voxel of every
    channel matches the oracle (steps 2-7 of the Algorithm end to end)."""
    print(f"\n[case] field n={n} precision={precision}", flush=True)
    ph = geom.random_phases(n, seed=100 + n)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=3, want_field=True)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=3, precision=precision,
                          want_field=True, hist_cap=8)
    bar = 1e-11 if precision == 1 else 3e-5
    assert field_err(g.field, ref.field) <= bar
    assert tensor_err(g.K, ref.K) <= bar
    assert list(g.iters) == [3, 3, 3]
    for j in range(3):
        np.testing.assert_allclose(g.history[j], ref.history[j], rtol=bar * 10)


@pytest.mark.parametrize("n", [8, 16, 32])
def test_homogeneous_medium(n):
    """Every voxel one phase: K = k I after one iteration with residual 0."""
    print(f"\n[case] homogeneous n={n}", flush=True)
    ph = np.full((n, n, n), 1, dtype=np.uint8)
    with rh.rve_create_from_phases(ph) as r:
        for prec in (1, 0):
            g = rh.homogenize(r, [1.0, 3.5, 400.0], 1e-10, precision=prec)
            assert g.status == rh.RVE_OK
            assert list(g.iters) == [1, 1, 1]
            np.testing.assert_allclose(g.K, 3.5 * np.eye(3), atol=1e-12 if prec else 1e-5)


def test_config1_fp64_converged():
    """32^3, 8 RSA spheres, f = 0.2, l = 0.1, seed 1, k = (0.2, 0.3, 400),
    tol 1e-6, FP64: tensor within 1e-9 of the oracle, same iteration counts."""
    print("\n[case] config1 fp64", flush=True)
    ph, _, _ = geom.generate(32, 8, 0.2, 0.1, 1)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=1e-6)
    with rh.rve_create(32, 8, 0.2, 0.1, 1) as r:
        assert np.array_equal(rh.rve_get_phases(r), ph)
        g = rh.homogenize(r, K_PAPER_CFG, 1e-6, precision=1, hist_cap=1000)
    assert g.status == rh.RVE_OK
    assert list(g.iters) == list(ref.iters)
    assert tensor_err(g.K, ref.K) <= 1e-9
    for j in range(3):
        np.testing.assert_allclose(g.history[j], ref.history[j], rtol=1e-9)


@pytest.mark.parametrize("n", [32, 48, 64])
def test_fp32_converged_vs_oracle(n):
    """FP32 FFT/update with FP64 reductions: tensor within 1e-4 of the oracle."""
    print(f"\n[case] fp32 converged n={n}", flush=True)
    ph, _, _ = geom.generate(n, 8, 0.2, 0.1, 7)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=1e-6)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 1e-6, precision=0)
    assert g.status in (rh.RVE_OK, rh.RVE_STALLED)
    assert tensor_err(g.K, ref.K) <= 1e-4


@pytest.mark.parametrize("flags", [0, rh.PATH_NO_FUSED])
def test_split_plane_path_256_fp32(flags):
    """256^3 in FP32 uses the row-parity split of the xy-plane (two
    workgroups per plane), by default with the fused inverse + forward pass
    writing the parity-layout spectrum that the z pass combines, else with
    separate passes: two iterations of load case e_1 on an RSA RVE, field
    compared voxel by voxel with the oracle."""
    print(f"\n[case] split plane 256 fp32 flags={flags}", flush=True)
    ph, _, _ = geom.generate(256, 100, 0.3, 0.2, 3)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=2, want_field=True, lc_mask=1)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=2, precision=0, lc_mask=1,
                          want_field=True, path_flags=flags)
    assert field_err(g.field[0], ref.field[0]) <= 3e-5
    assert np.array_equal(g.field[1:], ref.field[1:])
    assert tensor_err(g.K[:, 0], ref.K[:, 0]) <= 3e-5


def test_split_plane_fused_equals_separate_256():
    """A full 256^3 FP32 solve (three load cases, every tile of the parity
    layout and both spectrum buffers in use): the fused pass and the
    separate passes reach the same tensor (FP32 rounding apart) in the same
    number of iterations give or take the last one."""
    print("\n[case] split plane fused vs separate 256", flush=True)
    k = [0.2, 0.3, 20.0]
    with rh.rve_create(256, 100, 0.4, 0.1, 3) as r:
        a = rh.homogenize(r, k, 1e-5, precision=0, fp32_refine=False)
        b = rh.homogenize(r, k, 1e-5, precision=0, fp32_refine=False, path_flags=rh.PATH_NO_FUSED)
        c = rh.homogenize(r, k, 1e-5, precision=1)
    print(list(a.iters), list(b.iters), list(c.iters), tensor_err(a.K, b.K), tensor_err(a.K, c.K), flush=True)
    assert a.status == rh.RVE_OK and b.status == rh.RVE_OK
    assert np.all(np.abs(a.iters - b.iters) <= 1)
    assert tensor_err(a.K, b.K) <= 2e-6
    assert tensor_err(a.K, c.K) <= 1e-5


@pytest.mark.parametrize("precision", [0, 1])
def test_mirror_covariance_on_gpu(precision):
    """Mirroring the microstructure along x flips the sign of row/column x
    of K (the Nyquist treatment keeps this exact on even grids)."""
    print(f"\n[case] mirror precision={precision}", flush=True)
    ph, _, _ = geom.generate(32, 6, 0.25, 0.3, 12)
    with rh.rve_create_from_phases(ph) as a, \
            rh.rve_create_from_phases(np.ascontiguousarray(ph[:, :, ::-1])) as b:
        ka = rh.homogenize(a, K_PAPER_CFG, 1e-9, precision=precision, stall_window=0).K
        kb = rh.homogenize(b, K_PAPER_CFG, 1e-9, precision=precision, stall_window=0).K
    R = np.diag([-1.0, 1.0, 1.0])
    assert tensor_err(kb, R @ ka @ R) <= (1e-9 if precision else 1e-4)


@pytest.mark.parametrize("n", [16, 32])
def test_equilibrium_error_fp64(n):
    """eps_eq of step 1 at exit (fixed iteration count) and the two-stage
    stop (eps_comp then eps_eq below tol) against the oracle."""
    print(f"\n[case] equilibrium n={n}", flush=True)
    ph, _, _ = geom.generate(n, 4, 0.2, 0.3, 4)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=25)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=25, precision=1)
        np.testing.assert_allclose(g.eps_eq, ref.eps_eq, rtol=1e-9)
        ref2 = oracle.homogenize(ph, K_PAPER_CFG, tol=1e-6, eq_check=True)
        g2 = rh.homogenize(r, K_PAPER_CFG, 1e-6, precision=1, equilibrium_check=True)
    assert g2.status == rh.RVE_OK
    assert list(g2.iters) == list(ref2.iters)
    assert np.all(g2.eps_eq < 1e-6)
    assert tensor_err(g2.K, ref2.K) <= 1e-9


@pytest.mark.parametrize("n,precision", [(128, 0), (144, 1), (192, 1), (256, 0), (256, 1)])
def test_equilibrium_error_at_exit_every_path(n, precision):
    """eps_eq reported at exit, on the paths whose flux transform differs from
    the 16^3-32^3 whole planes: whole planes in FP32 (128), split planes in
    FP64 (144; 192, whose iterations use the parity layout), split planes in
    FP32 and the five-pass flux transform (256; FP64 iterates in quarter
    planes).  Checked against the oracle's
    equilibrium error of the final field the GPU returns, load case by load
    case (the FP32 flux transform rounds at ~1e-6 of the flux)."""
    print(f"\n[case] eps_eq at exit n={n} precision={precision}", flush=True)
    ph, _, _ = geom.generate(n, 30, 0.3, 0.2, 11)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=6, precision=precision, want_field=True)
    kvox = np.asarray(K_PAPER_CFG)[ph]
    for j in range(3):
        ref = oracle.equilibrium_error(kvox, g.field[j])
        assert ref > 0
        assert abs(g.eps_eq[j] - ref) <= (1e-9 if precision == 1 else 1e-3) * ref, (j, g.eps_eq[j], ref)


def _golden_all():
    import json
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_refs.json")
    with open(path) as f:
        return json.load(f)


def _golden(name):
    return _golden_all()[name]


@pytest.mark.parametrize("precision", [0, 1])
def test_config2_128_vs_stored_oracle(precision):
    """The benchmark workload (128^3, 50 RSA spheres, f = 0.3, l = 0.2,
    seed 2, tol 1e-6) in the launch configuration bench.py times, against
    the stored oracle tensor (tests/golden/make_oracle_refs.py)."""
    print(f"\n[case] config2 128 precision={precision}", flush=True)
    ref = _golden("rve128_50sph_f0.30_l0.20_seed2")
    g0 = ref["geometry"]
    with rh.rve_create(g0["n"], g0["n_spheres"], g0["volume_fraction"], g0["layer"],
                       g0["seed"]) as r:
        frac = np.bincount(rh.rve_get_phases(r).ravel(), minlength=3) / 128 ** 3
        np.testing.assert_allclose(frac, ref["phase_fractions"], atol=1e-12)
        g = rh.homogenize(r, ref["k_phases"], ref["tol"], precision=precision)
    Kr = np.array(ref["K"])
    if precision == 1:
        assert g.status == rh.RVE_OK
        assert list(g.iters) == ref["iters"]
        assert tensor_err(g.K, Kr) <= 1e-9
    else:
        # FP32 stops at its rounding floor above tol; the FP64 continuation
        # takes the stalled load cases below tol
        assert g.status == rh.RVE_OK, (list(g.lc_status), list(g.refine_iters))
        assert np.all(g.final_residual < ref["tol"])
        assert tensor_err(g.K, Kr) <= 1e-4


@pytest.mark.parametrize("name", ["rve256_100sph_f0.40_l0.10_c1e3_seed3", "rve256_100sph_f0.40_l0.20_c1e2_seed3",
                                  "rve256_100sph_f0.40_l0.05_c1e4_seed3"])
def test_config3_256_vs_stored_oracle(name):
    """The 256^3 RVE (100 spheres, f = 0.40 through the generator's fallback,
    seed 3) at the (layer, contrast) points with stored oracle solves
    (tests/golden/make_oracle_refs.py): FP64 (quarter planes) with the
    oracle's iteration counts and within 1e-9; FP32 in the configuration the
    benchmark times (split planes, load-case chains, FP64 continuation past
    the FP32 floor) within 1e-4, converged."""
    refs = _golden_all()
    if name not in refs:
        pytest.skip(f"no stored oracle solve for {name}")
    ref = refs[name]
    print(f"\n[case] config3 {name}", flush=True)
    g0 = ref["geometry"]
    Kr = np.array(ref["K"])
    with rh.rve_create(g0["n"], g0["n_spheres"], g0["volume_fraction"], g0["layer"], g0["seed"]) as r:
        frac = np.bincount(rh.rve_get_phases(r).ravel(), minlength=3) / 256 ** 3
        np.testing.assert_allclose(frac, ref["phase_fractions"], atol=1e-12)
        g64 = rh.homogenize(r, ref["k_phases"], ref["tol"], precision=1)
        g32 = rh.homogenize(r, ref["k_phases"], ref["tol"], precision=0)
    print(list(g64.iters), list(g32.iters), list(g32.refine_iters), tensor_err(g64.K, Kr), tensor_err(g32.K, Kr),
          flush=True)
    assert g64.status == rh.RVE_OK and list(g64.iters) == ref["iters"]
    assert tensor_err(g64.K, Kr) <= 1e-9
    assert g32.status == rh.RVE_OK
    assert tensor_err(g32.K, Kr) <= 1e-4


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("n", [36, 72, 144, 192])
def test_smooth_sizes_fixed_iterations(n, precision):
    """{2,3}-smooth grids with two radix-3 stages (36, 144) or one beyond
    96 (72, 192), on the paths their planes take (whole planes; split
    planes for FP64 144 and 192, with the parity layout at 192): three
    iterations from E, every voxel of every channel against the oracle."""
    print(f"\n[case] smooth field n={n} precision={precision}", flush=True)
    ph = geom.random_phases(n, seed=700 + n)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=3, want_field=True)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=3, precision=precision,
                          want_field=True, hist_cap=8)
    bar = 1e-11 if precision == 1 else 3e-5
    assert field_err(g.field, ref.field) <= bar
    assert tensor_err(g.K, ref.K) <= bar
    assert list(g.iters) == [3, 3, 3]


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("n", [288, 384])
def test_smooth_sizes_five_pass(n, precision):
    """288 and 384 run the five-pass form in both precisions: two
    iterations of load case e_1 on an RSA RVE, voxel by voxel."""
    print(f"\n[case] smooth five-pass n={n} precision={precision}", flush=True)
    ph, _, _ = geom.generate(n, 60, 0.3, 0.2, 9)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=2, want_field=True, lc_mask=1)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=2, precision=precision, lc_mask=1,
                          want_field=True)
    bar = 1e-11 if precision == 1 else 3e-5
    assert field_err(g.field[0], ref.field[0]) <= bar
    assert tensor_err(g.K[:, 0], ref.K[:, 0]) <= bar


@pytest.mark.parametrize("precision", [1, 0])
def test_five_pass_512_vs_oracle(precision):
    """512^3 (five-pass form in both precisions) on an RSA RVE: two
    iterations of load case e_1, the tensor column and the residual history
    against the oracle (the voxel field would need ~20 GB of host memory)."""
    print(f"\n[case] five-pass 512 precision={precision}", flush=True)
    ph, _, _ = geom.generate(512, 100, 0.3, 0.2, 7)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=2, lc_mask=1)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=2, precision=precision, lc_mask=1, hist_cap=4)
    bar = 1e-11 if precision == 1 else 3e-5
    assert tensor_err(g.K[:, 0], ref.K[:, 0]) <= bar
    np.testing.assert_allclose(g.history[0], ref.history[0], rtol=bar * 10)


@pytest.mark.parametrize("flags", [0, 2])
def test_five_pass_256_fp64_vs_oracle(flags):
    """FP64 at 256^3, whose half xy-plane does not fit in LDS: by default
    the fused pass in quarter planes with the four-quarter z pass (the
    first forward pass too), else (flags 2) the five-pass form: two
    iterations of load case e_1, voxel by voxel against the oracle."""
    print(f"\n[case] 256 fp64 flags={flags}", flush=True)
    ph, _, _ = geom.generate(256, 100, 0.3, 0.2, 3)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=2, want_field=True, lc_mask=1)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=2, precision=1, lc_mask=1,
                          want_field=True, path_flags=flags)
    assert field_err(g.field[0], ref.field[0]) <= 1e-11
    assert np.array_equal(g.field[1:], ref.field[1:])
    assert tensor_err(g.K[:, 0], ref.K[:, 0]) <= 1e-11


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n,precision", [(512, 0), (256, 1), (512, 1)])
def test_large_grid_laminate_exact(n, precision, axis):
    """Closed form at sizes the oracle cannot run in a test: a laminate
    normal to direction `axis` (x, y or z, so that each of the x, y and z
    transforms carries the variation) with odd layer widths gives <k> on the
    diagonal and 1/<1/k> in the normal direction."""
    print(f"\n[case] laminate n={n} precision={precision} axis={axis}", flush=True)
    k = np.array([1.0, 0.2, 4.0])
    widths = [n // 2 - 1, 3, n // 2 - 2]
    prof = np.concatenate([np.full(w, p, np.uint8) for w, p in zip(widths, [0, 2, 1])])
    shape = [1, 1, 1]
    shape[2 - axis] = n  # the phase image is [z][y][x]
    ph = np.ascontiguousarray(np.broadcast_to(prof.reshape(shape), (n, n, n)))
    kv = k[prof]
    Kex = np.eye(3) * kv.mean()
    Kex[axis, axis] = 1.0 / (1.0 / kv).mean()
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, k, 1e-10 if precision else 1e-6, precision=precision)
    assert tensor_err(g.K, Kex) <= (1e-9 if precision else 2e-5)


def test_graph_replays_match_eager_launches():
    """Chunks of iterations replayed from a captured graph give bitwise the
    result of kernel-by-kernel launches, over several solves with host work
    and synchronisation in between."""

    print("\n[case] graph replay vs eager", flush=True)
    ph, _, _ = geom.generate(48, 10, 0.25, 0.2, 8)
    with rh.rve_create_from_phases(ph) as r:
        eager = rh.homogenize(r, K_PAPER_CFG, 1e-6, precision=0, path_flags=rh.PATH_NO_GRAPHS)
        for rep in range(3):
            g = rh.homogenize(r, K_PAPER_CFG, 1e-6, precision=0)
            assert np.array_equal(g.K, eager.K), rep
            assert np.array_equal(g.iters, eager.iters), rep
            _ = rh.rve_get_phases(r)


def test_basic_scheme_fp64_vs_oracle():
    """The basic scheme option: field after 5 iterations equals the oracle's."""
    print("\n[case] basic scheme", flush=True)
    ph = geom.random_phases(24, 77)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=5, want_field=True, scheme=1)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=5, precision=1, want_field=True,
                          scheme="basic")
    assert field_err(g.field, ref.field) <= 1e-11


AL = "augmented_lagrangian"


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("n", [8, 12, 24, 48, 64, 96, 128])
def test_augmented_lagrangian_fixed_iterations(n, precision):
    """Augmented-Lagrangian scheme (named in Sec. 3; k0 of Sec. 5): after
    four iterations from E, the state lam - k0 d of every voxel of every
    channel, the tensor <k d> and the residual history match the oracle."""
    print(f"\n[case] augmented lagrangian n={n} precision={precision}", flush=True)
    ph = geom.random_phases(n, seed=300 + n)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=4, want_field=True, scheme=2)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=4, precision=precision,
                          want_field=True, hist_cap=8, scheme=AL)
    bar = 1e-11 if precision == 1 else 3e-5
    assert field_err(g.field, ref.field) <= bar
    assert tensor_err(g.K, ref.K) <= bar
    assert list(g.iters) == [4, 4, 4]
    for j in range(3):
        np.testing.assert_allclose(g.history[j], ref.history[j], rtol=bar * 10)


def test_augmented_lagrangian_start_field():
    """A start field takes the place of E in d and e (lam = k d): three
    iterations from the field of two accelerated iterations, voxel by voxel."""
    print("\n[case] augmented lagrangian start field", flush=True)
    ph = geom.random_phases(24, 91)
    init = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=2, want_field=True).field
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=3, want_field=True,
                            init_field=init, scheme=2)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=3, precision=1, want_field=True,
                          init_field=init, scheme=AL)
    assert field_err(g.field, ref.field) <= 1e-11
    assert tensor_err(g.K, ref.K) <= 1e-11


def test_augmented_lagrangian_converged_fp64_vs_oracle():
    """32^3, 8 RSA spheres, f = 0.2, l = 0.1, seed 1, tol 1e-6, FP64: the
    augmented-Lagrangian tensor within 1e-9 of the oracle's, same iteration
    counts and residual histories."""
    print("\n[case] augmented lagrangian converged fp64", flush=True)
    ph, _, _ = geom.generate(32, 8, 0.2, 0.1, 1)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=1e-6, scheme=2)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 1e-6, precision=1, hist_cap=1000, scheme=AL)
    assert g.status == rh.RVE_OK
    assert list(g.iters) == list(ref.iters)
    assert tensor_err(g.K, ref.K) <= 1e-9
    for j in range(3):
        np.testing.assert_allclose(g.history[j], ref.history[j], rtol=1e-9)


@pytest.mark.parametrize("precision", [0, 1])
def test_augmented_lagrangian_config2_128(precision):
    """The benchmark workload with the augmented-Lagrangian scheme (in the
    load-case chains bench.py uses): the same discrete solution as the stored
    oracle tensor of the accelerated scheme, within the FP32 bar (FP64:
    1e-5, the two stop at tol 1e-6 on different residuals), after more
    iterations than the accelerated scheme."""
    print(f"\n[case] augmented lagrangian config2 128 precision={precision}", flush=True)
    ref = _golden("rve128_50sph_f0.30_l0.20_seed2")
    g0 = ref["geometry"]
    with rh.rve_create(g0["n"], g0["n_spheres"], g0["volume_fraction"], g0["layer"],
                       g0["seed"]) as r:
        g = rh.homogenize(r, ref["k_phases"], ref["tol"], precision=precision, scheme=AL)
    assert g.status == rh.RVE_OK  # FP32: with the FP64 continuation past its floor
    assert tensor_err(g.K, np.array(ref["K"])) <= (1e-4 if precision == 0 else 1e-5)
    assert int(min(g.iters)) > max(ref["iters"])


def test_augmented_lagrangian_256_split_and_five_pass():
    """256^3 with the augmented-Lagrangian update: in the fused passes
    (split planes with the parity layout in FP32, quarter planes in FP64)
    and in the five-pass form's inverse pass (FP64, flags 2).  Two
    iterations of load case e_1 on an RSA RVE, voxel by voxel against the
    oracle."""
    print("\n[case] augmented lagrangian 256", flush=True)
    ph, _, _ = geom.generate(256, 100, 0.3, 0.2, 3)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=2, want_field=True, lc_mask=1, scheme=2)
    with rh.rve_create_from_phases(ph) as r:
        for prec, bar, flags in ((0, 3e-5, 0), (1, 1e-11, 0), (1, 1e-11, 2)):
            print(f"[case] augmented lagrangian 256 precision={prec} flags={flags}", flush=True)
            g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=2, precision=prec, lc_mask=1,
                              want_field=True, hist_cap=4, scheme=AL, path_flags=flags)
            assert field_err(g.field[0], ref.field[0]) <= bar
            assert tensor_err(g.K[:, 0], ref.K[:, 0]) <= bar
            for j in range(2):
                np.testing.assert_allclose(g.history[0][j], ref.history[0][j], rtol=bar * 10)


def test_augmented_lagrangian_fused_equals_separate_passes():
    """The fused pass and the separate forward / inverse passes carry the same
    augmented-Lagrangian iteration: FP64 tensors and iteration counts agree."""

    print("\n[case] augmented lagrangian fused vs separate", flush=True)
    ph, _, _ = geom.generate(64, 12, 0.3, 0.2, 41)
    with rh.rve_create_from_phases(ph) as r:
        fused = rh.homogenize(r, K_PAPER_CFG, 1e-8, precision=1, scheme=AL)
        sep = rh.homogenize(r, K_PAPER_CFG, 1e-8, precision=1, scheme=AL, path_flags=rh.PATH_NO_FUSED)
    assert np.array_equal(fused.iters, sep.iters)
    assert tensor_err(sep.K, fused.K) <= 1e-12


def test_augmented_lagrangian_rejections():
    """The equilibrium check and unknown schemes are refused before any work."""
    print("\n[case] augmented lagrangian rejections", flush=True)
    with rh.rve_create_from_phases(geom.random_phases(16, 5)) as r:
        with pytest.raises(rh.RveError):
            rh.homogenize(r, K_PAPER_CFG, 1e-6, precision=1, scheme=AL, equilibrium_check=True)
        with pytest.raises(rh.RveError):
            rh.homogenize(r, K_PAPER_CFG, 1e-6, precision=1, scheme=5)
        ok = rh.homogenize(r, K_PAPER_CFG, 1e-6, precision=1, scheme=AL)
        assert ok.status == rh.RVE_OK


@pytest.mark.parametrize("precision", [1, 0])
def test_fibers_fixed_iterations_vs_oracle(precision):
    """Aligned coated fibres (cylindrical inclusions, Sec. 6): three
    iterations from E, voxel by voxel against the oracle."""
    print(f"\n[case] fibres fixed iterations precision={precision}", flush=True)
    ph, _, _ = geom.generate_fibers(48, 10, 0.35, 0.2, 6)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=3, want_field=True)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=3, precision=precision, want_field=True)
    bar = 1e-11 if precision == 1 else 3e-5
    assert field_err(g.field, ref.field) <= bar
    assert tensor_err(g.K, ref.K) <= bar


@pytest.mark.parametrize("precision", [1, 0])
def test_fibers_128_axial_exact(precision):
    """128^3, 40 coated fibres along z, f = 0.4, l = 0.2: the axial load case
    converges in one iteration to K_33 = <k> (closed form), K_13 = K_23 = 0;
    the transverse tensor agrees between precisions within the FP32 bar."""
    print(f"\n[case] fibres 128 axial precision={precision}", flush=True)
    ph, _, _ = geom.generate_fibers(128, 40, 0.4, 0.2, 8)
    k = np.array([1.0, 0.2, 400.0])
    kmean = k[ph].mean()
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, k, 1e-6, precision=precision)
        g64 = g if precision == 1 else rh.homogenize(r, k, 1e-6, precision=1)
    assert int(g.iters[2]) == 1
    assert abs(g.K[2, 2] - kmean) <= (1e-12 if precision == 1 else 1e-6) * kmean
    assert np.abs(g.K[:2, 2]).max() <= 1e-6 * kmean
    assert tensor_err(g.K, g64.K) <= 1e-4


def test_mixed_inclusions_fixed_iterations_vs_oracle():
    """Spheres and fibres in one cell: three FP64 iterations, voxel by voxel."""
    print("\n[case] mixed inclusions", flush=True)
    ph = geom.generate_mixed(48, 6, 0.1, 5, 0.15, 0.2, 9)
    ref = oracle.homogenize(ph, K_PAPER_CFG, tol=0.0, max_iter=3, want_field=True)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_PAPER_CFG, 0.0, max_iter=3, precision=1, want_field=True)
    assert field_err(g.field, ref.field) <= 1e-11
    assert tensor_err(g.K, ref.K) <= 1e-11
