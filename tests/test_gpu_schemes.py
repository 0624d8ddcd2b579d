"""GPU parity of the dual and polarization schemes named in Sec. 3 (their
equations come from the cited works; the readings are those of the oracle):
fields voxel by voxel after a few iterations on every grid path, converged
tensors and iteration counts, the fused pass against the separate passes,
and the special cases of the polarization relaxation."""
import numpy as np
import pytest

import oracle
import paper_1504_07499_amd as rh
from paper_1504_07499_amd import geom

pytestmark = pytest.mark.gpu

K_CFG = np.array([0.2, 0.3, 400.0])
K_LOW = np.array([0.2, 0.3, 4.0])  # contrast 20: the dual scheme converges at the basic rate


def tensor_err(K, Kref):
    return float(np.abs(K - Kref).max() / np.abs(Kref).max())


def field_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("n", [8, 12, 24, 48, 64, 96, 128])
@pytest.mark.parametrize("scheme,alpha", [(3, 0.0), (4, 1.5)])
def test_fixed_iterations_vs_oracle(scheme, alpha, n, precision):
    """Four iterations from the start: the iterate (flux or polarization) of
    every voxel of every channel, the tensor and the residual history."""
    print(f"\n[case] scheme {scheme} n={n} precision={precision}", flush=True)
    ph = geom.random_phases(n, seed=500 + n)
    ref = oracle.homogenize(ph, K_CFG, tol=0.0, max_iter=4, want_field=True, scheme=scheme,
                            alpha=alpha if alpha else 2.0)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, K_CFG, 0.0, max_iter=4, precision=precision, want_field=True, hist_cap=8,
                          scheme=scheme, alpha=alpha)
    bar = 1e-11 if precision == 1 else 3e-5
    assert field_err(g.field, ref.field) <= bar
    assert tensor_err(g.K, ref.K) <= bar
    assert list(g.iters) == [4, 4, 4]
    for j in range(3):
        np.testing.assert_allclose(g.history[j], ref.history[j], rtol=bar * 10)


@pytest.mark.parametrize("scheme,alpha,k", [(3, 0.0, K_LOW), (4, 1.5, K_CFG)])
def test_converged_vs_oracle(scheme, alpha, k):
    """32^3, 8 RSA spheres, f = 0.2, l = 0.1, seed 1, tol 1e-6: FP64 within
    1e-9 of the oracle with the same iteration counts; FP32 (with the FP64
    continuation) within 1e-4."""
    print(f"\n[case] scheme {scheme} converged", flush=True)
    ph, _, _ = geom.generate(32, 8, 0.2, 0.1, 1)
    ref = oracle.homogenize(ph, k, tol=1e-6, scheme=scheme, alpha=alpha if alpha else 2.0)
    with rh.rve_create_from_phases(ph) as r:
        g = rh.homogenize(r, k, 1e-6, precision=1, scheme=scheme, alpha=alpha)
        f = rh.homogenize(r, k, 1e-6, precision=0, scheme=scheme, alpha=alpha)
    assert g.status == rh.RVE_OK and f.status == rh.RVE_OK
    assert list(g.iters) == list(ref.iters)
    assert tensor_err(g.K, ref.K) <= 1e-9
    assert tensor_err(f.K, ref.K) <= 1e-4
    assert np.all(g.eps_eq == -1)


@pytest.mark.parametrize("scheme,alpha", [(3, 0.0), (4, 1.5)])
def test_256_split_and_five_pass(scheme, alpha):
    """256^3: split planes with the parity-layout fused pass in FP32,
    quarter planes with the four-quarter z pass in FP64, and the five-pass
    form in FP64 (flags 2).  Two iterations of load case e_1 on an RSA RVE,
    voxel by voxel against the oracle."""
    print(f"\n[case] scheme {scheme} 256", flush=True)
    ph, _, _ = geom.generate(256, 100, 0.3, 0.2, 3)
    ref = oracle.homogenize(ph, K_CFG, tol=0.0, max_iter=2, want_field=True, lc_mask=1, scheme=scheme,
                            alpha=alpha if alpha else 2.0)
    with rh.rve_create_from_phases(ph) as r:
        for prec, bar, flags in ((0, 3e-5, 0), (1, 1e-11, 0), (1, 1e-11, 2)):
            g = rh.homogenize(r, K_CFG, 0.0, max_iter=2, precision=prec, lc_mask=1, want_field=True,
                              hist_cap=4, scheme=scheme, alpha=alpha, path_flags=flags)
            assert field_err(g.field[0], ref.field[0]) <= bar
            assert tensor_err(g.K[:, 0], ref.K[:, 0]) <= bar


@pytest.mark.parametrize("scheme,alpha", [(3, 0.0), (4, 1.5)])
def test_fused_equals_separate_passes(scheme, alpha):
    print(f"\n[case] scheme {scheme} fused vs separate", flush=True)
    ph, _, _ = geom.generate(64, 12, 0.3, 0.2, 41)
    with rh.rve_create_from_phases(ph) as r:
        fused = rh.homogenize(r, K_LOW, 1e-8, precision=1, scheme=scheme, alpha=alpha)
        sep = rh.homogenize(r, K_LOW, 1e-8, precision=1, scheme=scheme, alpha=alpha,
                            path_flags=rh.PATH_NO_FUSED)
    assert np.array_equal(fused.iters, sep.iters)
    assert tensor_err(sep.K, fused.K) <= 1e-12


def test_polarization_special_cases():
    """alpha = 1 runs the augmented-Lagrangian kernels with the same step
    (bitwise the same result); the default alpha is 2."""
    print("\n[case] polarization special cases", flush=True)
    ph, _, _ = geom.generate(48, 10, 0.25, 0.2, 9)
    with rh.rve_create_from_phases(ph) as r:
        al = rh.homogenize(r, K_CFG, 1e-6, precision=1, scheme="augmented_lagrangian")
        p1 = rh.homogenize(r, K_CFG, 1e-6, precision=1, scheme="polarization", alpha=1.0)
        p2 = rh.homogenize(r, K_CFG, 1e-6, precision=1, scheme="polarization")
        p2b = rh.homogenize(r, K_CFG, 1e-6, precision=1, scheme="polarization", alpha=2.0)
    assert np.array_equal(al.K, p1.K) and np.array_equal(al.iters, p1.iters)
    assert np.array_equal(p2.K, p2b.K) and np.array_equal(p2.iters, p2b.iters)
    assert np.all(p2.iters < al.iters)


def test_rejections():
    print("\n[case] scheme rejections", flush=True)
    n = 16
    with rh.rve_create_from_phases(geom.random_phases(n, 5)) as r:
        init = np.zeros((3, 3, n, n, n))
        for kw in ({"scheme": "dual", "init_field": init}, {"scheme": "dual", "equilibrium_check": True},
                   {"scheme": "polarization", "alpha": 2.5}, {"scheme": "polarization", "alpha": -1.0},
                   {"scheme": "polarization", "equilibrium_check": True}):
            with pytest.raises(rh.RveError) as ei:
                rh.homogenize(r, K_CFG, 1e-6, precision=1, **kw)
            assert ei.value.status == rh.RVE_ERR_ARG


@pytest.mark.parametrize("precision", [1, 0])
def test_scheme_switches_on_one_handle(precision):
    """Solves of different schemes one after another on one RVE handle (the
    solvers, workspaces and cached iteration graphs are reused) give what
    each scheme gives on a fresh handle, bit for bit: the cached graphs are
    keyed by the scheme's update kernels."""
    print(f"\n[case] scheme switches precision={precision}", flush=True)
    ph, _, _ = geom.generate(32, 8, 0.2, 0.1, 1)
    order = [("accelerated", 0.0), ("dual", 0.0), ("augmented_lagrangian", 0.0), ("dual", 0.0),
             ("polarization", 1.5), ("accelerated", 0.0), ("basic", 0.0), ("dual", 0.0)]
    fresh = {}
    for sch, alpha in set(order):
        with rh.rve_create_from_phases(ph) as r:
            fresh[sch] = rh.homogenize(r, K_LOW, 1e-6, precision=precision, scheme=sch, alpha=alpha)
    with rh.rve_create_from_phases(ph) as r:
        for sch, alpha in order:
            g = rh.homogenize(r, K_LOW, 1e-6, precision=precision, scheme=sch, alpha=alpha)
            assert g.status == rh.RVE_OK, sch
            assert list(g.iters) == list(fresh[sch].iters), sch
            assert np.array_equal(g.K, fresh[sch].K), sch
