"""homogenize_no_alloc (the entry point for callers that cannot allocate)
against homogenize, through the C ABI: the same kernels in the same order,
so the same tensors, iteration counts and residual histories; two calls in
a row on the shared scratch array, the second on a smaller grid; grids whose
workspaces exceed the array are refused."""
import numpy as np
import pytest

import paper_1504_07499_amd as rh
from paper_1504_07499_amd import geom

pytestmark = pytest.mark.gpu

K3 = np.array([0.2, 0.3, 400.0])


def _same(a, b):
    assert a.status == b.status, (a.lc_status, b.lc_status)
    assert np.array_equal(a.K, b.K), np.abs(a.K - b.K).max()
    assert np.array_equal(a.iters, b.iters) and np.array_equal(a.refine_iters, b.refine_iters)
    assert np.array_equal(a.lc_status, b.lc_status)
    assert np.array_equal(a.final_residual, b.final_residual)
    for j in range(3):
        np.testing.assert_array_equal(a.history[j], b.history[j])


@pytest.mark.parametrize("precision,scheme", [(0, "accelerated"), (1, "accelerated"),
                                              (0, "augmented_lagrangian"), (0, "dual"), (1, "polarization")])
def test_no_alloc_equals_homogenize_two_calls(precision, scheme):
    print(f"\n[case] no-alloc precision={precision} scheme={scheme}", flush=True)
    for n, nsp, seed in ((64, 12, 51), (32, 8, 52)):  # second call: smaller grid
        ph, _, _ = geom.generate(n, nsp, 0.3, 0.2, seed)
        with rh.rve_create_from_phases(ph) as r:
            ref = rh.homogenize(r, K3, 1e-6, precision=precision, scheme=scheme, hist_cap=2048)
            got = rh.homogenize_no_alloc(r, K3, 1e-6, precision=precision, scheme=scheme, hist_cap=2048)
        print(n, list(got.iters), list(got.refine_iters), flush=True)
        _same(got, ref)


def test_no_alloc_partial_load_cases_and_refine_off():
    print("\n[case] no-alloc lc_mask / refine off", flush=True)
    ph, _, _ = geom.generate(48, 10, 0.25, 0.1, 53)
    with rh.rve_create_from_phases(ph) as r:
        for kw in ({"lc_mask": 5}, {"fp32_refine": False}, {"lc_mask": 2, "precision": 1}):
            ref = rh.homogenize(r, K3, 1e-6, hist_cap=1024, **kw)
            got = rh.homogenize_no_alloc(r, K3, 1e-6, hist_cap=1024, **kw)
            _same(got, ref)


def test_no_alloc_rejects_grids_beyond_the_array():
    print("\n[case] no-alloc size limit", flush=True)
    with rh.rve_create(128, 20, 0.2, 0.2, 54) as r:
        with pytest.raises(rh.RveError) as ei:
            rh.homogenize_no_alloc(r, K3, 1e-6)
        assert ei.value.status == rh.RVE_ERR_ARG
        assert "scratch" in str(ei.value)
