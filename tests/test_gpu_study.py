"""The paper's stochastic study (Sec. 5) through the batched GPU path: the
qualitative trends the paper reports (no curve values are printed)."""
import numpy as np
import pytest

import oracle
from paper_1504_07499_amd import geom, study

pytestmark = pytest.mark.gpu


def test_isotropic_conductivity_grows_with_layer():
    """Sec. 5: the homogenized conductivity increases with the layer l, with
    the coating (400) far better conducting than matrix (1) and inclusions
    (0.2)."""
    print("\n[case] study trend", flush=True)
    rows = [study.run_set(64, 30, layer, 3) for layer in (0.05, 0.2, 0.5)]
    vals = [r["k_iso_mean"] for r in rows]
    assert vals[0] < vals[1] < vals[2]
    for r in rows:
        assert all(s == 0 for s in r["status"])
        assert r["k_iso_std"] < 0.5 * r["k_iso_mean"]


def test_study_set_matches_oracle():
    """One set of the study (batched, FP32 with the FP64 continuation): each
    sample's tensor against the FP64 oracle on the same seeded phases."""
    print("\n[case] study set vs oracle", flush=True)
    row = study.run_set(32, 30, 0.2, 2)
    for seed, K in zip(row["seeds"], row["K"]):
        ph, _, _ = geom.generate(32, 30, 0.3, 0.2, seed)
        ref = oracle.homogenize(ph, study.PAPER_K, tol=1e-5)
        K = np.array(K)
        assert np.abs(K - ref.K).max() / np.abs(ref.K).max() <= 1e-4
