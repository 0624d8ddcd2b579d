"""The paper's stochastic study (Sec. 5) through the batched GPU path: the
qualitative trends the paper reports (no curve values are printed)."""
import numpy as np
import pytest

from paper_1504_07499_amd import study

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
        assert all(s in (0, 2) for s in r["status"])
        assert r["k_iso_std"] < 0.5 * r["k_iso_mean"]
