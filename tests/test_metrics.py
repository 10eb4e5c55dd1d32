"""Host-side normal-quality metrics (Sec. 5.1.4) on hand values."""
import numpy as np
import pytest


def test_metrics_by_hand():
    """AE_pcd and P_co on hand values: same, opposite and perpendicular
    normals; unnormalized inputs; rows without a reference are left out."""
    from paper_2405_16634_amd.metrics import ae_pcd, flip_rate, p_co
    gt = np.array([[0, 0, 1.0], [0, 0, 1.0], [1.0, 0, 0], [np.nan, np.nan, np.nan]])
    n = np.array([[0, 0, 3.0], [0, 0, -1.0], [0, 2.0, 0], [1.0, 0, 0]])
    assert ae_pcd(n, gt) == pytest.approx((0.0 + 1.0 + 0.5) / 3)
    assert p_co(n, gt) == pytest.approx(1 / 3)
    assert flip_rate(n, gt) == pytest.approx(2 / 3)
    assert p_co(n, gt, mask=[True, False, False, True]) == 1.0
