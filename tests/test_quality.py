"""The accuracy measures of Sec. 4.2 and Eq. (14) on hand-made maps."""
import numpy as np

from paper_1907_13449_amd import quality


def test_badpix_counts_errors_above_the_threshold():
    gt = np.zeros((2, 4))
    d = np.array([[0.0, 0.07, 0.0701, -0.5], [0.01, -0.07, 0.2, 0.0]])
    # 0.07 itself is not bad (strictly greater); 0.0701, -0.5 and 0.2 are
    assert quality.badpix(d, gt) == 100.0 * 3 / 8
    assert quality.badpix(d, gt, thr=0.3) == 100.0 * 1 / 8


def test_mse_and_border_crop():
    gt = np.zeros((4, 4))
    d = np.full((4, 4), 3.0)
    d[1:3, 1:3] = 1.0
    assert quality.mse(d, gt) == (12 * 9 + 4 * 1) / 16
    assert quality.mse(d, gt, border=1) == 1.0
    assert quality.badpix(d, gt, border=1) == 100.0


def test_m_metric():
    assert quality.m_metric(10.0, 2.0) == 45.0
    assert quality.m_metric(0.0, 0.5) == 200.0
