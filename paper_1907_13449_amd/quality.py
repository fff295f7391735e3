"""Accuracy measures of Sec. 4.2 against synthetic ground truth: BadPix (the
percentage of pixels whose absolute disparity error exceeds a threshold, 0.07 in
the paper), the mean squared error, and the M-metric of Eq. (14) (percentage of
correct pixels per second of runtime).  Host-side numpy on finished maps; used
by bench.py to compare the bounded search with the boundary-less one."""
from __future__ import annotations

import numpy as np


def _crop(a, border):
    a = np.asarray(a, dtype=np.float64)
    return a[border:a.shape[0] - border, border:a.shape[1] - border] if border else a


def badpix(disp, gt, thr: float = 0.07, border: int = 0) -> float:
    """Percentage of pixels with |disp - gt| > thr (inside `border` pixels)."""
    err = np.abs(_crop(disp, border) - _crop(gt, border))
    return float(100.0 * np.mean(err > thr))


def mse(disp, gt, border: int = 0) -> float:
    """Mean squared disparity error (inside `border` pixels)."""
    d = _crop(disp, border) - _crop(gt, border)
    return float(np.mean(d * d))


def m_metric(badpix_pct: float, runtime_s: float) -> float:
    """Eq. (14): (100 % - BadPix) / runtime, in percent per second."""
    return (100.0 - badpix_pct) / runtime_s
