"""Transfer function RF = TF(F) (Sec. 3, Transfer Function).  Test infrastructure.

The paper leaves the form of TF open; the workloads use a piecewise-linear map from a scalar in
[0, 1] to RGBA through ascending control points, held constant beyond the end points.
"""
from __future__ import annotations

import numpy as np


def apply(F: np.ndarray, xs: np.ndarray, rgba: np.ndarray) -> np.ndarray:
    """F [..] (already normalised to [0, 1]) -> RGBA [4][..] in FP64 by linear interpolation."""
    F = np.asarray(F, dtype=np.float64)
    xs = np.asarray(xs, dtype=np.float64)
    rgba = np.asarray(rgba, dtype=np.float64)
    return np.stack([np.interp(F, xs, rgba[:, c]) for c in range(4)])
