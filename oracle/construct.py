"""Analytical Gaussian construction from kept coefficients (Sec. 4.3).  Test infrastructure.

For a kept coefficient at packed index idx = (j, o, k):
  * p = |A_{j,o,k,:}| * w_{j,o}                              (eq. per_location_weight)
  * amplitude s_j * p with s_j = 2^{-3j/2}                      (eq. wavelet_gaussian_kernel)
  * centre u_{j,o} + 2^j k + delta, delta = 1/2 per axis         (eq. translation_operator,
    eq. gaussian_covariation; delta read as the index -> cell-centre offset of the embedding into R^3)
  * covariance Sigma_{j,o}, shared by the whole subband.
World coordinates: the volume occupies [-1, 1]^3 with voxel i spanning [-1 + h i, -1 + h (i+1)],
h = 2/G, so mean_world = -1 + h * centre_idx and scale_world = h * scale_idx.
Amplitude -> 3DGS parameters: opacity = clamp(amp_alpha, 1e-3, 0.99), rgb = clamp(amp_rgb, 0, 1).
``s_mode`` = "paper" applies s_j literally; "none" drops it (the paper's w already carries the
2^{-3j/2} decay of an orthonormal transform, so the literal factor attenuates twice).

Ablation variants (Sec. 5, ablation studies):
  * ``isotropic``: without the transition bank's covariances every Gaussian gets sigma_iso^2 I
    (scales all sigma_iso, identity rotation) with sigma_iso the average spatial extent of the full
    model, read as the mean over the built Gaussians of the mean of their three full-model scales;
  * ``unit_weight``: without the energy projection, w_{j,o} = 1.
"""
from __future__ import annotations

import numpy as np

from . import dwt as _dwt


def construct(coeffs: np.ndarray, kept: np.ndarray, G: int, J: int, bank: list, s_mode: str = "paper",
              delta: float = 0.5, isotropic: bool = False, unit_weight: bool = False):
    """coeffs [4][G^3] packed, kept [K] packed indices, bank in packed block order.

    Returns a dict of FP64 arrays: means [3][K], scales [3][K], quats [4][K], opacity [K], rgb [3][K].
    """
    offs = _dwt.block_offsets(G, J)
    order = _dwt.block_order(J)
    starts = np.array([offs[b][0] for b in order])
    kept = np.asarray(kept, dtype=np.int64)
    blk = np.searchsorted(starts, kept, side="right") - 1
    h = 2.0 / G
    K = kept.shape[0]
    means = np.empty((3, K))
    scales = np.empty((3, K))
    quats = np.empty((4, K))
    opacity = np.empty(K)
    rgb = np.empty((3, K))
    A = np.abs(np.asarray(coeffs, dtype=np.float64)[:, kept])   # [4][K]
    for b, (j, o) in enumerate(order):
        sel = blk == b
        if not np.any(sel):
            continue
        e = bank[b]
        assert (e.j, e.o) == (j, o)
        off, n = offs[(j, o)]
        r = kept[sel] - off
        k = np.stack([r % n, (r // n) % n, r // (n * n)])       # (kx, ky, kz)
        centre = e.u[:, None] + (1 << j) * k + delta
        means[:, sel] = -1.0 + h * centre
        scales[:, sel] = h * e.scale[:, None]
        quats[:, sel] = e.quat[:, None]
        s = 2.0 ** (-1.5 * j) if s_mode == "paper" else 1.0
        amp = s * A[:, sel] * (1.0 if unit_weight else e.w)
        rgb[:, sel] = np.clip(amp[:3], 0.0, 1.0)
        opacity[sel] = np.clip(amp[3], 1e-3, 0.99)
    if isotropic and K > 0:
        sigma_iso = np.mean(scales.mean(axis=0))
        scales[:] = sigma_iso
        quats[:] = np.array([1.0, 0.0, 0.0, 0.0])[:, None]
    return dict(means=means, scales=scales, quats=quats, opacity=opacity, rgb=rgb)
