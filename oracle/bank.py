"""Wavelet-to-Gaussian Transition Bank (Sec. 4.2).  Test infrastructure.

For each subband (j, o) -- the seven detail orientations of every level j = 1..J plus the final
LLL at j = J, i.e. 7J + 1 entries (the paper's count "8(J+1)" is read as this) -- the oracle:

1. builds the canonical wavelet psi_{j,o} = W^{-1}[e_{j,o,0}] (eq. wavelet_impulse,
   eq. canonical_wavelet).  The 3D transform is a tensor product of 1D transforms and the levels
   below j only apply low-pass synthesis on every axis, so psi_{j,o} is exactly the outer product
   of 1D impulse responses r_{j,o_x} (x) r_{j,o_y} (x) r_{j,o_z}; each 1D response is synthesised
   on a periodic line long enough that nothing wraps.
2. normalises W = |psi| / sum |psi| and keeps the region of interest W > tau * max W (eq. roi);
3. takes the W-weighted centroid u and covariance Sigma over the ROI (eq. moment) in voxel-index
   units relative to the impulse's origin 2^j k;
4. fits the amplitude w by ridge regression of |Y| on the Gaussian G of eq. canonical_gaussian
   sampled on the ROI: w = <G, |Y|> / (<G, G> + lambda) (eq. ridge_regression);
5. factors Sigma = R diag(scale^2) R^T.  When Sigma is diagonal (always the case for the symmetric
   filter banks here) R = I and scale = sqrt(diag Sigma) in (x, y, z) order; otherwise the
   eigenvectors (ascending eigenvalues, det +1) give R, returned as a unit quaternion (w >= 0).

tau and lambda are not given in the paper: tau = 0.1 and lambda = 1e-8 by default.
The bior4.4 values of (u, Sigma, w) have no printed counterpart: parity unpinned.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import dwt as _dwt
from . import wavelets


@dataclasses.dataclass
class BankEntry:
    j: int
    o: int
    w: float
    u: np.ndarray        # (3,) x, y, z voxel-index units relative to 2^j k
    sigma: np.ndarray    # (3, 3)
    scale: np.ndarray    # (3,)
    quat: np.ndarray     # (4,) w, x, y, z
    roi_size: int


def response_1d(bank: wavelets.FilterBank, j: int, band: str, n_coarse: int = 64):
    """1D impulse response of a level-j coefficient in band 'L' or 'H'.

    Returns (values, rel) where rel[i] is the sample position relative to the impulse origin 2^j k.
    """
    n = n_coarse
    k0 = n // 2
    lo = np.zeros(n)
    hi = np.zeros(n)
    (lo if band == "L" else hi)[k0] = 1.0
    cur = _dwt.synthesis_1d(lo, hi, bank, axis=0)
    for _ in range(j - 1):
        cur = _dwt.synthesis_1d(cur, np.zeros_like(cur), bank, axis=0)
    nz = np.nonzero(cur)[0]
    lo_i, hi_i = nz[0], nz[-1] + 1
    assert lo_i > 0 and hi_i < len(cur), "impulse response wrapped around the periodic line"
    rel = np.arange(lo_i, hi_i) - (1 << j) * k0
    return cur[lo_i:hi_i], rel


def canonical_wavelet(wavelet: str, j: int, o: int):
    """psi_{j,o} as a 3D array [z][y][x] plus per-axis relative coordinates (x, y, z)."""
    bank = wavelets.get(wavelet)
    r = []
    for d in range(3):
        band = "H" if (o >> d) & 1 else "L"
        r.append(response_1d(bank, j, band))
    (rx, cx), (ry, cy), (rz, cz) = r
    psi = rz[:, None, None] * ry[None, :, None] * rx[None, None, :]
    return psi, (cx, cy, cz)


def quat_from_rotation(R: np.ndarray) -> np.ndarray:
    """Unit quaternion (w, x, y, z), w >= 0, of a proper rotation matrix (Shepperd's method)."""
    t = np.trace(R)
    if t > 0:
        s = np.sqrt(t + 1.0) * 2
        q = np.array([0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s])
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        q = np.array([(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s])
    elif R[1, 1] > R[2, 2]:
        s = np.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        q = np.array([(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s])
    else:
        s = np.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        q = np.array([(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s])
    q = q / np.linalg.norm(q)
    return -q if q[0] < 0 else q


def factor_covariance(S: np.ndarray):
    """Sigma -> (scale, quat) with Sigma = R(quat) diag(scale^2) R(quat)^T."""
    off = max(abs(S[0, 1]), abs(S[0, 2]), abs(S[1, 2]))
    if off <= 1e-12 * np.max(np.abs(np.diag(S))):
        return np.sqrt(np.diag(S)), np.array([1.0, 0.0, 0.0, 0.0])
    evals, evecs = np.linalg.eigh(S)
    if np.linalg.det(evecs) < 0:
        evecs[:, 0] = -evecs[:, 0]
    return np.sqrt(evals), quat_from_rotation(evecs)


def fit_entry(psi: np.ndarray, coords, tau: float, lam: float):
    """Dominant-lobe estimation + ridge weight for one canonical wavelet.  Returns (u, Sigma, w, roi)."""
    cx, cy, cz = coords
    a = np.abs(psi)
    W = a / a.sum()
    roi = W > tau * W.max()
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    pts = np.stack([X[roi], Y[roi], Z[roi]], axis=1).astype(np.float64)   # (n, 3) as (x, y, z)
    wts = W[roi]
    sw = wts.sum()
    u = (wts[:, None] * pts).sum(0) / sw
    d = pts - u
    Sigma = (wts[:, None, None] * d[:, :, None] * d[:, None, :]).sum(0) / sw
    Sinv = np.linalg.inv(Sigma)
    g = np.exp(-0.5 * np.einsum("ni,ij,nj->n", d, Sinv, d))
    yv = a[roi]
    w = float(g @ yv) / (float(g @ g) + lam)
    return u, Sigma, w, int(roi.sum())


def build_bank(wavelet: str, J: int, tau: float = 0.1, lam: float = 1e-8) -> list:
    """All 7J+1 entries, in the packed block order [(J,0), (J,1..7), (J-1,1..7), ..., (1,1..7)]."""
    out = []
    for (j, o) in _dwt.block_order(J):
        psi, coords = canonical_wavelet(wavelet, j, o)
        u, Sigma, w, nroi = fit_entry(psi, coords, tau, lam)
        scale, quat = factor_covariance(Sigma)
        out.append(BankEntry(j=j, o=o, w=w, u=u, sigma=Sigma, scale=scale, quat=quat, roi_size=nroi))
    return out
