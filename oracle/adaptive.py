"""Adaptive per-subband coefficient selection (Supp. A: global budget allocation across subbands,
joint multi-channel sparsification, robust MAD-based thresholding, top-K selection under sparsity
constraints).  Test infrastructure: plain numpy, used only by the tests and the benchmark's CPU leg.

For each subband (j, o) of the packed layout (the LLL block is one subband like the detail blocks):
  E = sum_k |A_{j,o,k,c_ref}|^2, N = #k, S = E^alpha N^beta,
  K_{j,o} = max(min_band, floor(K_tot S / sum S))                        (global budget allocation)
  v(k) = |A_{j,o,k,:}|_2 over R, G, B, A                                  (joint magnitude)
  MAD = median_k |v(k) - median(v)|, sigma = MAD / 0.6745, T = lambda sigma
  C = {k : v(k) >= T}, K = min(K_{j,o}, |C|), v_(K) = K-th largest v in C
  keep k  <=>  v(k) >= max(T, v_(K))                                      (none when K = 0)

Readings where the supplement is silent or loose (each one also in the design notes):
  * alpha, beta and lambda are not given: parameters, defaults alpha = beta = 1/2 (S = sqrt(E N),
    N times the subband's RMS reference amplitude: with alpha = 1, beta = 0 the LLL block, which
    holds most of the energy in few locations, would absorb nearly the whole budget) and lambda = 3
    (a three-sigma noise floor);
  * c_ref is the opacity channel (index 3), the supplement's typical choice;
  * the median of an even count is the mean of the two middle order statistics;
  * v, |v - median|, the medians, sigma and T are float32, evaluated in a fixed order, so that both
    sides take every keep/drop decision in the same precision (v in the order of the top-K key);
    E, S and the budget quotient are float64 (sum S = 0 gives quotient 0);
  * keep means v >= max(T, v_(K)) literally: values tied with v_(K) are all kept, so a subband can
    keep more than K;
  * the per-band minimum can push the total over K_tot (the supplement's bound fails then); it is
    kept as written.
"""
from __future__ import annotations

import numpy as np

from .dwt import block_offsets
from .select import joint_norm_f32

DEFAULTS = dict(alpha=0.5, beta=0.5, lam=3.0, ref=3, min_band=10)
_HALF = np.float32(0.5)
_MAD_TO_SIGMA = np.float32(0.6745)


def bands(G: int, J: int) -> list:
    """[(j, o, offset, count)] in packed order."""
    return [(j, o, off, n ** 3) for (j, o), (off, n) in block_offsets(G, J).items()]


def median_f32(x: np.ndarray) -> np.float32:
    """Median of a float32 array: the middle order statistic, or for an even count the mean of the
    two middle ones, (a + b) * 0.5 in float32."""
    s = np.sort(np.asarray(x, dtype=np.float32))
    n = s.shape[0]
    lo, hi = s[(n - 1) // 2], s[n // 2]
    return np.float32(np.float32(lo + hi) * _HALF)


def energies(coeffs: np.ndarray, G: int, J: int, ref: int = 3) -> np.ndarray:
    """E per subband: sum of squares of the reference channel, float64."""
    a = np.asarray(coeffs[ref], dtype=np.float64)
    return np.array([np.sum(a[off:off + n] ** 2) for (_, _, off, n) in bands(G, J)])


def budget_quotients(E: np.ndarray, N: np.ndarray, K_tot: int, alpha: float, beta: float) -> np.ndarray:
    """K_tot S / sum S with S = E^alpha N^beta (float64)."""
    S = np.power(np.asarray(E, np.float64), alpha) * np.power(np.asarray(N, np.float64), beta)
    tot = S.sum()
    return np.zeros_like(S) if tot == 0.0 else K_tot * S / tot


def budgets(E: np.ndarray, N: np.ndarray, K_tot: int, alpha: float, beta: float, min_band: int) -> np.ndarray:
    return np.maximum(min_band, np.floor(budget_quotients(E, N, K_tot, alpha, beta))).astype(np.int64)


def band_filter(v: np.ndarray, K_band: int, lam: float) -> dict:
    """The MAD threshold and capped top-K of one subband's joint norms (float32)."""
    v = np.asarray(v, dtype=np.float32)
    med = median_f32(v)
    mad = median_f32(np.abs(v - med))
    sigma = np.float32(mad / _MAD_TO_SIGMA)
    T = np.float32(np.float32(lam) * sigma)
    C = int(np.count_nonzero(v >= T))
    K = min(int(K_band), C)
    if K >= 1:
        vK = np.sort(v)[v.shape[0] - K]
        keep = v >= max(T, vK)
    else:
        vK = np.float32(np.inf)
        keep = np.zeros(v.shape[0], dtype=bool)
    return dict(median=med, mad=mad, sigma=sigma, T=T, C=C, K=K, vK=np.float32(vK), keep=keep)


def select(coeffs: np.ndarray, G: int, J: int, K_tot: int, alpha: float = DEFAULTS["alpha"],
           beta: float = DEFAULTS["beta"], lam: float = DEFAULTS["lam"], ref: int = DEFAULTS["ref"],
           min_band: int = DEFAULTS["min_band"], band_budgets=None):
    """Kept packed indices (ascending int64) and per-subband statistics.

    band_budgets, when given, replaces the computed K_{j,o} (stage isolation: a caller can feed in
    another implementation's budgets)."""
    coeffs = np.asarray(coeffs, dtype=np.float32)
    v = joint_norm_f32(coeffs)
    bl = bands(G, J)
    E = energies(coeffs, G, J, ref)
    N = np.array([n for (_, _, _, n) in bl], dtype=np.int64)
    q = budget_quotients(E, N, K_tot, alpha, beta)
    Kb = np.maximum(min_band, np.floor(q)).astype(np.int64) if band_budgets is None else \
        np.asarray(band_budgets, dtype=np.int64)
    kept, stats = [], []
    for b, (j, o, off, n) in enumerate(bl):
        r = band_filter(v[off:off + n], Kb[b], lam)
        kept.append(off + np.nonzero(r.pop("keep"))[0])
        stats.append(dict(j=j, o=o, offset=off, N=n, E=E[b], quotient=q[b], K_band=int(Kb[b]),
                          kept=int(kept[-1].size), **r))
    return np.concatenate(kept).astype(np.int64), stats
