"""Two-channel filter banks used by the oracle DWT (test infrastructure; see package docstring).

A filter is ``(taps, first)``: ``taps[i]`` is the coefficient at integer position ``first + i``.
Analysis (periodised, signal length N):
    a[k] = sum_m lo_a[m] x[(2k + m) mod N],      d[k] = sum_m hi_a[m] x[(2k + m) mod N]
Synthesis (the exact inverse):
    x[(2k + m) mod N] += a[k] lo_s[m] + d[k] hi_s[m]
High-pass filters follow from the low-pass pair by the alternating flip
    hi_a[n] = (-1)^n lo_s[1 - n],   hi_s[n] = (-1)^n lo_a[1 - n].

The paper uses the biorthogonal 4.4 wavelet (Sec. 4.2, Translation Consistency) and names Haar in
its ablation (Sec. 5.4).  bior4.4 is the CDF 9/7 pair; it is derived here from first principles
because no wavelet library is available: both low-pass filters carry the factor cos^4(w/2); their
remaining factors split the Bezout polynomial P(y) = 1 + 4y + 10y^2 + 20y^3, y = sin^2(w/2)
(Daubechies, Ten Lectures, Sec. 8.3): the real root goes to the 7-tap filter and the complex pair
to the 9-tap one; the 9-tap filter is the analysis low-pass.  Each low-pass sums to sqrt(2).
"""
from __future__ import annotations

import numpy as np

SQRT2 = np.sqrt(2.0)


def _conv(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.convolve(a, b)


def _laurent_one_minus_y_over(r: complex) -> np.ndarray:
    """Coefficients at z^-1, z^0, z^1 of 1 - y/r with y = (2 - z - 1/z)/4."""
    return np.array([1.0 / (4.0 * r), 1.0 - 1.0 / (2.0 * r), 1.0 / (4.0 * r)], dtype=complex)


def cdf97_lowpass_pair():
    """Returns (lo9, lo7): symmetric 9- and 7-tap low-pass filters centred at 0, each summing to sqrt(2)."""
    roots = np.roots([20.0, 10.0, 4.0, 1.0])               # 20y^3 + 10y^2 + 4y + 1
    real = [r for r in roots if abs(r.imag) < 1e-12]
    cplx = [r for r in roots if abs(r.imag) >= 1e-12]
    assert len(real) == 1 and len(cplx) == 2
    cos2 = np.array([0.25, 0.5, 0.25])                       # cos^2(w/2) = (2 + z + 1/z)/4
    base = _conv(cos2, cos2).astype(complex)                 # cos^4(w/2): 5 taps
    lo7 = _conv(base, _laurent_one_minus_y_over(real[0].real))
    lo9 = _conv(_conv(base, _laurent_one_minus_y_over(cplx[0])), _laurent_one_minus_y_over(cplx[1]))
    assert np.max(np.abs(lo7.imag)) < 1e-12 and np.max(np.abs(lo9.imag)) < 1e-12
    lo7 = lo7.real
    lo9 = lo9.real
    lo7 *= SQRT2 / lo7.sum()
    lo9 *= SQRT2 / lo9.sum()
    return lo9, lo7


class FilterBank:
    """Analysis/synthesis low- and high-pass filters with their integer start positions."""

    def __init__(self, name: str, lo_a, lo_a_first: int, lo_s, lo_s_first: int):
        self.name = name
        self.lo_a = (np.asarray(lo_a, dtype=np.float64), int(lo_a_first))
        self.lo_s = (np.asarray(lo_s, dtype=np.float64), int(lo_s_first))
        self.hi_a = self._flip(self.lo_s)
        self.hi_s = self._flip(self.lo_a)

    @staticmethod
    def _flip(f):
        """g[n] = (-1)^n f[1 - n]."""
        taps, first = f
        last = first + len(taps) - 1
        g_first = 1 - last
        g = np.empty(len(taps))
        for i in range(len(taps)):
            n = g_first + i
            g[i] = (-1.0) ** (n % 2) * taps[(1 - n) - first]
        return g, g_first


def haar() -> FilterBank:
    h = np.array([1.0, 1.0]) / SQRT2
    return FilterBank("haar", h, 0, h, 0)


def bior44() -> FilterBank:
    lo9, lo7 = cdf97_lowpass_pair()
    return FilterBank("bior4.4", lo9, -4, lo7, -3)


def get(name: str) -> FilterBank:
    if name == "haar":
        return haar()
    if name in ("bior4.4", "bior44", "cdf97"):
        return bior44()
    raise ValueError(name)
