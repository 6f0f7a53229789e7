"""Periodised separable J-level 3D DWT, its inverse, and the packed coefficient layout.

Test infrastructure (see package docstring).  Follows Sec. 3 (3D Wavelet Transform) and
Sec. 4.3 (Multichannel Wavelet Transform, eq. mul_wavelet_coff): each level filters the current
approximation along x, then y, then z; the next level acts on the LLL octant only.  Boundary
handling is periodisation (the paper allows symmetric or periodic extension; periodic keeps every
subband at exactly G/2^j per axis and makes the translation theorem of Supp. B exact).

Arrays are indexed [z][y][x] (x fastest in memory).  Orientation code ``o`` has bit d set when the
high-pass was taken along axis d (bit 0 = x, bit 1 = y, bit 2 = z); o = 0 is LLL.

Packed layout (per channel, G^3 values): [LLL_J] then for j = J, J-1, ..., 1 the seven blocks
o = 1..7 of level j; each block is [n_j^3] in [z][y][x] order with n_j = G / 2^j.
"""
from __future__ import annotations

import numpy as np
import torch

from . import wavelets


def analysis_1d(x, bank: wavelets.FilterBank, axis: int):
    """One periodised analysis step along ``axis``: returns (low, high), each half as long.

    The signal is extended periodically by the filter reach on both sides so that every tap
    x[(2k + m) mod N] is a plain strided slice of the extended array.  Accepts a numpy array or a
    float64 CPU torch tensor (the multi-level transform keeps torch tensors between levels so that
    the elementwise sums run multi-threaded) and returns the same kind.
    """
    is_np = isinstance(x, np.ndarray)
    xt = torch.from_numpy(np.asarray(x, dtype=np.float64)) if is_np else x
    N = xt.shape[axis]
    assert N % 2 == 0
    xm = xt.movedim(axis, 0)
    firsts = [bank.lo_a[1], bank.hi_a[1]]
    lasts = [bank.lo_a[1] + len(bank.lo_a[0]) - 1, bank.hi_a[1] + len(bank.hi_a[0]) - 1]
    lo_pad, hi_pad = max(0, -min(firsts)), max(0, max(lasts) - 1) + 1
    if lo_pad <= N and hi_pad <= N:
        ext = torch.cat([xm[N - lo_pad:], xm, xm[:hi_pad]], 0)
        base = lo_pad
    else:                                                       # filter longer than the signal
        reps = -(-max(lo_pad, hi_pad) // N) + 1
        ext = torch.cat([xm] * (2 * reps + 1), 0)
        base = reps * N
    out = []
    for taps, first in (bank.lo_a, bank.hi_a):
        acc = None
        for i, c in enumerate(taps):
            m = first + i
            term = float(c) * ext[base + m: base + m + N: 2]
            acc = term if acc is None else acc.add_(term)
        acc = acc.movedim(0, axis).contiguous()
        out.append(acc.numpy() if is_np else acc)
    return out[0], out[1]


def synthesis_1d(lo: np.ndarray, hi: np.ndarray, bank: wavelets.FilterBank, axis: int) -> np.ndarray:
    """Exact inverse of :func:`analysis_1d`."""
    n = lo.shape[axis]
    N = 2 * n
    shape = list(lo.shape)
    shape[axis] = N
    x = np.zeros(shape, dtype=np.result_type(lo, hi, np.float64))
    k = np.arange(n)
    xm = np.moveaxis(x, axis, 0)
    lom = np.moveaxis(lo, axis, 0)
    him = np.moveaxis(hi, axis, 0)
    for (taps, first), src in ((bank.lo_s, lom), (bank.hi_s, him)):
        for i, c in enumerate(taps):
            m = first + i
            np.add.at(xm, (2 * k + m) % N, c * src)
    return x


def analysis_level(x: np.ndarray, bank) -> dict:
    """One 3D level: returns {o: octant} for o = 0..7 (o = 0 is LLL)."""
    cur = {0: x}
    for d, axis in enumerate((2, 1, 0)):          # x, y, z
        nxt = {}
        for o, arr in cur.items():
            lo, hi = analysis_1d(arr, bank, axis)
            nxt[o] = lo
            nxt[o | (1 << d)] = hi
        cur = nxt
    return cur


def synthesis_level(octants: dict, bank) -> np.ndarray:
    cur = dict(octants)
    for d, axis in reversed(list(enumerate((2, 1, 0)))):
        nxt = {}
        for o in list(cur.keys()):
            if o & (1 << d):
                continue
            nxt[o] = synthesis_1d(cur[o], cur[o | (1 << d)], bank, axis)
        cur = nxt
    return cur[0]


def dwt3d(x: np.ndarray, J: int, wavelet: str) -> dict:
    """J-level 3D DWT of one channel.  Returns {(j, o): block}; LLL is stored as (J, 0)."""
    bank = wavelets.get(wavelet)
    G = x.shape[0]
    assert x.shape == (G, G, G) and G % (1 << J) == 0
    out = {}
    cur = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
    for j in range(1, J + 1):
        oct_ = analysis_level(cur, bank)
        for o in range(1, 8):
            out[(j, o)] = oct_[o].numpy()
        cur = oct_[0]
    out[(J, 0)] = cur.numpy()
    return out


def idwt3d(coeffs: dict, J: int, wavelet: str) -> np.ndarray:
    bank = wavelets.get(wavelet)
    cur = coeffs[(J, 0)]
    for j in range(J, 0, -1):
        octs = {0: cur}
        for o in range(1, 8):
            octs[o] = coeffs[(j, o)]
        cur = synthesis_level(octs, bank)
    return cur


def block_order(J: int):
    """The (j, o) blocks in packed order."""
    order = [(J, 0)]
    for j in range(J, 0, -1):
        for o in range(1, 8):
            order.append((j, o))
    return order


def block_offsets(G: int, J: int) -> dict:
    """{(j, o): (offset, n_j)} into the packed per-channel array of G^3 values."""
    off = 0
    res = {}
    for (j, o) in block_order(J):
        n = G >> j
        res[(j, o)] = (off, n)
        off += n ** 3
    assert off == G ** 3
    return res


def pack(coeffs: dict, G: int, J: int) -> np.ndarray:
    offs = block_offsets(G, J)
    flat = np.empty(G ** 3, dtype=np.float64)
    for key, (off, n) in offs.items():
        flat[off:off + n ** 3] = coeffs[key].reshape(-1)
    return flat


def unpack(flat: np.ndarray, G: int, J: int) -> dict:
    offs = block_offsets(G, J)
    return {key: flat[off:off + n ** 3].reshape(n, n, n) for key, (off, n) in offs.items()}


def decode_index(idx: int, G: int, J: int):
    """Packed linear index -> (j, o, (kx, ky, kz))."""
    for (j, o), (off, n) in block_offsets(G, J).items():
        if off <= idx < off + n ** 3:
            r = idx - off
            return j, o, (r % n, (r // n) % n, r // (n * n))
    raise IndexError(idx)


def dwt3d_rgba(rgba: np.ndarray, J: int, wavelet: str) -> np.ndarray:
    """rgba [4][G][G][G] -> packed coefficients [4][G^3] (FP64)."""
    G = rgba.shape[1]
    return np.stack([pack(dwt3d(rgba[c], J, wavelet), G, J) for c in range(rgba.shape[0])])
