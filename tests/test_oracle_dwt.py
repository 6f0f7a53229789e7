"""Pins of the oracle DWT and filter banks against mathematics that does not depend on the oracle."""
import numpy as np
import pytest

from oracle import dwt, wavelets


@pytest.mark.parametrize("wav", ["haar", "bior4.4"])
@pytest.mark.parametrize("J", [1, 2, 3])
def test_perfect_reconstruction(wav, J):
    x = np.random.default_rng(J).normal(size=(16, 16, 16))
    c = dwt.dwt3d(x, J, wav)
    assert np.abs(dwt.idwt3d(c, J, wav) - x).max() <= 1e-12


@pytest.mark.parametrize("wav", ["haar", "bior4.4"])
def test_constant_input_only_lll(wav):
    J, c0 = 3, 0.37
    c = dwt.dwt3d(np.full((16, 16, 16), c0), J, wav)
    assert np.allclose(c[(J, 0)], c0 * 2 ** (1.5 * J), rtol=0, atol=1e-12)
    for key, blk in c.items():
        if key != (J, 0):
            assert np.abs(blk).max() <= 1e-12


def test_haar_2x2x2_by_hand():
    x = np.arange(8, dtype=np.float64).reshape(2, 2, 2) ** 1.5 + 1.0   # [z][y][x]
    c = dwt.dwt3d(x, 1, "haar")
    for o in range(8):
        s = 0.0
        for z in range(2):
            for y in range(2):
                for xx in range(2):
                    sign = 1.0
                    for d, idx in enumerate((xx, y, z)):
                        if (o >> d) & 1 and idx == 1:
                            sign = -sign
                    s += sign * x[z, y, xx]
        expect = s / 2 ** 1.5
        got = c[(1, 0)] if o == 0 else c[(1, o)]
        assert abs(got.item() - expect) <= 1e-14


def test_haar_parseval():
    x = np.random.default_rng(5).normal(size=(32, 32, 32))
    c = dwt.dwt3d(x, 3, "haar")
    assert abs(sum((b ** 2).sum() for b in c.values()) - (x ** 2).sum()) <= 1e-9 * (x ** 2).sum()


def test_cdf97_biorthogonal_and_vanishing_moments():
    b = wavelets.bior44()
    lo_a, fa = b.lo_a
    lo_s, fs = b.lo_s
    assert len(lo_a) == 9 and len(lo_s) == 7
    assert np.allclose(lo_a, lo_a[::-1], atol=1e-15) and np.allclose(lo_s, lo_s[::-1], atol=1e-15)
    assert abs(lo_a.sum() - np.sqrt(2)) < 1e-14 and abs(lo_s.sum() - np.sqrt(2)) < 1e-14
    # sum_n lo_a[n] lo_s[n + 2k] = delta_k
    for k in range(-4, 5):
        s = 0.0
        for i, c in enumerate(lo_a):
            n = fa + i
            m = n + 2 * k - fs
            if 0 <= m < len(lo_s):
                s += c * lo_s[m]
        assert abs(s - (1.0 if k == 0 else 0.0)) < 1e-14
    # four vanishing moments on both high-pass filters
    for taps, first in (b.hi_a, b.hi_s):
        n = first + np.arange(len(taps))
        for p in range(4):
            assert abs((taps * n.astype(float) ** p).sum()) < 1e-11 * max(1.0, np.abs(n).max() ** p)


@pytest.mark.parametrize("wav", ["haar", "bior4.4"])
def test_translation_theorem_exact_on_periodic_grid(wav):
    """W^-1[e_{j,o,k}] = roll(W^-1[e_{j,o,0}], 2^j k) exactly (Supp. B, Theorem)."""
    G, J = 32, 3
    rng = np.random.default_rng(11)
    offs = dwt.block_offsets(G, J)
    for (j, o) in [(1, 5), (2, 3), (3, 0), (3, 7)]:
        off, n = offs[(j, o)]
        k = tuple(int(v) for v in rng.integers(0, n, size=3))
        flat0 = np.zeros(G ** 3)
        flat0[off] = 1.0
        flatk = np.zeros(G ** 3)
        flatk[off + (k[2] * n + k[1]) * n + k[0]] = 1.0
        r0 = dwt.idwt3d(dwt.unpack(flat0, G, J), J, wav)
        rk = dwt.idwt3d(dwt.unpack(flatk, G, J), J, wav)
        s = 1 << j
        shifted = np.roll(r0, (s * k[2], s * k[1], s * k[0]), axis=(0, 1, 2))
        assert np.abs(rk - shifted).max() <= 1e-14


def test_packing_roundtrip_and_decode():
    G, J = 16, 2
    flat = np.arange(G ** 3, dtype=np.float64)
    assert np.array_equal(dwt.pack(dwt.unpack(flat, G, J), G, J), flat)
    j, o, k = dwt.decode_index(0, G, J)
    assert (j, o, k) == (2, 0, (0, 0, 0))
    j, o, k = dwt.decode_index(G ** 3 - 1, G, J)
    assert (j, o, k) == (1, 7, (7, 7, 7))
