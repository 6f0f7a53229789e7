"""Pins of the oracle transition bank (Sec. 4.2) and Gaussian construction (Sec. 4.3)."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import bank, construct, dwt, select


def _haar_closed_form(j, lam=1e-8):
    """Haar: |psi| = 2^{-3j/2} on a 2^j cube, so u = (2^j-1)/2, Sigma = (4^j-1)/12 I, and the ridge weight
    w = y0 sum G / (sum G^2 + lam) with G separable on the cube."""
    n = 1 << j
    u = (n - 1) / 2.0
    var = (4.0 ** j - 1) / 12.0
    i = np.arange(n)
    g1 = np.exp(-0.5 * (i - u) ** 2 / var)
    sG = g1.sum() ** 3
    sG2 = (g1 ** 2).sum() ** 3
    y0 = 2.0 ** (-1.5 * j)
    return u, var, y0 * sG / (sG2 + lam)


def test_haar_bank_closed_form():
    J = 4
    for e in bank.build_bank("haar", J):
        u, var, w = _haar_closed_form(e.j)
        assert np.allclose(e.u, u, atol=1e-12)
        assert np.allclose(e.sigma, var * np.eye(3), atol=1e-10)
        assert abs(e.w - w) <= 1e-12 * w
        assert e.roi_size == (1 << e.j) ** 3
        assert np.array_equal(e.quat, [1.0, 0.0, 0.0, 0.0])


def test_bank_entry_count_and_order():
    b = bank.build_bank("haar", 3)
    assert len(b) == 7 * 3 + 1
    assert [(e.j, e.o) for e in b] == dwt.block_order(3)


@pytest.mark.parametrize("wav", ["haar", "bior4.4"])
def test_outer_product_equals_full_3d_idwt(wav):
    G, J = 64, 2
    offs = dwt.block_offsets(G, J)
    for (j, o) in [(1, 1), (1, 6), (2, 0), (2, 7)]:
        off, n = offs[(j, o)]
        k = n // 2
        flat = np.zeros(G ** 3)
        flat[off + (k * n + k) * n + k] = 1.0
        full = dwt.idwt3d(dwt.unpack(flat, G, J), J, wav)
        psi, (cx, cy, cz) = bank.canonical_wavelet(wav, j, o)
        origin = (1 << j) * k
        sub = full[np.ix_(origin + cz, origin + cy, origin + cx)]
        assert np.abs(sub - psi).max() <= 1e-14
        assert abs(np.abs(full).sum() - np.abs(psi).sum()) <= 1e-12


def test_bior_bank_symmetric_diagonal():
    for e in bank.build_bank("bior4.4", 3):
        off = np.abs(e.sigma - np.diag(np.diag(e.sigma))).max()
        assert off <= 1e-12 * np.abs(e.sigma).max()
        assert np.all(np.diag(e.sigma) > 0) and e.w > 0


def test_separability_with_zero_threshold():
    """tau = 0 keeps every non-zero sample, so Sigma is the diagonal of the 1D |r| variances."""
    for wav in ("haar", "bior4.4"):
        fb = __import__("oracle.wavelets", fromlist=["get"]).get(wav)
        j, o = 2, 5
        psi, coords = bank.canonical_wavelet(wav, j, o)
        u, S, w, nroi = bank.fit_entry(psi, coords, 0.0, 1e-8)
        for d in range(3):
            r, rel = bank.response_1d(fb, j, "H" if (o >> d) & 1 else "L")
            p = np.abs(r) / np.abs(r).sum()
            mu = (p * rel).sum()
            assert abs(u[d] - mu) <= 1e-12
            assert abs(S[d, d] - (p * (rel - mu) ** 2).sum()) <= 1e-10
        assert np.abs(S - np.diag(np.diag(S))).max() <= 1e-12


def test_quaternion_factorisation_general_case():
    rng = np.random.default_rng(3)
    for _ in range(20):
        R = Rotation.random(random_state=rng).as_matrix()
        s = rng.uniform(0.5, 3.0, size=3)
        S = R @ np.diag(s ** 2) @ R.T
        sc, q = bank.factor_covariance(S)
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        assert q[0] >= 0
        assert np.allclose(Rq @ np.diag(sc ** 2) @ Rq.T, S, atol=1e-12)


def test_select_topk_bruteforce_with_ties():
    rng = np.random.default_rng(7)
    c = rng.normal(size=(4, 500)).astype(np.float32)
    c[:, 100] = c[:, 7]
    c[:, 300] = c[:, 7]
    v = select.joint_norm_f32(c)
    K = 60
    kept = select.topk(c, K)
    ranked = sorted(range(500), key=lambda i: (-float(v[i]), i))
    assert list(kept) == sorted(ranked[:K])
    # ties at the threshold go to the lower index
    thr = float(v[ranked[K - 1]])
    tied = [i for i in range(500) if float(v[i]) == thr]
    assert all((i in kept) == (i in ranked[:K]) for i in tied)
    assert np.array_equal(kept, select.topk_bruteforce(c, K))
    for K2 in (1, 99, 100, 101, 499, 500):
        assert np.array_equal(select.topk(c, K2), select.topk_bruteforce(c, K2))


def test_joint_norm_is_float32_fixed_order():
    c = np.array([[3.0], [4.0], [12.0], [84.0]], dtype=np.float32)
    assert select.joint_norm_f32(c)[0] == np.float32(85.0)


def test_haar_construction_centres_at_cube_centres():
    G, J = 16, 2
    rng = np.random.default_rng(2)
    coeffs = rng.normal(size=(4, G ** 3))
    kept = np.sort(rng.choice(G ** 3, size=200, replace=False))
    b = bank.build_bank("haar", J)
    out = construct.construct(coeffs, kept, G, J, b, s_mode="paper")
    h = 2.0 / G
    for n, idx in enumerate(kept):
        j, o, k = dwt.decode_index(int(idx), G, J)
        centre = (1 << j) * np.array(k) + (1 << (j - 1))
        assert np.allclose(out["means"][:, n], -1 + h * centre, atol=1e-12)
        e = b[dwt.block_order(J).index((j, o))]
        amp = 2.0 ** (-1.5 * j) * np.abs(coeffs[:, idx]) * e.w
        assert abs(out["opacity"][n] - np.clip(amp[3], 1e-3, 0.99)) <= 1e-15
        assert np.allclose(out["rgb"][:, n], np.clip(amp[:3], 0, 1), atol=1e-15)
        assert np.allclose(out["scales"][:, n], h * np.sqrt((4.0 ** j - 1) / 12.0), atol=1e-12)
