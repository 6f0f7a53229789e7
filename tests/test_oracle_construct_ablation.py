"""Pins of the construction ablation variants (Sec. 5): without the bank's covariances every
Gaussian shares sigma_iso^2 I at the full model's mean extent; without the energy projection
w = 1.  Checked against the full construction and the bank itself."""
import numpy as np

from oracle import bank as obank
from oracle import construct as C
from oracle import select as S


def _case(G=16, J=2, wav="bior4.4", K=300, seed=1):
    rng = np.random.default_rng(seed)
    c = rng.normal(size=(4, G ** 3)).astype(np.float32)
    return c, S.topk(c, K), obank.build_bank(wav, J)


def test_isotropic_variant_shares_the_mean_extent():
    c, kept, bank = _case()
    full = C.construct(c, kept, 16, 2, bank)
    iso = C.construct(c, kept, 16, 2, bank, isotropic=True)
    sigma = np.mean([np.mean(full["scales"][:, i]) for i in range(kept.size)])   # per-Gaussian loop
    assert np.allclose(iso["scales"], sigma, rtol=1e-14, atol=0)
    assert np.array_equal(iso["quats"], np.tile([[1.0], [0.0], [0.0], [0.0]], (1, kept.size)))
    for k in ("means", "opacity", "rgb"):                       # centres and appearance unchanged
        assert np.array_equal(iso[k], full[k])
    # the covariance is isotropic: R diag(s^2) R^T = sigma^2 I
    assert np.all(iso["scales"][0] == iso["scales"][1]) and np.all(iso["scales"][1] == iso["scales"][2])


def test_unit_weight_variant_drops_the_energy_projection():
    c, kept, bank = _case(J=1, wav="haar", K=200, seed=2)
    full = C.construct(c, kept, 16, 1, bank, s_mode="none")
    unit = C.construct(c, kept, 16, 1, bank, s_mode="none", unit_weight=True)
    # Haar: every subband's weight is the same closed-form w, so unit weight scales amplitudes by 1/w
    # before clamping; compare unclamped entries
    w = bank[0].w
    assert all(np.isclose(e.w, w, rtol=1e-12) for e in bank)
    A = np.abs(c[:, kept].astype(np.float64))
    ok = (A[:3] < 1.0) & (A[:3] * w < 1.0)
    assert np.allclose(unit["rgb"][ok], A[:3][ok], rtol=1e-14)
    assert np.allclose(full["rgb"][ok], (A[:3] * w)[ok], rtol=1e-14)
    for k in ("means", "scales", "quats"):
        assert np.array_equal(unit[k], full[k])
