"""GPU parity of the adaptive per-subband selection (Supp. A) and of construction from an index
list, against the oracle on the same float32 coefficients: the oracle's FP64 DWT of TF(F) cast
to float32 (or seeded synthetic values), uploaded for the HIP path.

Budgets are float64 quotients floored to integers and must match exactly (the fixtures have no
quotient within 1e-9 of an integer).  Everything after the budgets is float32 decided in the same
order on both sides and must match bit for bit: medians, MAD, sigma, T, #(v >= T), K, v_(K) and
the kept index list."""
import numpy as np
import pytest
import torch

import vbm_inputs as vi
from oracle import adaptive as oadaptive
from oracle import bank as obank
from oracle import construct as oconstruct
from oracle import dwt as odwt
from oracle import tf as otf
from paper_2601_09417_amd import _lib as L
from tests.gpu_common import ROWS, adaptive_check, dev, say

pytestmark = pytest.mark.gpu


def _api():
    from paper_2601_09417_amd import api
    return api


def _coeffs(G, J, wav, seed):
    """float32 coefficients of the oracle's DWT of TF(F) for a seeded blob volume."""
    vol = vi.minmax(vi.blob_volume(G, 6, seed)).astype(np.float32)
    tf = vi.transfer_function(seed)
    return odwt.dwt3d_rgba(otf.apply(vol, tf.xs, tf.rgba), J, wav).astype(np.float32)


@pytest.mark.parametrize("G,J,wav,K_tot,params", [
    (32, 3, "bior4.4", 4000, dict()),
    (32, 3, "bior4.4", 4000, dict(alpha=1.0, beta=0.0)),
    (32, 2, "haar", 2000, dict(alpha=0.5, beta=0.5, lam=1.5)),
    (48, 3, "bior4.4", 30000, dict(alpha=0.0, beta=1.0, lam=0.0)),
    (32, 3, "haar", 50, dict(lam=2.0)),            # the per-band minimum fires: total above K_tot
    (16, 1, "bior4.4", 16 ** 3, dict(ref=0, min_band=0)),
    (40, 3, "bior4.4", 3000, dict()),              # odd coarsest side: subbands of 125 locations
])
def test_adaptive_select_matches_oracle(G, J, wav, K_tot, params):
    api = _api()
    say(f"adaptive G={G} J={J} {wav} K_tot={K_tot} {params}")
    c = _coeffs(G, J, wav, G + J)
    kept, stats = api.adaptive_select(torch.from_numpy(c).to(dev()), G, J, K_tot, **params)
    kept_o, so = adaptive_check(c, G, J, kept.cpu().numpy(), stats.cpu().numpy(), K_tot, **params)
    say(f"  kept {kept_o.size} over {len(so)} subbands")


def test_adaptive_ties_and_capacity():
    api = _api()
    G, J = 16, 2
    rng = np.random.default_rng(5)
    c = (rng.integers(0, 4, size=(4, G ** 3)) * 0.25).astype(np.float32)   # many exact ties
    coeffs = torch.from_numpy(c).to(dev())
    kept, stats = api.adaptive_select(coeffs, G, J, 300, lam=0.5)
    S = stats.cpu().numpy()
    adaptive_check(c, G, J, kept.cpu().numpy(), S, 300, lam=0.5)
    assert np.any(S[:, 11] > S[:, 9])                       # some subband keeps ties beyond K
    with pytest.raises(L.VBMError):
        api.adaptive_select(coeffs, G, J, 300, lam=0.5, capacity=5)


def test_adaptive_rejects_bad_arguments():
    api = _api()
    coeffs = torch.zeros(4, 16 ** 3, device=dev())
    for kw in (dict(K_tot=0), dict(K_tot=100, lam=-1.0), dict(K_tot=100, ref=4), dict(K_tot=100, alpha=-1.0)):
        with pytest.raises(L.VBMError):
            api.adaptive_select(coeffs, 16, 2, **kw)


def test_construct_from_adaptive_indices():
    api = _api()
    G, J, wav = 32, 3, "bior4.4"
    c = _coeffs(G, J, wav, 9)
    coeffs = torch.from_numpy(c).to(dev())
    kept_o, _ = oadaptive.select(c, G, J, 3000)
    kept, _ = api.adaptive_select(coeffs, G, J, 3000)
    assert np.array_equal(kept.cpu().numpy(), kept_o)
    _, packed = api.bank_build(wav, J)
    for s_mode in ("paper", "none"):
        P = api.construct_gaussians(coeffs, G, J, packed, torch.from_numpy(kept_o).to(dev()), s_mode=s_mode)
        ref = oconstruct.construct(c, kept_o, G, J, obank.build_bank(wav, J), s_mode=s_mode)
        Pn = P.cpu().numpy()
        for name, rows in ROWS.items():
            r = ref[name].reshape(rows.stop - rows.start, -1)
            assert np.abs(Pn[rows] - r).max() <= 1e-6 * max(np.abs(r).max(), 1e-6), (s_mode, name)
