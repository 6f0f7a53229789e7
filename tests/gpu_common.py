"""Shared helpers of the GPU parity tests (comparison protocol and scene builders)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import vbm_inputs as vi

IMG_TOL = 1e-5      # images: max |gpu - oracle| / max |oracle| over unflagged pixels
GRAD_TOL = 1e-4     # gradients: per parameter group, max |gpu - oracle| / max |oracle|
ITEM_MASK = (1 << 27) - 1   # pair values: item id below bit 27, forward lane-group marks above
ROWS = dict(means=slice(0, 3), scales=slice(3, 6), quats=slice(6, 10), opacity=slice(10, 11), rgb=slice(11, 14))


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def dev():
    return torch.device("cuda:0")


def to_dev(gs: vi.GaussianSet):
    from paper_2601_09417_amd import api
    return api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())


def image_error(gpu: np.ndarray, ref: np.ndarray, flagged: np.ndarray) -> float:
    ok = ~flagged
    if not ok.any():
        return 0.0
    return float(np.abs(gpu - ref)[:, ok].max() / max(np.abs(ref).max(), 1e-6))


def group_error(gpu: np.ndarray, ref: np.ndarray) -> float:
    scale = max(float(np.abs(ref).max()), 1e-12)
    return float(np.abs(gpu - ref).max() / scale)


def masked_dL(cams, flagged_list, seed=0):
    """Random image gradients, zero at pixels where float32 and float64 may branch apart."""
    rng = np.random.default_rng(seed)
    out = []
    for c, fl in zip(cams, flagged_list):
        d = rng.normal(size=(3, c.height, c.width)).astype(np.float32)
        d[:, fl] = 0.0
        out.append(d)
    return out


def flat(arrs) -> torch.Tensor:
    return torch.from_numpy(np.concatenate([np.asarray(a, np.float32).reshape(-1) for a in arrs])).to(dev())


def adaptive_check(coeffs_np, G, J, kept_gpu, stats_gpu, K_tot, **kw):
    """Parity of one vbm_adaptive_select result with the oracle run on the same float32 coefficients
    (made by the oracle or by the seeded generators, never by the HIP path).  Budgets are float64
    quotients floored to integers, summed in different orders on the two sides; the fixtures keep
    every quotient at least 1e-3 away from an integer unless it is one exactly (with alpha = 0 and
    power-of-two band sizes every operation is exact), so the budgets are unique and compared exactly.
    Everything after the budgets is float32 decided in the same order on both sides and must match
    bit for bit."""
    from oracle import adaptive as A
    from paper_2601_09417_amd import _lib as L
    S = {name: stats_gpu[:, i] for i, name in enumerate(L.ADAPTIVE_STATS)}
    kept_o, so = A.select(coeffs_np, G, J, K_tot, **kw)
    E = np.array([s["E"] for s in so])
    N = np.array([s["N"] for s in so])
    q = np.array([s["quotient"] for s in so])
    assert np.allclose(S["E"], E, rtol=1e-12, atol=0.0)
    assert np.array_equal(S["N"].astype(np.int64), N)
    assert np.allclose(S["quotient"], q, rtol=1e-11, atol=1e-300)
    assert np.array_equal(S["K_band"].astype(np.int64), np.array([s["K_band"] for s in so]))
    for b, s in enumerate(so):
        for name in ("median", "mad", "sigma", "T", "vK"):
            assert np.float32(S[name][b]) == s[name], (b, name, S[name][b], s[name])
        assert int(S["C"][b]) == s["C"] and int(S["K"][b]) == s["K"] and int(S["kept"][b]) == s["kept"], b
    assert np.array_equal(kept_gpu, kept_o)
    return kept_o, so
