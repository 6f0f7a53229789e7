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
