"""GPU gradients at the differentiated-batch size against FP64 central finite differences.

Workload: the 256^3 blobs + noise volume and its transfer function, bior4.4 J=4, the oracle's top
500,000 Gaussians, 8 orbit views at 1024x1024 in one batched launch, 16x16 tiles.  The sampled-tile
parity (pair lists bit-exact, images, every Gaussian's gradient against the oracle's autodiff) runs
first; then for 64 seeded Gaussians of the sampled tiles every one of their 14 parameters is moved
by +-h and +-h/2 and the FP64 functional sum(dL/dI * I) over the sampled tiles (the oracle's
compositing of the same lists) is differenced.  Where the two step sizes disagree the step crossed a
decision of the compositing (an alpha threshold, the 0.99 clamp, the transmittance stop) and the
scalar is not compared; everywhere else the GPU gradient must match the (Richardson-extrapolated)
difference.
"""
import numpy as np
import pytest
import torch

import vbm_inputs as vi
from oracle import render
from tests.gpu_common import GRAD_TOL, ROWS, dev, oracle_gaussians, sampled_tile_parity, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

G, J, WAV, K = 256, 4, "bior4.4", 500_000
VIEWS, W, H, TILE = 8, 1024, 1024, 16
N_FD, STEP = 64, 1e-5


def _phi(tile, gs64, gi, name, row, delta, cams):
    """FP64 sum(dL/dI * I) over one sampled tile with parameter (name, row) of Gaussian gi moved by delta."""
    v, glob, xs, ys, d = tile
    p = {k: gs64[k][..., glob].copy() for k in gs64}
    col = int(np.nonzero(glob == gi)[0][0])
    if name == "opacity":
        p[name][col] += delta
    else:
        p[name][row, col] += delta
    t = render._t
    m2d, con, _ = render.project_fp64(t(p["means"]), t(p["scales"]), t(p["quats"]), cams[v])
    pix = torch.stack([t(xs + 0.5), t(ys + 0.5)], 1)
    c, _, _, _, _ = render.composite_tile(pix, m2d, con, t(p["opacity"]), t(p["rgb"]).T, t(cams[v].bg))
    return float((c * t(d.T.astype(np.float64))).sum())


def test_fullsize_gradient_central_differences():
    from paper_2601_09417_amd import api
    say("256^3 volume, oracle set of 500k Gaussians, 8 views 1024x1024")
    _, ((_, _, gs),) = oracle_gaussians(vi.volume_for_config(2), vi.transfer_function(2), J, WAV, K)
    cams = vi.orbit_cameras(VIEWS, W, H)
    P = api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())
    N = P.shape[1]
    rp = api.plan_batch(cams, [0, N], tile=TILE, sort_bits=8, pair_capacity=40_000_000, mode="batched")
    tiles, g, involved, _ = sampled_tile_parity(rp, P, gs, cams, [0] * VIEWS, [0, N], TILE, (2, 5), 8, 55)

    gs64 = {k: np.asarray(getattr(gs, k), np.float64) for k in ("means", "scales", "quats", "opacity", "rgb")}
    # half of the Gaussians at random, half among the anisotropic ones (an isotropic Gaussian's
    # rotation gradient is exactly zero)
    rng = np.random.default_rng(56)
    sc = gs64["scales"][:, involved]
    aniso = involved[sc.max(0) > 1.2 * sc.min(0)]
    half = min(N_FD // 2, aniso.size)
    pick = rng.choice(aniso, half, replace=False)
    rest = np.setdiff1d(involved, pick)
    pick = np.concatenate([pick, rng.choice(rest, min(N_FD - half, rest.size), replace=False)])
    checked, skipped = 0, 0
    res = {}
    for name, rows in ROWS.items():
        gpu, fd = [], []
        for gi in pick:
            mine = [t for t in tiles if gi in t[1]]
            for r in range(rows.stop - rows.start):
                base = abs(gs64[name][r, gi]) if name != "opacity" else abs(gs64[name][gi])
                h = STEP * max(base, 1e-2) if name in ("scales", "opacity") else STEP
                f = lambda dl: sum(_phi(t, gs64, gi, name, r, dl, cams) for t in mine)  # noqa: E731
                d1 = (f(h) - f(-h)) / (2 * h)
                d2 = (f(h / 2) - f(-h / 2)) / h
                if abs(d1 - d2) > 1e-4 * max(abs(d1), abs(d2)) + 1e-9:
                    skipped += 1          # the step crossed a compositing decision
                    continue
                gpu.append(g[rows.start + r, gi])
                fd.append((4.0 * d2 - d1) / 3.0)      # Richardson: error O(h^4)
                checked += 1
        res[name] = (np.array(gpu), np.array(fd))
    top = max(float(np.abs(fd).max(initial=0.0)) for _, fd in res.values())
    for name, (gpu, fd) in res.items():
        # relative to the group's largest difference quotient, floored at 1e-3 of the largest of all
        # groups so that a group of near-zero derivatives is not measured against its own noise
        scale = max(float(np.abs(fd).max(initial=0.0)), 1e-3 * top)
        err = float(np.abs(gpu - fd).max(initial=0.0)) / scale
        say(f"  {name}: {gpu.size} scalars, max |gpu - fd| / scale = {err:.2e}")
        assert err <= 2 * GRAD_TOL, name
    say(f"  checked {checked} scalars of {pick.size} Gaussians ({half} anisotropic), {skipped} skipped at "
        f"decisions")
    assert checked >= 0.9 * (checked + skipped)
