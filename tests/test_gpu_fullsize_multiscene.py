"""GPU parity of the uneven multi-scene batch at full size, on sampled tiles.

Workload: four independent volumes (64^3, 128^3, 256^3 and 384^3 blobs + k^-2 noise) with one
transfer function, bior4.4 with J = 3, 3, 4, 5, the top 50k, 200k, 800k and 1.5M Gaussians; scene i
is seen by 4 orbit views at resolution i (512x512, 800x800, 1280x720, 1920x1080), all 16 views in
one batched launch with per-scene Gaussian ranges, 16x16 tiles.  Each scene's Gaussian set is the
oracle's (its FP64 DWT rounded to float32, its top-K and construction); one sampled view per scene
has its sampled tiles' pair lists compared bit for bit, their images, and every Gaussian's gradient
with dL/dI nonzero only on those tiles.
"""
import numpy as np
import pytest
import torch

import vbm_inputs as vi
from tests.gpu_common import dev, oracle_gaussians, sampled_tile_parity, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

SCENES = [dict(G=64, J=3, K=50_000, res=(512, 512)), dict(G=128, J=3, K=200_000, res=(800, 800)),
          dict(G=256, J=4, K=800_000, res=(1280, 720)), dict(G=384, J=5, K=1_500_000, res=(1920, 1080))]
VIEWS_PER_SCENE, TILE, WAV = 4, 16, "bior4.4"


def test_multiscene_fullsize_sampled_tiles():
    from paper_2601_09417_amd import api
    tfn = vi.transfer_function(4)
    sets = []
    for s, sc in enumerate(SCENES):
        vol = vi.scene_volume(4, s, sc["G"])
        _, ((_, _, gs),) = oracle_gaussians(vol, tfn, sc["J"], WAV, sc["K"])
        sets.append(gs)
        say(f"scene {s}: {sc['G']}^3 J={sc['J']}, oracle set of {gs.n} Gaussians")
    gs = vi.GaussianSet.concat(sets)
    so = np.concatenate([[0], np.cumsum([g.n for g in sets])]).astype(np.int64)
    cams, view_scene = [], []
    for s, sc in enumerate(SCENES):
        cams += vi.orbit_cameras(VIEWS_PER_SCENE, sc["res"][0], sc["res"][1], azimuth0=0.4 * s)
        view_scene += [s] * VIEWS_PER_SCENE
    P = api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())
    rp = api.plan_batch(cams, so, view_scene, tile=TILE, sort_bits=8, pair_capacity=64_000_000, mode="batched")
    say(f"batch: {len(cams)} views over {len(SCENES)} scenes, {gs.n} Gaussians, {int(rp.plan.n_tiles)} tiles")
    sample = [s * VIEWS_PER_SCENE + 1 for s in range(len(SCENES))]
    sampled_tile_parity(rp, P, gs, cams, view_scene, so, TILE, sample, 6, 44)
    torch.cuda.synchronize()
