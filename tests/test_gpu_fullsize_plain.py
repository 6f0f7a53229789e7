"""GPU parity of the plain one-view-per-launch schedule at the medium workload's full size.

Workload: the 128^3 volume (64 blobs + k^-2 noise) with its transfer function, Haar J=3, the top
100,000 Gaussians, 16 orbit views at 800x800; every view planned and rendered on its own in the
exact mode (one host sync sizes its sort), 16x16 tiles with 8-bit and 4-bit tile-sort digits.  The
Gaussian set is the oracle's (its FP64 DWT rounded to float32, its top-K and construction).  Sampled
views have their whole pair lists, counts and ranges compared bit for bit, sampled tiles' images
compared with the oracle's compositing, and every Gaussian's gradient with dL/dI nonzero only on
those tiles.
"""
import numpy as np
import pytest
import torch

import vbm_inputs as vi
from tests.gpu_common import dev, oracle_gaussians, sampled_tile_parity, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

WL = vi.WORKLOADS["c1"]


@pytest.fixture(scope="module")
def c1_set():
    vol = vi.volume_for_config(1)
    tfn = vi.transfer_function(1)
    _, ((_, _, gs),) = oracle_gaussians(vol, tfn, WL.J, WL.wavelet, WL.K)
    say(f"c1: {WL.G}^3 Haar J={WL.J}, oracle set of {gs.n} Gaussians")
    return gs


@pytest.mark.parametrize("bits", [8, 4])
def test_plain_schedule_fullsize_sampled_tiles(c1_set, bits):
    from paper_2601_09417_amd import api
    gs = c1_set
    cams = vi.orbit_cameras(WL.n_views, WL.width, WL.height)
    P = api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())
    N = P.shape[1]
    for v in (0, 5, 11):
        say(f"  view {v} of {WL.n_views}, {WL.width}x{WL.height}, exact mode, {bits}-bit digits")
        rp = api.plan_batch([cams[v]], [0, N], tile=WL.tile, sort_bits=bits, pair_capacity=4_000_000, mode="exact")
        sampled_tile_parity(rp, P, gs, [cams[v]], [0], [0, N], WL.tile, [0], 8, 60 + v)
    torch.cuda.synchronize()
