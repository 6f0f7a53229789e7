"""GPU edge cases at the limits the boundary accepts, and degenerate inputs of the method.

* the largest view a plan accepts (16384 x 16384, a million 16x16 tiles): sampled tiles' pair lists,
  images and gradients against the oracle;
* the largest grid the DWT accepts (1024^3), one Haar level: every coefficient of sampled 2x2x2
  blocks against the oracle's transform of that block (a Haar level-1 coefficient depends on its
  own block only);
* one-pixel and one-row views next to a regular one in one batch;
* a transfer function that is zero everywhere (all coefficients zero, every key tied) and K = 1.
"""
import numpy as np
import pytest
import torch

import vbm_inputs as vi
from oracle import bank as obank
from oracle import construct as oconstruct
from oracle import dwt as odwt
from oracle import render
from oracle import select as oselect
from oracle import tf as otf
from tests.gpu_common import (GRAD_TOL, IMG_TOL, ROWS, dev, flat, group_error, image_error, masked_dL,
                              sampled_tile_parity, say, to_dev)

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


def _api():
    from paper_2601_09417_amd import api
    return api


def test_largest_view():
    api = _api()
    W = H = 16384
    gs = vi.random_gaussians(20_000, 61, extent=0.9, log_scale_mean=-5.0, log_scale_std=0.4)
    cams = vi.orbit_cameras(1, W, H, distance=3.0)
    say(f"one {W}x{H} view, {gs.n} Gaussians")
    P = to_dev(gs)
    rp = api.plan_batch(cams, [0, gs.n], tile=16, pair_capacity=12_000_000)
    assert int(rp.plan.n_tiles) == (W // 16) * (H // 16)
    sampled_tile_parity(rp, P, gs, cams, [0], [0, gs.n], 16, (0,), 12, 62)
    torch.cuda.synchronize()


def test_largest_dwt_grid_haar():
    api = _api()
    G, J = 1024, 1
    rng = vi.rng(71, vi.STREAM_VOLUME)
    vol = rng.random((G, G, G), dtype=np.float32)
    tf = vi.transfer_function(71)
    say(f"DWT of a {G}^3 volume, Haar J={J}")
    coeffs = api.dwt3d(torch.from_numpy(vol).to(dev()), J, "haar", (tf.xs, tf.rgba))
    offs = odwt.block_offsets(G, J)
    n = G // 2
    picks = np.random.default_rng(72).integers(0, n, size=(48, 3))
    picks = np.concatenate([picks, [[0, 0, 0], [n - 1, n - 1, n - 1], [n - 1, 0, 5]]])
    idx = {b: [] for b in offs}
    for kx, ky, kz in picks:
        for b, (off, nb) in offs.items():
            idx[b].append(off + (kz * nb + ky) * nb + kx)
    got = {b: coeffs[:, torch.as_tensor(v, device=dev())].cpu().numpy() for b, v in idx.items()}
    del coeffs
    for s, (kx, ky, kz) in enumerate(picks):
        block = vol[2 * kz:2 * kz + 2, 2 * ky:2 * ky + 2, 2 * kx:2 * kx + 2]
        ref = odwt.dwt3d_rgba(otf.apply(block, tf.xs, tf.rgba), J, "haar")     # [4][8] for the 2^3 block
        small = odwt.block_offsets(2, J)
        for b in offs:
            r = ref[:, small[b][0]]
            assert np.abs(got[b][:, s] - r).max() <= 1e-6 * max(np.abs(r).max(), 1.0), (b, s)
    say(f"  {len(picks)} blocks x 8 subbands x 4 channels match")


def test_one_pixel_and_one_row_views():
    api = _api()
    gs = vi.random_gaussians(3000, 63, log_scale_mean=-3.0)
    cams = [vi.orbit_cameras(1, 1, 1, distance=3.0)[0], vi.orbit_cameras(1, 97, 1, azimuth0=0.7)[0],
            vi.orbit_cameras(1, 1, 53, azimuth0=1.4)[0], vi.orbit_cameras(1, 40, 29, azimuth0=2.1)[0]]
    say("views 1x1, 97x1, 1x53 and 40x29 in one batch")
    P = to_dev(gs)
    rp = api.plan_batch(cams, [0, gs.n], tile=16, pair_capacity=1 << 18)
    out = api.render_fwd(rp, P)
    torch.cuda.synchronize()
    assert int(out.status[0]) == 0
    batch = render.Batch(gs, cams, 16)
    ref = render.render_forward(batch)
    imgs = api.split_views(out.image, cams)
    for v in range(len(cams)):
        assert image_error(imgs[v].cpu().numpy(), ref[v]["image"], ref[v]["flagged"]) <= IMG_TOL, v
    dL = masked_dL(cams, [r["flagged"] for r in ref], seed=64)
    g = api.render_bwd(rp, P, flat(dL), out).cpu().numpy()
    g_ref, _ = render.render_backward(batch, dL)
    for name, rows in ROWS.items():
        assert group_error(g[rows], g_ref[name].reshape(rows.stop - rows.start, -1)) <= GRAD_TOL, name


@pytest.mark.parametrize("K", [1, 200])
def test_zero_transfer_function_and_single_gaussian(K):
    """All coefficients zero: every key ties, so the top-K is the K lowest packed indices, and every
    Gaussian takes the lower opacity clamp and black colour; K = 1 keeps one Gaussian."""
    api = _api()
    G, J, wav = 16, 2, "bior4.4"
    vol = vi.minmax(vi.blob_volume(G, 4, 81)).astype(np.float32)
    xs = np.array([0.0, 1.0], np.float32)
    rgba = np.zeros((2, 4), np.float32)
    c = odwt.dwt3d_rgba(otf.apply(vol, xs, rgba), J, wav).astype(np.float32)
    assert not c.any()
    say(f"zero transfer function, K={K}")
    coeffs = api.dwt3d(torch.from_numpy(vol).to(dev()), J, wav, (xs, rgba))
    assert not coeffs.any()
    _, packed = api.bank_build(wav, J)
    P, kept = api.build_gaussians(torch.from_numpy(c).to(dev()), G, J, packed, K)
    ref_kept = oselect.topk(c, K)
    assert np.array_equal(ref_kept, np.arange(K)) and np.array_equal(kept.cpu().numpy(), ref_kept)
    ref = oconstruct.construct(c, ref_kept, G, J, obank.build_bank(wav, J))
    Pn = P.cpu().numpy()
    for name, rows in ROWS.items():
        r = ref[name].reshape(rows.stop - rows.start, -1)
        assert np.abs(Pn[rows] - r).max() <= 1e-6 * max(np.abs(r).max(), 1e-6), name
    assert np.all(Pn[10] == np.float32(1e-3)) and not Pn[11:14].any()
