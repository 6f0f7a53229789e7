"""GPU parity at the benchmark's full size and at the large-batch size.

Workloads: the 512^3 turbulence volume and its transfer function, bior4.4 J=5; the benchmark's top
1,000,000 Gaussians with 8 orbit views at 1920x1080, and the large batch's top 2,000,000 with 16
views at 1920x1080; 16x16 tiles, one batched launch over all views (the launch configuration
bench.py times).  The oracle computes the whole FP64 DWT of TF(F) once (about a minute on the
host); its float32 rounding is the input both sides select from, and the oracle's own top-K and
construction give the Gaussian sets both sides render.  Checked against the oracle:

* DWT: every coefficient of the GPU's transform of the same volume (per subband, relative to the
  subband maximum);
* selection: the complete top-K sets (bit-exact) and every constructed Gaussian, and the adaptive
  per-subband selection with all its statistics;
* rendering: sampled views' pair lists of sampled tiles (bit-exact) and their images; for the
  backward, dL/dI is nonzero only on those tiles, so the oracle's autodiff over the same tiles gives
  every Gaussian's exact gradient.
"""
import dataclasses

import numpy as np
import pytest
import torch

import vbm_inputs as vi
from oracle import dvr as odvr
from oracle import dwt as odwt
from tests.gpu_common import ROWS, adaptive_check, dev, oracle_gaussians, sampled_tile_parity, say

# the module fixture runs the oracle's full-size DWT once: allow for it in the first test's limit
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

G, J, WAV = 512, 5, "bior4.4"
W, H = 1920, 1080
CASES = {"1M-8views": dict(K=1_000_000, views=8, sample=(1, 6)),
         "2M-16views": dict(K=2_000_000, views=16, sample=(3, 12))}


@pytest.fixture(scope="module")
def h_case():
    from paper_2601_09417_amd import api
    say("full size: the 512^3 volume, the oracle's FP64 DWT of TF(F), its top-1M and top-2M sets")
    vol = vi.volume_for_config(3)
    tfn = vi.transfer_function(3)
    coeffs, sets = oracle_gaussians(vol, tfn, J, WAV, [c["K"] for c in CASES.values()])
    say("  oracle DWT, top-K and construction done")
    gpu_coeffs = api.dwt3d(torch.from_numpy(vol).to(dev()), J, WAV, (tfn.xs, tfn.rgba))
    torch.cuda.synchronize()
    return dict(api=api, coeffs=coeffs, coeffs_d=torch.from_numpy(coeffs).to(dev()), gpu_coeffs=gpu_coeffs,
                sets=dict(zip(CASES, sets)), vol=vol, tf=tfn)


def test_fullsize_dwt_every_coefficient(h_case):
    got = h_case["gpu_coeffs"]
    ref = h_case["coeffs_d"]
    worst = 0.0
    for (j, o), (off, n) in odwt.block_offsets(G, J).items():
        blk = slice(off, off + n ** 3)
        scale = max(float(ref[:, blk].abs().max()), 1e-6)
        err = float((got[:, blk] - ref[:, blk]).abs().max()) / scale
        worst = max(worst, err)
        assert err <= 1e-5, ((j, o), err)
    say(f"  {G ** 3} coefficients x 4 channels within {worst:.1e} of their subband maximum")


@pytest.mark.parametrize("case", list(CASES))
def test_fullsize_selection_and_construction(h_case, case):
    api = h_case["api"]
    kept_o, ref, _ = h_case["sets"][case]
    _, packed = api.bank_build(WAV, J)
    P, kept = api.build_gaussians(h_case["coeffs_d"], G, J, packed, CASES[case]["K"], s_mode="none")
    assert np.array_equal(kept.cpu().numpy(), kept_o)
    Pn = P.cpu().numpy()
    for name, rows in ROWS.items():
        r = ref[name].reshape(rows.stop - rows.start, -1)
        err = np.abs(Pn[rows] - r).max() / max(np.abs(r).max(), 1e-6)
        assert err <= 1e-6, (name, err)


def test_fullsize_adaptive_selection(h_case):
    """The adaptive per-subband selection on the full coefficient set (36 subbands, 134M locations)
    against the oracle on the same float32 coefficients, budget 1M."""
    api = h_case["api"]
    K = CASES["1M-8views"]["K"]
    kept, stats = api.adaptive_select(h_case["coeffs_d"], G, J, K)
    kept_o, so = adaptive_check(h_case["coeffs"], G, J, kept.cpu().numpy(), stats.cpu().numpy(), K)
    say(f"  adaptive: kept {kept_o.size} (budget {K}), T of the finest subbands "
        f"{[round(float(s['T']), 5) for s in so[-7:]]}")


# every schedule the autotuner chooses from (tile edge, tile-sort digit width) at the benchmark's
# size, and the autotuner's usual pick at the large batch
SCHEDULES = [("1M-8views", 16, 8, 0, 0), ("1M-8views", 16, 4, 0, 0), ("1M-8views", 8, 8, 0, 0),
             ("1M-8views", 32, 8, 0, 0), ("1M-8views", 16, 8, 32, 0), ("1M-8views", 16, 8, 64, 0),
             ("1M-8views", 16, 8, 32, 32), ("2M-16views", 16, 8, 0, 0)]


@pytest.mark.parametrize("case,tile,bits,lds,lds_bwd", SCHEDULES)
def test_fullsize_render_sampled_tiles(h_case, case, tile, bits, lds, lds_bwd):
    api = h_case["api"]
    _, _, gs = h_case["sets"][case]
    cfg = CASES[case]
    cams = vi.orbit_cameras(cfg["views"], W, H)
    P = api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())
    N = P.shape[1]
    say(f"  {case}: {N} Gaussians, {cfg['views']} views {W}x{H}, tile {tile}, {bits}-bit digits, LDS batch {lds}/{lds_bwd}")
    rp = api.plan_batch(cams, [0, N], tile=tile, sort_bits=bits, pair_capacity=8_000_000 * cfg["views"],
                        mode="batched", lds_batch=lds, lds_batch_bwd=lds_bwd)
    sampled_tile_parity(rp, P, gs, cams, [0] * len(cams), [0, N], tile, cfg["sample"], 10, 33)


def test_fullsize_schedules_list_the_tuner_candidates():
    from paper_2601_09417_amd import trainer
    assert {(t, b, k, kb) for c, t, b, k, kb in SCHEDULES if c == "1M-8views"} == set(trainer.TUNE_CANDIDATES)


def test_fullsize_dvr_sampled_pixels(h_case):
    """The supervision renderer at the size whose images the benchmark fits: the 512^3 volume from the
    8 orbit views at 1920x1080, 400 random pixels per view plus the corners and the centre, against
    the oracle's ray-marcher on the same rays, within 1e-5 of the sampled image maximum."""
    api = h_case["api"]
    vol, tfn = h_case["vol"], h_case["tf"]
    cams = [dataclasses.replace(c, fx=float(np.float32(c.fx)), fy=float(np.float32(c.fy)))
            for c in vi.orbit_cameras(8, W, H)]
    img = api.dvr_render(torch.from_numpy(vol).to(dev()), (tfn.xs, tfn.rgba), cams)
    views = api.split_views(img, cams)
    rng = np.random.default_rng(8)
    worst, n_near, n_pix = 0.0, 0, 0
    for v, c in enumerate(cams):
        px = np.concatenate([rng.integers(0, W, 400), [0, W - 1, 0, W - 1, W // 2]])
        py = np.concatenate([rng.integers(0, H, 400), [0, 0, H - 1, H - 1, H // 2]])
        ref, _, near = odvr.render(vol, tfn.xs, tfn.rgba, c, pixels=(px, py), flag_rel=1e-6)
        got = views[v][:, torch.as_tensor(py), torch.as_tensor(px)].cpu().numpy()
        n_near += int(near.sum())
        n_pix += px.size
        err = float(np.abs(got - ref)[:, ~near].max() / max(np.abs(ref).max(), 1e-6))
        worst = max(worst, err)
        assert err <= 1e-5, (v, err)
    say(f"  dvr 512^3 at {W}x{H}: {n_pix} rays, error {worst:.2e} of the image maximum, {n_near} near the stop")
    assert n_near <= 2
