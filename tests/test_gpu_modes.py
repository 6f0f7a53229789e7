"""Visual modes (Sec. 4.4): one transfer function per value interval of the field, one Gaussian set
per mode, the sets stored side by side as the scenes of one batch, fine-tuned together and rendered
separately or concatenated.  Oracle inputs are made by the oracle (its FP64 DWT of TF_h(F), cast
to float32), and the same float32 values are uploaded for the HIP path."""
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
from tests.gpu_common import GRAD_TOL, IMG_TOL, ROWS, dev, flat, group_error, image_error, masked_dL, say

pytestmark = pytest.mark.gpu

G, J, WAV, K = 32, 2, "bior4.4", 300


def _api():
    from paper_2601_09417_amd import api
    return api


def _modes():
    vol = vi.volume_for_config(0)
    return vol, vi.mode_transfer_functions(vol, 0)


def _oracle_sets(vol, tfs):
    """Per mode: float32 coefficients of the oracle's DWT of TF_h(F), its top-K and construction."""
    ob = obank.build_bank(WAV, J)
    out = []
    for tf in tfs:
        c = odwt.dwt3d_rgba(otf.apply(vol, tf.xs, tf.rgba), J, WAV).astype(np.float32)
        kept = oselect.topk(c, K)
        out.append((c, kept, oconstruct.construct(c, kept, G, J, ob, s_mode="none")))
    return out


def _as_set(ref) -> vi.GaussianSet:
    f = np.float32
    return vi.GaussianSet(ref["means"].astype(f), ref["scales"].astype(f), ref["quats"].astype(f),
                          ref["opacity"].astype(f), ref["rgb"].astype(f))


def test_mode_sets_built_into_one_buffer():
    """Each mode's top-K and construction written into its own columns of one buffer; the columns
    of the other modes stay untouched."""
    api = _api()
    vol, tfs = _modes()
    sets = _oracle_sets(vol, tfs)
    say(f"mode sets: {len(tfs)} modes, G={G} J={J} {WAV} K={K} each")
    _, packed = api.bank_build(WAV, J)
    P = torch.full((14, K * len(tfs)), float("nan"), dtype=torch.float32, device=dev())
    for h, (c, kept, _) in enumerate(sets):
        _, kh = api.build_gaussians(torch.from_numpy(c).to(dev()), G, J, packed, K, s_mode="none", out=P,
                                    offset=h * K)
        assert np.array_equal(kh.cpu().numpy(), kept), h
    Pn = P.cpu().numpy()
    assert not np.isnan(Pn).any()
    for h, (_, _, ref) in enumerate(sets):
        cols = slice(h * K, (h + 1) * K)
        for name, rows in ROWS.items():
            r = ref[name].reshape(rows.stop - rows.start, -1)
            err = np.abs(Pn[rows, cols] - r).max() / max(np.abs(r).max(), 1e-6)
            assert err <= 1e-6, (h, name, err)
    with pytest.raises(ValueError):
        api.build_gaussians(torch.from_numpy(sets[0][0]).to(dev()), G, J, packed, K, out=P, offset=4 * K + 1)


def test_build_mode_sets_equals_per_mode_builds():
    api = _api()
    vol, tfs = _modes()
    vol_d = torch.from_numpy(vol).to(dev())
    pairs = [(t.xs, t.rgba) for t in tfs]
    Ks = [200, 300, 150, 400, 250]
    say("build_mode_sets vs one build per mode")
    P, offs, kept = api.build_mode_sets(vol_d, pairs, J, WAV, Ks, s_mode="none")
    assert list(offs) == list(np.concatenate([[0], np.cumsum(Ks)]))
    _, packed = api.bank_build(WAV, J)
    for h, tf in enumerate(pairs):
        Ph, kh = api.build_gaussians(api.dwt3d(vol_d, J, WAV, tf), G, J, packed, Ks[h], s_mode="none")
        assert torch.equal(P[:, offs[h]:offs[h + 1]], Ph), h
        assert torch.equal(kept[h], kh), h


def test_dwt_of_union_tf_is_sum_of_mode_dwts():
    api = _api()
    vol, tfs = _modes()
    vol_d = torch.from_numpy(vol).to(dev())
    u = vi.union_transfer_function(tfs)
    say("dwt of the union transfer function vs the sum over modes")
    total = sum(api.dwt3d(vol_d, J, WAV, (t.xs, t.rgba)) for t in tfs)
    whole = api.dwt3d(vol_d, J, WAV, (u.xs, u.rgba))
    assert (whole - total).abs().max().item() <= 1e-5 * whole.abs().max().item()


def test_mode_batch_render_parity_separate_and_concatenated():
    """The modes as scenes of one batch (each rendered separately from every camera) and all sets
    concatenated into one scene, forward and backward against the oracle."""
    from paper_2601_09417_amd import trainer
    api = _api()
    vol, tfs = _modes()
    sets = [_as_set(ref) for _, _, ref in _oracle_sets(vol, tfs)]
    gs = vi.GaussianSet.concat(sets)
    so = [h * K for h in range(len(tfs) + 1)]
    cams = vi.orbit_cameras(2, 56, 48, distance=3.0)
    cams_all, view_scene = api.mode_views(cams, len(tfs))
    assert view_scene == [h for h in range(len(tfs)) for _ in cams]
    P = api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())

    say(f"mode batch: {len(tfs)} scenes x {len(cams)} views 56x48, separate")
    rp = api.plan_batch(cams_all, so, view_scene, tile=16, pair_capacity=1 << 18)
    out = api.render_fwd(rp, P)
    torch.cuda.synchronize()
    assert int(out.status[0]) == 0
    batch = render.Batch(gs, cams_all, 16, view_scene, so)
    ref = render.render_forward(batch)
    imgs = api.split_views(out.image, cams_all)
    for v in range(len(cams_all)):
        assert image_error(imgs[v].cpu().numpy(), ref[v]["image"], ref[v]["flagged"]) <= IMG_TOL, v
    dL = masked_dL(cams_all, [r["flagged"] for r in ref], seed=9)
    grads = api.render_bwd(rp, P, flat(dL), out).cpu().numpy()
    g_ref, _ = render.render_backward(batch, dL)
    for name, rows in ROWS.items():
        assert group_error(grads[rows], g_ref[name].reshape(rows.stop - rows.start, -1)) <= GRAD_TOL, name

    say("mode sets concatenated into one scene")
    img = trainer.render_images(P, cams, tile=16)
    ref_c = render.render_forward(render.Batch(gs, cams, 16))
    for v, got in enumerate(api.split_views(img, cams)):
        assert image_error(got.cpu().numpy(), ref_c[v]["image"], ref_c[v]["flagged"]) <= IMG_TOL, v


@pytest.mark.parametrize("loss", ["l1", "l1_dssim"])
def test_mode_batch_step_matches_separate_steps(loss):
    """Modes share no Gaussians and no views, so one batched step over all modes renders every view
    as the separate per-mode steps do, and (the loss being the mean over the whole batch) its
    gradients are the per-mode gradients divided by the number of modes."""
    from paper_2601_09417_amd import trainer
    api = _api()
    vol, tfs = _modes()
    vol_d = torch.from_numpy(vol).to(dev())
    pairs = [(t.xs, t.rgba) for t in tfs]
    n = len(tfs)
    P, offs, _ = api.build_mode_sets(vol_d, pairs, J, WAV, K, s_mode="none")
    cams = vi.orbit_cameras(3, 64, 64, distance=3.0)
    cams_all, view_scene = api.mode_views(cams, n)
    targets = api.dvr_render_modes(vol_d, pairs, cams)
    per = targets.numel() // n
    say(f"mode batch step vs separate steps, loss={loss}")
    ft = trainer.FineTuner(P, cams_all, targets, offs, view_scene, loss=loss, schedule="batched")
    ft.step()
    torch.cuda.synchronize()
    assert not ft.overflowed()
    for h in range(n):
        a, b = int(offs[h]), int(offs[h + 1])
        fh = trainer.FineTuner(P[:, a:b].contiguous(), cams, targets[h * per:(h + 1) * per].clone(), loss=loss,
                               schedule="batched")
        fh.step()
        torch.cuda.synchronize()
        assert not fh.overflowed()
        assert torch.equal(ft.image[h * per:(h + 1) * per], fh.image), h
        g, gh = (n * ft.grads[:, a:b]).cpu().numpy(), fh.grads.cpu().numpy()
        for name, rows in ROWS.items():
            assert group_error(g[rows], gh[rows]) <= 1e-5, (h, name)
