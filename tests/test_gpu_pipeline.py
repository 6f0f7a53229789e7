"""GPU parity of the upstream stages (TF + DWT, selection, construction), the loss, Adam, the DVR
supervision renderer, and of the step schedules (plain, batched, graph replay)."""
import dataclasses

import numpy as np
import pytest
import torch

import vbm_inputs as vi
from oracle import adam as oadam
from oracle import bank as obank
from oracle import construct as oconstruct
from oracle import dvr as odvr
from oracle import dwt as odwt
from oracle import loss as oloss
from oracle import select as oselect
from oracle import tf as otf
from tests.gpu_common import IMG_TOL, dev, say

pytestmark = pytest.mark.gpu


def _api():
    from paper_2601_09417_amd import api
    return api


def _dwt_case(G, J, wav, seed):
    vol = vi.blob_volume(G, 6, seed).astype(np.float32)
    vol = vi.minmax(vol).astype(np.float32)
    tf = vi.transfer_function(seed)
    return vol, tf


def _oracle_coeffs(vol, tf, J, wav):
    """float32 coefficients of the oracle's FP64 DWT of TF(F): the input both sides select from."""
    return odwt.dwt3d_rgba(otf.apply(vol, tf.xs, tf.rgba), J, wav).astype(np.float32)


@pytest.mark.parametrize("G,J,wav", [(32, 1, "haar"), (32, 3, "haar"), (32, 2, "bior4.4"), (48, 3, "bior4.4"),
                                     (16, 3, "bior4.4")])
def test_dwt_matches_oracle(G, J, wav):
    api = _api()
    say(f"dwt G={G} J={J} {wav}")
    vol, tf = _dwt_case(G, J, wav, G + J)
    coeffs = api.dwt3d(torch.from_numpy(vol).to(dev()), J, wav, (tf.xs, tf.rgba)).cpu().numpy()
    rgba = otf.apply(vol, tf.xs, tf.rgba)
    ref = odwt.dwt3d_rgba(rgba, J, wav)
    tol = 1e-6 if wav == "haar" else 1e-5
    for (j, o), (off, n) in odwt.block_offsets(G, J).items():
        blk = slice(off, off + n ** 3)
        scale = max(np.abs(ref[:, blk]).max(), 1e-6)
        err = np.abs(coeffs[:, blk] - ref[:, blk]).max() / scale
        assert err <= tol, ((j, o), err)


def test_dwt_rgba_input_path():
    api = _api()
    G, J = 16, 2
    rgba = np.random.default_rng(1).uniform(size=(4, G ** 3)).astype(np.float32)
    coeffs = api.dwt3d(torch.from_numpy(rgba).to(dev()), J, "bior4.4", None).cpu().numpy()
    ref = odwt.dwt3d_rgba(rgba.reshape(4, G, G, G), J, "bior4.4")
    assert np.abs(coeffs - ref).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("G,J,wav,K,s_mode", [(32, 1, "haar", 2048, "paper"), (32, 3, "bior4.4", 5000, "none"),
                                              (16, 2, "haar", 16 ** 3, "paper")])
def test_select_bit_exact_and_construction(G, J, wav, K, s_mode):
    api = _api()
    say(f"select/build G={G} J={J} {wav} K={K}")
    coeffs = _oracle_coeffs(*_dwt_case(G, J, wav, 7), J, wav)
    entries, packed = api.bank_build(wav, J)
    P, kept = api.build_gaussians(torch.from_numpy(coeffs).to(dev()), G, J, packed, K, s_mode=s_mode)
    ref_kept = oselect.topk(coeffs, K)
    assert np.array_equal(kept.cpu().numpy(), ref_kept)
    ob = obank.build_bank(wav, J)
    ref = oconstruct.construct(coeffs, ref_kept, G, J, ob, s_mode=s_mode)
    Pn = P.cpu().numpy()
    for name, rows in (("means", slice(0, 3)), ("scales", slice(3, 6)), ("quats", slice(6, 10)),
                       ("opacity", slice(10, 11)), ("rgb", slice(11, 14))):
        r = ref[name].reshape(rows.stop - rows.start, -1)
        err = np.abs(Pn[rows] - r).max() / max(np.abs(r).max(), 1e-6)
        assert err <= 1e-6, (name, err)


def test_select_ties_go_to_lower_index():
    api = _api()
    G, J = 16, 1
    c = np.zeros((4, G ** 3), np.float32)
    c[3, ::7] = 1.0          # many exact ties
    c[0, 5] = 2.0
    coeffs = torch.from_numpy(c).to(dev())
    _, packed = api.bank_build("haar", J)
    K = 100
    _, kept = api.build_gaussians(coeffs, G, J, packed, K)
    assert np.array_equal(kept.cpu().numpy(), oselect.topk(c, K))


@pytest.mark.parametrize("kind", ["l1", "l1_dssim"])
def test_loss_matches_oracle(kind):
    api = _api()
    rng = np.random.default_rng(4)
    # ragged and multi-tile for 32x32 loss tiles; runs of equal sizes share one launch per pass
    dims = [(37, 29), (64, 48), (64, 48), (101, 70), (37, 29), (37, 29)]
    imgs = [rng.uniform(size=(3, h, w)).astype(np.float32) for w, h in dims]
    tgts = [np.clip(i + 0.1 * rng.normal(size=i.shape), 0, 1).astype(np.float32) for i in imgs]
    x = torch.from_numpy(np.concatenate([i.reshape(-1) for i in imgs])).to(dev())
    y = torch.from_numpy(np.concatenate([t.reshape(-1) for t in tgts])).to(dev())
    lf = api.ImageLoss(dims, kind, 0.2)
    g = torch.empty_like(x)
    loss = float(lf(x, y, g).item())
    ref_loss, ref_g = oloss.loss_and_grad(imgs, tgts, kind)
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    rg = np.concatenate([a.reshape(-1) for a in ref_g])
    assert np.abs(g.cpu().numpy() - rg).max() <= 1e-4 * np.abs(rg).max()


def test_adam_matches_oracle():
    api = _api()
    rng = np.random.default_rng(9)
    N = 1000
    gs = vi.random_gaussians(N, 2)
    P = api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())
    ls, lo = oadam.raw_from_activated(gs.scales, gs.opacity)
    # the optimiser's initial state on the GPU (vbm_adam_init) against the oracle's activated -> raw
    # map, with opacities up to the construction's clamps and columns past n left untouched
    Pw = torch.full((14, N + 37), 7.0, dtype=torch.float32, device=dev())
    Pw[:, :N] = P
    Pw[10, :2] = torch.tensor([1e-3, 0.99], device=dev())
    raw_i, m_i, v_i = api.adam_init(Pw, n=N)
    raw_gpu = raw_i.cpu().numpy().astype(np.float64)
    op = Pw[10, :N].cpu().numpy().astype(np.float64)
    ls_w, lo_w = oadam.raw_from_activated(Pw[3:6, :N].cpu().numpy(), op)
    assert np.abs(raw_gpu[3:6, :N] - ls_w).max() <= 1e-6 * np.abs(ls_w).max()
    assert np.abs(raw_gpu[10, :N] - lo_w).max() <= 1e-6 * np.abs(lo_w).max()
    for rows in (slice(0, 3), slice(6, 10), slice(11, 14)):
        assert np.array_equal(raw_gpu[rows, :N], Pw[rows, :N].cpu().numpy().astype(np.float64))
    assert float(m_i[:, :N].abs().max()) == 0.0 and float(v_i[:, :N].abs().max()) == 0.0
    # both sides start from the oracle's raw values rounded to float32
    R = np.concatenate([gs.means, ls, gs.quats, lo[None], gs.rgb], 0).astype(np.float32).astype(np.float64)
    raw = torch.from_numpy(R.astype(np.float32)).to(dev())
    m = torch.zeros_like(raw)
    v = torch.zeros_like(raw)
    act = P.clone()
    oraw = dict(means=R[0:3], log_scales=R[3:6], quats=R[6:10], logit_opacity=R[10], rgb=R[11:14])
    om = {k: np.zeros_like(a) for k, a in oraw.items()}
    ov = {k: np.zeros_like(a) for k, a in oraw.items()}
    step_dev = torch.zeros(1, dtype=torch.int32, device=dev())
    for t in range(1, 4):
        G = rng.normal(size=(14, N)).astype(np.float32)
        grads = torch.from_numpy(G).to(dev())
        api.adam_step(raw, m, v, grads, act, step_dev=step_dev)
        act_g = dict(means=G[0:3], scales=G[3:6], quats=G[6:10], opacity=G[10], rgb=G[11:14])
        og = oadam.chain_grads(act_g, oraw)
        oraw, om, ov = oadam.step(oraw, og, om, ov, t)
    Rn = raw.cpu().numpy()
    for k, rows in (("means", slice(0, 3)), ("log_scales", slice(3, 6)), ("quats", slice(6, 10)),
                    ("logit_opacity", slice(10, 11)), ("rgb", slice(11, 14))):
        ref = np.asarray(oraw[k]).reshape(rows.stop - rows.start, -1)
        init = R[rows]
        # parity relative to the learning rate: 3 steps move each value by at most 3 lr
        lr = oadam.DEFAULT_LR[k]
        assert np.abs((Rn[rows] - init) - (ref - init)).max() <= 1e-3 * lr, k
    assert int(step_dev.item()) == 3
    A = act.cpu().numpy()
    assert np.allclose(A[3:6], np.exp(Rn[3:6]), rtol=1e-6)
    assert np.allclose(A[10], 1 / (1 + np.exp(-Rn[10])), rtol=1e-6)


def test_dvr_matches_oracle():
    api = _api()
    G = 32
    vol = vi.volume_for_config(0)
    tf = vi.transfer_function(0)
    # intrinsics rounded to float32, the values the library receives
    cams = [dataclasses.replace(c, fx=float(np.float32(c.fx)), fy=float(np.float32(c.fy)))
            for c in vi.orbit_cameras(2, 40, 30) + vi.orbit_cameras(1, 23, 41, distance=0.9)]
    say("dvr 32^3, views 40x30 x2 and 23x41 from inside the box")
    img = api.dvr_render(torch.from_numpy(vol).to(dev()), (tf.xs, tf.rgba), cams).cpu().numpy()
    off = 0
    for c in cams:
        ref, _, near = odvr.render(vol, tf.xs, tf.rgba, c, flag_rel=1e-6)
        got = img[off:off + 3 * c.width * c.height].reshape(3, c.height, c.width)
        off += 3 * c.width * c.height
        assert near.sum() <= 2
        err = np.abs(got - ref)[:, ~near].max() / max(np.abs(ref).max(), 1e-6)
        say(f"  {c.width}x{c.height}: {err:.2e}")
        assert err <= 1e-5


def _tuner_inputs(seed=3):
    gs = vi.random_gaussians(2000, seed, log_scale_mean=-3.2)
    cams = vi.orbit_cameras(3, 80, 64)
    tgt = torch.rand(sum(3 * c.width * c.height for c in cams), device=dev())
    return gs, cams, tgt


@pytest.mark.parametrize("loss", ["l1", "l1_dssim"])
def test_schedules_agree(loss):
    from paper_2601_09417_amd import trainer
    gs, cams, tgt = _tuner_inputs()
    api = _api()
    P = api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())
    say(f"schedules plain/batched/graph, loss={loss}")
    runs = {}
    for sched in ("plain", "batched", "graph"):
        ft = trainer.FineTuner(P, cams, tgt, loss=loss, schedule=sched)
        imgs = []
        for _ in range(3):
            ft.step()
            torch.cuda.synchronize()
            imgs.append(ft.image.clone())
            assert not ft.overflowed()
        runs[sched] = (imgs, ft.act.clone())
    # first iteration's forward is identical bit for bit (same parameters, same pair lists)
    assert torch.equal(runs["plain"][0][0], runs["batched"][0][0])
    assert torch.equal(runs["batched"][0][0], runs["graph"][0][0])
    # later iterations differ only through float atomics order in the backward
    for s in ("plain", "graph"):
        d = (runs[s][1] - runs["batched"][1]).abs().max().item()
        assert d <= 1e-4, (s, d)


def test_autotune_pick_matches_oracle_and_digit_widths_agree():
    """trainer.autotune on a small batch times every candidate; the schedule it picks renders the
    oracle's pair lists bit for bit; and every digit width of the tile sort (4 to 8 bits) gives the
    same pair values (lane-group marks included), ranges and first forward bit for bit, since the
    list order is fixed by its definition, not by the sort."""
    from oracle import binning
    from paper_2601_09417_amd import trainer
    from tests.gpu_common import ITEM_MASK
    gs, cams, tgt = _tuner_inputs(11)
    api = _api()
    P = api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())
    res = trainer.autotune(P, cams, tgt, steps=2, warmup=1)
    say(f"autotune: {res['table']} -> tile {res['tile']}, {res['sort_bits']}-bit digits")
    assert [(r["tile"], r["sort_bits"], r["lds_batch"], r["lds_batch_bwd"]) for r in res["table"]] == \
        list(trainer.TUNE_CANDIDATES)
    assert all(np.isfinite(r["ms"]) and r["ms"] > 0 for r in res["table"])
    fastest = min(r["ms"] for r in res["table"])
    first_close = next(r for r in res["table"] if r["ms"] <= fastest * (1 + trainer.TUNE_MARGIN))
    assert all(res[k] == first_close[k] for k in ("tile", "sort_bits", "lds_batch", "lds_batch_bwd", "ms"))

    def run(tile, bits, lds=0):
        rp = api.plan_batch(cams, [0, gs.n], tile=tile, sort_bits=bits, pair_capacity=1 << 20, lds_batch=lds,
                            lds_batch_bwd=lds)
        out = api.render_fwd(rp, P)
        torch.cuda.synchronize()
        assert int(out.status[0]) == 0
        n = int(out.status[1])
        return dict(tile=rp.region("pair_tile", torch.int32)[:n].cpu().numpy(),
                    item=rp.region("pair_item", torch.int32)[:n].cpu().numpy(),
                    ranges=rp.region("ranges", torch.int32).cpu().numpy(),
                    image=out.image.cpu().numpy(), final_T=out.final_T.cpu().numpy(),
                    n_contrib=out.n_contrib.cpu().numpy())

    pick = run(res["tile"], res["sort_bits"], res["lds_batch"])
    ref = binning.pair_lists(gs, cams, res["tile"])
    assert np.array_equal(pick["tile"], ref["tile"])
    assert np.array_equal(pick["item"] & ITEM_MASK, ref["item"])
    for tile in sorted({16, res["tile"]}):
        base = run(tile, 8)
        for bits in (4, 5, 6, 7):
            other = run(tile, bits)
            for k in base:
                assert np.array_equal(base[k], other[k]), (tile, bits, k)
        if tile <= 16:
            # the LDS-staged list walk composites in the same order: the same forward bit for bit
            for lds in (32, 64):
                other = run(tile, 8, lds)
                for k in ("tile", "item", "ranges", "image", "final_T", "n_contrib"):
                    assert np.array_equal(base[k], other[k]), (tile, lds, k)


def test_graph_replay_matches_eager_repeatedly():
    from paper_2601_09417_amd import trainer
    gs, cams, tgt = _tuner_inputs(5)
    api = _api()
    P = api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())
    eager = trainer.FineTuner(P, cams, tgt, schedule="batched")
    graph = trainer.FineTuner(P, cams, tgt, schedule="graph")
    for it in range(4):
        eager.step()
        graph.step()
        torch.cuda.synchronize()
        d = (eager.image - graph.image).abs().max().item()
        assert d <= 1e-4, (it, d)
        _ = eager.loss()   # host work between replays
    assert int(graph.step_dev.item()) == 4 and int(eager.step_dev.item()) == 4


@pytest.mark.parametrize("isotropic,unit_weight", [(True, False), (False, True), (True, True)])
def test_construction_ablation_variants(isotropic, unit_weight):
    """Without the bank's covariances (isotropic) and without the energy projection (w = 1),
    through the top-K build and through construction from an index list."""
    api = _api()
    G, J, wav, K = 32, 3, "bior4.4", 4000
    say(f"ablation isotropic={isotropic} unit_weight={unit_weight}")
    coeffs = _oracle_coeffs(*_dwt_case(G, J, wav, 11), J, wav)
    coeffs_d = torch.from_numpy(coeffs).to(dev())
    ref_kept = oselect.topk(coeffs, K)
    _, packed = api.bank_build(wav, J)
    P, kept = api.build_gaussians(coeffs_d, G, J, packed, K, s_mode="none", isotropic=isotropic,
                                  unit_weight=unit_weight)
    assert np.array_equal(kept.cpu().numpy(), ref_kept)
    P2 = api.construct_gaussians(coeffs_d, G, J, packed, torch.from_numpy(ref_kept).to(dev()), s_mode="none",
                                 isotropic=isotropic, unit_weight=unit_weight)
    ref = oconstruct.construct(coeffs, ref_kept, G, J, obank.build_bank(wav, J),
                               s_mode="none", isotropic=isotropic, unit_weight=unit_weight)
    for Pn in (P.cpu().numpy(), P2.cpu().numpy()):
        for name, rows in (("means", slice(0, 3)), ("scales", slice(3, 6)), ("quats", slice(6, 10)),
                           ("opacity", slice(10, 11)), ("rgb", slice(11, 14))):
            r = ref[name].reshape(rows.stop - rows.start, -1)
            err = np.abs(Pn[rows] - r).max() / max(np.abs(r).max(), 1e-6)
            assert err <= 1e-6, (name, err)
    if isotropic:
        S = P.cpu().numpy()[3:6]
        assert np.all(S == S[0, 0])


def test_trainer_replans_after_overflow():
    """A step whose pair lists outgrow the plan is flagged; check_capacity re-plans from exact counts
    (and captures the graph again), after which the step renders complete lists: its image equals
    that of a step runner planned with enough room from the start, given the same parameters."""
    from paper_2601_09417_amd import trainer
    gs, cams, tgt = _tuner_inputs(7)
    api = _api()
    P = api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())
    say("trainer re-plan after a pair overflow")
    ft = trainer.FineTuner(P, cams, tgt, schedule="graph", pair_capacity=64)
    ft.step()
    torch.cuda.synchronize()
    assert ft.check_capacity() and ft.overflows == 1
    assert not ft.check_capacity()          # flags were read and cleared
    act = ft.act.clone()
    ft.step()
    torch.cuda.synchronize()
    assert not ft.overflowed()
    ref = trainer.FineTuner(act, cams, tgt, schedule="batched")
    ref.step()
    torch.cuda.synchronize()
    assert torch.equal(ft.image, ref.image)


def test_size_class_schedules_match_the_single_schedule():
    """A batch of two scenes seen at two resolutions, rendered with one plan per size class and a
    different (tile, digit width) in each, gives the first forward of one plan over the whole batch
    bit for bit (a tiling changes a tile's list only by Gaussians that no pixel of it takes) and the
    same step up to float atomics order; the per-class autotuner returns a candidate per class."""
    from oracle import render
    from paper_2601_09417_amd import trainer
    from tests.gpu_common import IMG_TOL, image_error
    api = _api()
    s1 = vi.random_gaussians(900, 31, log_scale_mean=-3.2)
    s2 = vi.random_gaussians(1400, 32, log_scale_mean=-3.4)
    gs = vi.GaussianSet.concat([s1, s2])
    so = [0, s1.n, s1.n + s2.n]
    cams = vi.orbit_cameras(2, 96, 72) + vi.orbit_cameras(3, 61, 45, azimuth0=0.7)
    vs = [0, 1, 1, 0, 1]
    classes = trainer.size_classes(cams)
    assert classes == [(0, 2), (2, 5)]
    tgt = torch.rand(sum(3 * c.width * c.height for c in cams), device=dev())
    P = api.pack_params(gs.means, gs.scales, gs.quats, gs.opacity, gs.rgb, dev())
    say("size classes: 2 x 96x72 (tile 8, 8-bit) and 3 x 61x45 (tile 32, 4-bit) against one 16x16 plan")
    a = trainer.FineTuner(P, cams, tgt, so, vs, tile=16, sort_bits=8, schedule="batched")
    b = trainer.FineTuner(P, cams, tgt, so, vs, schedule="graph", classes=classes, class_schedules=[(8, 8), (32, 4)])
    a.step()
    b.step()
    torch.cuda.synchronize()
    assert not a.overflowed() and not b.overflowed()
    assert torch.equal(a.image, b.image)
    assert (a.act - b.act).abs().max().item() <= 1e-4
    ref = render.render_forward(render.Batch(gs, cams, 16, vs, so))
    for v, got in enumerate(api.split_views(b.image, cams)):
        assert image_error(got.cpu().numpy(), ref[v]["image"], ref[v]["flagged"]) <= IMG_TOL, v
    res = trainer.autotune_classes(P, cams, tgt, so, vs, steps=1, warmup=1)
    assert res["classes"] == classes and len(res["schedules"]) == 2
    assert all(tuple(s) in trainer.TUNE_CANDIDATES for s in res["schedules"])
    full = trainer.autotune_schedule(P, cams, tgt, so, vs, steps=1, warmup=1)
    assert full["per_class"]["schedules"] and np.isfinite(full["ms"])
