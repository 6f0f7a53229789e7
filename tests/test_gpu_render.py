"""GPU parity of the renderer against the oracle: float32 binning decisions and pair lists bit-exact,
images within 1e-5 and gradients within 1e-4 (relative to the group maximum)."""
import numpy as np
import pytest
import torch

import vbm_inputs as vi
from oracle import binning, render
from tests.gpu_common import (GRAD_TOL, IMG_TOL, ITEM_MASK, ROWS, dev, flat, group_error, image_error, masked_dL, say,
                              to_dev)

pytestmark = pytest.mark.gpu


def _api():
    from paper_2601_09417_amd import api
    return api


def _scene(n, seed, views, W, H, log_scale=-3.0, opacity=(0.05, 0.95)):
    gs = vi.random_gaussians(n, seed, log_scale_mean=log_scale, opacity_range=opacity)
    cams = vi.orbit_cameras(views, W, H, azimuth0=0.3 * seed)
    return gs, cams


# Opacities of (0.001, 0.007): about half of the Gaussians are below 1/255 and reach no pixel (the
# projection marks them invisible).
LOW_OPACITY = (0.001, 0.007)


# every (tile, digit width) schedule the autotuner tries, and digit widths between
@pytest.mark.parametrize("tile,bits,opacity", [(8, 8, (0.05, 0.95)), (16, 8, (0.05, 0.95)), (32, 8, (0.05, 0.95)),
                                               (16, 4, (0.05, 0.95)), (16, 8, LOW_OPACITY), (16, 4, LOW_OPACITY),
                                               (8, 5, (0.05, 0.95)), (32, 6, (0.05, 0.95))])
def test_projection_and_pair_lists_bit_exact(tile, bits, opacity):
    api = _api()
    gs, cams = _scene(3000, 11, 3, 131, 77, opacity=opacity)
    say(f"pair lists tile={tile} digits={bits} n={gs.n} views=3 131x77 opacity {opacity}")
    P = to_dev(gs)
    rp = api.plan_batch(cams, [0, gs.n], tile=tile, sort_bits=bits, pair_capacity=1 << 20)
    out = api.render_fwd(rp, P)
    torch.cuda.synchronize()
    ref = binning.pair_lists(gs, cams, tile)
    assert int(out.status[0]) == 0
    P_ref = ref["tile"].size
    assert int(out.status[1]) == P_ref
    depth = rp.region("item_depth", torch.float32).cpu().numpy()
    bins = rp.region("item_rect", torch.int32).cpu().numpy().view(np.uint32).reshape(-1, 4)
    ntl = rp.region("item_ntiles", torch.int32).cpu().numpy()
    rec = rp.region("item_rec", torch.float32).cpu().numpy().reshape(-1, 4)
    coef = rp.region("item_coef", torch.float32).cpu().numpy().reshape(-1, 8)
    I = int(rp.plan.n_items)
    rx, ry = bins[:I, 0], bins[:I, 1] & 0x0FFF0FFF      # (the row-band bits sit above bit 11 of each half)
    assert np.array_equal(bins[:I, 3], ntl[:I])
    for v in range(3):
        pr = ref["proj"][v]
        sl = slice(v * gs.n, (v + 1) * gs.n)
        vis = pr["n_tiles"] > 0
        assert np.array_equal(ntl[sl], pr["n_tiles"])
        # the float32 spec values themselves (quaternion norm, divisions, square roots in one order)
        for arr, col, val in ((coef, 0, pr["px"]), (coef, 1, pr["py"]), (rec, 0, pr["conic"][0]),
                              (rec, 1, pr["conic"][1]), (rec, 2, pr["conic"][2])):
            assert np.array_equal(arr[sl][vis, col].view(np.uint32), np.asarray(val, np.float32)[vis].view(np.uint32))
        assert np.array_equal(depth[sl][vis].view(np.uint32), pr["depth"][vis].view(np.uint32))
        assert np.array_equal(rx[sl][vis] & 0xFFFF, pr["x0"][vis])
        assert np.array_equal(rx[sl][vis] >> 16, pr["x1"][vis])
        assert np.array_equal(ry[sl][vis] & 0xFFFF, pr["y0"][vis])
        assert np.array_equal(ry[sl][vis] >> 16, pr["y1"][vis])
    ptile = rp.region("pair_tile", torch.int32).cpu().numpy()[:P_ref]
    pitem = rp.region("pair_item", torch.int32).cpu().numpy()[:P_ref] & ITEM_MASK   # marks above bit 26
    assert np.array_equal(ptile, ref["tile"])
    assert np.array_equal(pitem, ref["item"])
    ranges = rp.region("ranges", torch.int32).cpu().numpy().reshape(-1, 2)
    ref_r = ref["ranges"]
    nonempty = ref_r[:, 1] > ref_r[:, 0]
    assert np.array_equal(ranges[nonempty], ref_r[nonempty])
    assert np.all(ranges[~nonempty, 0] == ranges[~nonempty, 1])      # empty tiles hold an empty range


def _band_scene(kind):
    if kind == "small":
        return _scene(3000, 21, 3, 131, 77, log_scale=-3.3)
    if kind == "needles":
        # one axis stretched 30x and another shrunk 5x: thin ellipses at every orientation, the case
        # where the footprint's row extent depends most on the conic's cross term
        gs, cams = _scene(2500, 22, 3, 160, 112, log_scale=-3.4)
        gs.scales[0] *= np.float32(30.0)
        gs.scales[1] *= np.float32(0.2)
        return gs, cams
    # large footprints that overflow the ballot-word buffer, so that the emission re-tests them
    gs = vi.random_gaussians(1200, 23, log_scale_mean=-1.5, log_scale_std=0.3)
    return gs, vi.orbit_cameras(1, 256, 192, azimuth0=0.4)


@pytest.mark.parametrize("kind", ["small", "needles", "overflow"])
def test_row_bands_cover_every_contributing_pixel(kind):
    """With 16x16 tiles each pair value carries, in bits 27..30, the 4-row bands of its tile that the
    footprint can reach, and the forward evaluates only those.  Every pixel of the tile where the
    Gaussian reaches alpha >= 1/255 (float64, from the oracle's float32 projection) must lie in a set
    band; the bands must also skip something, or the test would pass on an all-ones mask."""
    api = _api()
    gs, cams = _band_scene(kind)
    P = to_dev(gs)
    rp = api.plan_batch(cams, [0, gs.n], tile=16, pair_capacity=1 << 21)
    out = api.render_fwd(rp, P)
    torch.cuda.synchronize()
    ref = binning.pair_lists(gs, cams, 16)
    n = ref["tile"].size
    assert int(out.status[0]) == 0 and int(out.status[1]) == n
    if kind == "overflow":
        taken = int(rp.region("counters", torch.int32).cpu().numpy().view(np.uint64)[2])
        assert taken > int(rp.plan.region_bytes[22]) // 8
    pv = rp.region("pair_item", torch.int32).cpu().numpy()[:n].view(np.uint32)
    assert np.array_equal(pv & ITEM_MASK, ref["item"])
    bands = (pv >> 27) & 0xF
    W, H = cams[0].width, cams[0].height
    tx_n, ty_n = -(-W // 16), -(-H // 16)
    tile = ref["tile"].astype(np.int64)
    view, local = tile // (tx_n * ty_n), tile % (tx_n * ty_n)
    tx, ty = local % tx_n, local // tx_n
    gi = ref["item"].astype(np.int64) - view * gs.n
    px = np.empty(n); py = np.empty(n); A = np.empty(n); B = np.empty(n); C = np.empty(n)
    for v in range(len(cams)):
        sel = view == v
        pr = ref["proj"][v]
        px[sel], py[sel] = pr["px"][gi[sel]], pr["py"][gi[sel]]
        A[sel], B[sel], C[sel] = (np.asarray(c, np.float64)[gi[sel]] for c in pr["conic"])
    o = np.asarray(gs.opacity, np.float64)[gi]
    need = np.zeros(n, np.uint32)
    r = np.arange(16)
    xs = (tx[:, None] * 16 + r[None, :]).astype(np.float64) + 0.5          # [n, 16] pixel-centre columns
    xin = xs < W
    for row in range(16):
        y = ty * 16 + row
        dy = (y + 0.5) - py
        dx = xs - px[:, None]
        q = A[:, None] * dx * dx + 2 * B[:, None] * dx * dy[:, None] + C[:, None] * dy[:, None] ** 2
        hit = ((o[:, None] * np.exp(-0.5 * q) >= 1 / 255) & xin).any(1) & (y < H)
        need |= np.where(hit, np.uint32(1 << (row // 4)), np.uint32(0))
    say(f"row bands ({kind}): {n} pairs, {(bands != 0xF).mean():.2f} with a band skipped, "
        f"{np.count_nonzero(need & ~bands)} pairs missing a needed band")
    assert not np.any(need & ~bands)
    # (large footprints skip bands only in their first and last tile rows)
    assert (bands != 0xF).mean() > dict(small=0.5, needles=0.01, overflow=0.02)[kind]


@pytest.mark.parametrize("tile", [8, 16])
def test_pair_lists_large_footprints(tile):
    """Rectangles of more than 32 tiles take the wave-cooperative counting and emission paths; mixed
    with small ones so that blocks hold both kinds (up to a whole block of large ones)."""
    api = _api()
    big = vi.random_gaussians(1500, 12, log_scale_mean=-1.8)
    small = vi.random_gaussians(1500, 13, log_scale_mean=-3.2)
    gs = vi.GaussianSet.concat([small, big])
    cams = vi.orbit_cameras(2, 160, 120, azimuth0=0.7)
    say(f"large footprints tile={tile} n={gs.n}")
    P = to_dev(gs)
    rp = api.plan_batch(cams, [0, gs.n], tile=tile, pair_capacity=1 << 20)
    out = api.render_fwd(rp, P)
    torch.cuda.synchronize()
    ref = binning.pair_lists(gs, cams, tile)
    assert int(out.status[0]) == 0 and int(out.status[1]) == ref["tile"].size
    ntl = rp.region("item_ntiles", torch.int32).cpu().numpy()
    I = int(rp.plan.n_items)
    bins = rp.region("item_rect", torch.int32).cpu().numpy().view(np.uint32).reshape(-1, 4)[:I]
    rx, ry = bins[:, 0], bins[:, 1] & 0x0FFF0FFF
    area = ((rx >> 16) - (rx & 0xFFFF)) * ((ry >> 16) - (ry & 0xFFFF))
    assert (area > 32).sum() > 300 and (area[ntl > 0] <= 32).sum() > 1000
    for v in range(2):
        assert np.array_equal(ntl[v * gs.n:(v + 1) * gs.n], ref["proj"][v]["n_tiles"])
    n = ref["tile"].size
    assert np.array_equal(rp.region("pair_tile", torch.int32).cpu().numpy()[:n], ref["tile"])
    assert np.array_equal(rp.region("pair_item", torch.int32).cpu().numpy()[:n] & ITEM_MASK, ref["item"])


def test_large_footprints_beyond_the_ballot_word_buffer():
    """Large rectangles keep the projection's 64-tile ballots in a word buffer of max(n_items / 4, 1024)
    words that the emission reads back; rectangles that find it full are tested again by the emission.
    Footprints large enough to overflow it exercise both in one batch: pair lists bit-exact."""
    api = _api()
    gs = vi.random_gaussians(1200, 14, log_scale_mean=-1.5, log_scale_std=0.3)
    cams = vi.orbit_cameras(1, 256, 192, azimuth0=0.4)
    P = to_dev(gs)
    rp = api.plan_batch(cams, [0, gs.n], tile=8, pair_capacity=1 << 21)
    out = api.render_fwd(rp, P)
    torch.cuda.synchronize()
    ref = binning.pair_lists(gs, cams, 8)
    n = ref["tile"].size
    say(f"large footprints, word buffer overflow: {n} pairs")
    assert int(out.status[0]) == 0 and int(out.status[1]) == n
    I = int(rp.plan.n_items)
    cap = int(rp.plan.region_bytes[22]) // 8
    assert cap == max(I // 4, 1024)
    taken = int(rp.region("counters", torch.int32).cpu().numpy().view(np.uint64)[2])
    bins = rp.region("item_rect", torch.int32).cpu().numpy().view(np.uint32).reshape(-1, 4)[:I]
    rx, ry = bins[:, 0], bins[:, 1] & 0x0FFF0FFF
    area = ((rx >> 16) - (rx & 0xFFFF)) * ((ry >> 16) - (ry & 0xFFFF))
    large = (area > 32) & (ref["proj"][0]["n_tiles"] > 0)
    assert taken == int(((area[area > 32] + 63) // 64).sum()) and taken > cap
    first = bins[:, 2]
    stored = large & (first != 0xFFFFFFFF)
    assert stored.sum() > 10 and (large & ~stored).sum() > 10
    assert np.array_equal(rp.region("item_ntiles", torch.int32).cpu().numpy()[:I], ref["proj"][0]["n_tiles"])
    assert np.array_equal(rp.region("pair_tile", torch.int32).cpu().numpy()[:n], ref["tile"])
    assert np.array_equal(rp.region("pair_item", torch.int32).cpu().numpy()[:n] & ITEM_MASK, ref["item"])


# Opacities up to 1 and larger footprints: Gaussians whose alpha reaches the 0.99 clamp near their
# centre (a few pixels per view), mixed with ones that cannot reach it.
HIGH_OPACITY = dict(opacity=(0.9, 1.0), log_scale=-2.0)


# (the cases with lds > 0 stage the compositing lists in LDS batches of 32 or 64 entries)
@pytest.mark.parametrize("tile,W,H,lds,opacity", [(16, 64, 64, 0, None), (16, 101, 67, 0, None), (8, 50, 37, 0, None),
                                                  (32, 96, 80, 0, None), (16, 101, 67, 32, None),
                                                  (16, 64, 64, 64, None), (8, 50, 37, 64, None),
                                                  (16, 101, 67, 0, HIGH_OPACITY), (16, 101, 67, 32, HIGH_OPACITY),
                                                  (8, 50, 37, 0, HIGH_OPACITY), (32, 96, 80, 0, HIGH_OPACITY)])
def test_forward_backward_parity(tile, W, H, lds, opacity):
    api = _api()
    gs, cams = _scene(600, 3, 2, W, H, **(opacity or {}))
    say(f"fwd/bwd parity tile={tile} {W}x{H} n={gs.n} lds batch {lds}")
    P = to_dev(gs)
    rp = api.plan_batch(cams, [0, gs.n], tile=tile, pair_capacity=1 << 18, lds_batch=lds, lds_batch_bwd=lds)
    out = api.render_fwd(rp, P)
    batch = render.Batch(gs, cams, tile)
    ref = render.render_forward(batch)
    imgs = [t.cpu().numpy() for t in api.split_views(out.image, cams)]
    fts = [t.cpu().numpy() for t in api.split_views(out.final_T, cams, 1)]
    ncs = [t.cpu().numpy() for t in api.split_views(out.n_contrib, cams, 1)]
    for v in range(len(cams)):
        err = image_error(imgs[v], ref[v]["image"], ref[v]["flagged"])
        say(f"  view {v}: image err {err:.2e}, flagged {int(ref[v]['flagged'].sum())}")
        assert err <= IMG_TOL
        ok = ~ref[v]["flagged"]
        assert np.abs(fts[v] - ref[v]["final_T"])[ok].max() <= 1e-5
        # the number of list entries each pixel took into account (its stop position, else the list length)
        assert np.array_equal(ncs[v][ok], ref[v]["n_visited"][ok])
    dL = masked_dL(cams, [r["flagged"] for r in ref], seed=tile)
    grads = api.render_bwd(rp, P, flat(dL), out)
    g_ref, g2_ref = render.render_backward(batch, dL)
    G = grads.cpu().numpy()
    for name, rows in ROWS.items():
        e = group_error(G[rows], g_ref[name].reshape(rows.stop - rows.start, -1))
        say(f"  grad {name}: {e:.2e}")
        assert e <= GRAD_TOL, name
    # the region keeps the raw moments of dL/dpower; with power = -(A dx^2 + 2 B dx dy + C dy^2) / 2
    # and alpha = o exp(power) the 2D gradients are linear in them, given the item's conic and opacity
    mo = rp.region("grad2d", torch.float32).cpu().numpy().reshape(-1, 16)[:, :9].astype(np.float64)
    rec = rp.region("item_rec", torch.float32).cpu().numpy().reshape(-1, 4)[: len(mo)].astype(np.float64)
    nt = rp.region("item_ntiles", torch.int32).cpu().numpy()[: len(mo)]
    A, B, C, o = rec[:, 0], rec[:, 1], rec[:, 2], np.where(nt > 0, rec[:, 3], 1.0)
    g2 = np.stack([-(A * mo[:, 0] + B * mo[:, 1]), -(B * mo[:, 0] + C * mo[:, 1]), -0.5 * mo[:, 2], -mo[:, 3],
                   -0.5 * mo[:, 4], mo[:, 5] / o, mo[:, 6], mo[:, 7], mo[:, 8]])
    g2[:, nt == 0] = 0.0
    for name, rows, ref2 in (("mean2d", slice(0, 2), g2_ref["mean2d"].T), ("conic", slice(2, 5), g2_ref["conic"].T),
                             ("opacity", slice(5, 6), g2_ref["opacity"][None]), ("rgb", slice(6, 9), g2_ref["rgb"].T)):
        e = group_error(g2[rows], ref2)
        assert e <= GRAD_TOL, name


def test_tile_launch_order_is_longest_list_first():
    """The compositing launch order (last quarter of workspace region 21) is a permutation of the
    tiles whose list lengths, in steps of 8 entries, never increase; equal steps keep tile order."""
    api = _api()
    gs, cams = _scene(4000, 17, 2, 150, 90, log_scale=-2.6)
    P = to_dev(gs)
    rp = api.plan_batch(cams, [0, gs.n], tile=8, pair_capacity=1 << 20)
    out = api.render_fwd(rp, P)
    torch.cuda.synchronize()
    assert int(out.status[0]) == 0
    nt = int(rp.plan.n_tiles)
    off = int(rp.plan.region_offset[21])
    order = rp.ws[off:off + 16 * nt].view(torch.int32).cpu().numpy()[3 * nt:]
    assert np.array_equal(np.sort(order), np.arange(nt))
    ranges = rp.region("ranges", torch.int32).cpu().numpy().reshape(-1, 2)
    step = np.minimum((ranges[:, 1] - ranges[:, 0]) >> 3, 255)[order]
    assert np.all(np.diff(step) <= 0) and step[0] > step[-1]
    for k in np.unique(step):
        assert np.all(np.diff(order[step == k]) > 0)


def test_empty_and_fully_culled_views():
    api = _api()
    gs, cams = _scene(50, 5, 1, 40, 30)
    gs.means[2] += 10.0   # everything behind the camera or far off-screen
    cams2 = [vi.Camera(width=40, height=30, fx=30.0, fy=30.0, cx=20.0, cy=15.0, near=0.2,
                       viewmat=vi.look_at(np.array([0.0, 0.0, -50.0]), target=np.array([0.0, 0.0, -60.0]),
                                          up=np.array([0.0, 1.0, 0.0])).astype(np.float32))]
    P = to_dev(gs)
    rp = api.plan_batch(cams2, [0, gs.n], tile=16, pair_capacity=1024)
    out = api.render_fwd(rp, P)
    torch.cuda.synchronize()
    assert int(out.status[1]) == 0 and int(out.status[2]) == 0
    assert torch.all(out.final_T == 1.0) and torch.all(out.image == 0.0) and torch.all(out.n_contrib == 0)
    g = api.render_bwd(rp, P, torch.ones_like(out.image), out)
    assert torch.all(g == 0.0)


def test_capacity_overflow_is_flagged():
    api = _api()
    gs, cams = _scene(800, 8, 1, 64, 64)
    P = to_dev(gs)
    rp = api.plan_batch(cams, [0, gs.n], tile=16, pair_capacity=100)
    out = api.render_fwd(rp, P)
    torch.cuda.synchronize()
    assert int(out.status[0]) == 1 and int(out.status[1]) > 100
    api.render_fwd(rp, P, out)                      # a second overflowing forward into the same status
    torch.cuda.synchronize()
    assert int(out.status[3]) == 2
    rp2 = api.plan_batch(cams, [0, gs.n], tile=16, pair_capacity=int(out.status[1]))
    out2 = api.render_fwd(rp2, P)
    torch.cuda.synchronize()
    assert int(out2.status[0]) == 0


@pytest.mark.parametrize("opacity", [(0.05, 0.95), LOW_OPACITY])
def test_batched_equals_plain_and_multiscene(opacity):
    api = _api()
    s1, _ = _scene(300, 21, 1, 60, 40, opacity=opacity)
    s2, _ = _scene(900, 22, 1, 60, 40, log_scale=-3.5, opacity=opacity)
    gs = vi.GaussianSet.concat([s1, s2])
    cams = vi.orbit_cameras(2, 72, 56) + vi.orbit_cameras(2, 40, 33, azimuth0=1.0)
    view_scene = [0, 1, 1, 0]
    so = [0, s1.n, s1.n + s2.n]
    say("batched vs plain, 2 scenes, 4 uneven views")
    P = to_dev(gs)
    rp = api.plan_batch(cams, so, view_scene, tile=16, pair_capacity=1 << 18)
    out = api.render_fwd(rp, P)
    imgs = api.split_views(out.image, cams)
    for v, cam in enumerate(cams):
        rpv = api.plan_batch([cam], so, [view_scene[v]], tile=16, pair_capacity=1 << 16, mode="exact")
        ov = api.render_fwd(rpv, P)
        torch.cuda.synchronize()
        assert torch.equal(ov.image.view(3, cam.height, cam.width), imgs[v])
    # multi-scene oracle parity
    batch = render.Batch(gs, cams, 16, view_scene, so)
    ref = render.render_forward(batch)
    for v in range(len(cams)):
        assert image_error(imgs[v].cpu().numpy(), ref[v]["image"], ref[v]["flagged"]) <= IMG_TOL
    dL = masked_dL(cams, [r["flagged"] for r in ref], seed=5)
    grads = api.render_bwd(rp, P, flat(dL), out)
    g_ref, _ = render.render_backward(batch, dL)
    G = grads.cpu().numpy()
    for name, rows in ROWS.items():
        assert group_error(G[rows], g_ref[name].reshape(rows.stop - rows.start, -1)) <= GRAD_TOL, name


def test_forward_is_deterministic_and_accumulate_adds():
    api = _api()
    gs, cams = _scene(1500, 31, 2, 90, 70)
    P = to_dev(gs)
    rp = api.plan_batch(cams, [0, gs.n], tile=16, pair_capacity=1 << 18)
    a = api.render_fwd(rp, P)
    img_a = a.image.clone()
    b = api.render_fwd(rp, P)
    assert torch.equal(img_a, b.image)
    dL = torch.randn_like(b.image)
    g1 = api.render_bwd(rp, P, dL, b)
    g2 = api.render_bwd(rp, P, dL, b, grads=g1.clone(), accumulate=True)
    assert torch.allclose(g2, 2 * g1, rtol=1e-5, atol=1e-7 * float(g1.abs().max()))


def test_autograd_function_matches_oracle():
    """The torch.autograd.Function around the forward and backward: image = render(P) for a planned
    batch, a torch loss on it, and P.grad against the oracle's gradient of the same loss."""
    from paper_2601_09417_amd import trainer
    api = _api()
    gs, cams = _scene(1200, 41, 2, 72, 56)
    say("autograd Function, 2 views 72x56")
    P = to_dev(gs).requires_grad_(True)
    rp = api.plan_batch(cams, [0, gs.n], tile=16, pair_capacity=1 << 18)
    img = trainer.VBMRender.apply(P, rp)
    batch = render.Batch(gs, cams, 16)
    ref = render.render_forward(batch)
    for v, got in enumerate(api.split_views(img.detach(), cams)):
        assert image_error(got.cpu().numpy(), ref[v]["image"], ref[v]["flagged"]) <= IMG_TOL, v
    dL = masked_dL(cams, [r["flagged"] for r in ref], seed=42)
    w = flat(dL)
    (img * w).sum().backward()
    g_ref, _ = render.render_backward(batch, dL)
    G = P.grad.cpu().numpy()
    for name, rows in ROWS.items():
        assert group_error(G[rows], g_ref[name].reshape(rows.stop - rows.start, -1)) <= GRAD_TOL, name


def test_autograd_two_forwards_on_one_plan():
    """Two renders through one plan before either backward (a second loss, a re-render): the plan's
    workspace holds only the later forward's lists, so each backward re-runs its own forward first.
    Both gradients match the oracle's; a raw backward with the stale forward output is refused; a
    render whose pairs overflow the plan raises instead of returning an incomplete image."""
    from paper_2601_09417_amd import _lib as L
    from paper_2601_09417_amd import trainer
    api = _api()
    gs1, cams = _scene(1000, 45, 2, 72, 56)
    gs2 = vi.GaussianSet(gs1.means + np.float32(0.03) * np.random.default_rng(1).normal(size=gs1.means.shape).astype(
        np.float32), gs1.scales * np.float32(1.2), gs1.quats, np.clip(gs1.opacity * np.float32(0.9), 0.01, 0.99),
        gs1.rgb[::-1].copy())
    say("autograd Function: two forwards on one plan, then both backwards")
    rp = api.plan_batch(cams, [0, gs1.n], tile=16, pair_capacity=1 << 18)
    P1 = to_dev(gs1).requires_grad_(True)
    P2 = to_dev(gs2).requires_grad_(True)
    img1 = trainer.VBMRender.apply(P1, rp)
    img2 = trainer.VBMRender.apply(P2, rp)
    refs, dLs = [], []
    for k, gs in enumerate((gs1, gs2)):
        batch = render.Batch(gs, cams, 16)
        ref = render.render_forward(batch)
        refs.append((batch, ref))
        dLs.append(masked_dL(cams, [r["flagged"] for r in ref], seed=50 + k))
    for img, (batch, ref) in zip((img1, img2), refs):
        for v, got in enumerate(api.split_views(img.detach(), cams)):
            assert image_error(got.cpu().numpy(), ref[v]["image"], ref[v]["flagged"]) <= IMG_TOL, v
    (img1 * flat(dLs[0])).sum().backward()
    (img2 * flat(dLs[1])).sum().backward()
    for P, (batch, _), dL in ((P1, refs[0], dLs[0]), (P2, refs[1], dLs[1])):
        g_ref, _ = render.render_backward(batch, dL)
        G = P.grad.cpu().numpy()
        for name, rows in ROWS.items():
            assert group_error(G[rows], g_ref[name].reshape(rows.stop - rows.start, -1)) <= GRAD_TOL, name
    a = api.render_fwd(rp, P1.detach())
    api.render_fwd(rp, P2.detach())
    with pytest.raises(L.VBMError):
        api.render_bwd(rp, P1.detach(), torch.ones_like(a.image), a)
    small = api.plan_batch(cams, [0, gs1.n], tile=16, pair_capacity=64)
    with pytest.raises(L.VBMError):
        trainer.VBMRender.apply(P1, small)
