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


def group_error(gpu: np.ndarray, ref: np.ndarray, floor: float = 0.0) -> float:
    """max |gpu - ref| / max |ref| (the denominator floored at ``floor`` and at 1e-12)."""
    scale = max(float(np.abs(ref).max()), floor, 1e-12)
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


def oracle_gaussians(vol, tf, J, wav, K):
    """The oracle's Gaussian set for a volume: its FP64 DWT of TF(F) per channel, rounded to float32
    (the coefficients both sides select from), its top-K and its construction (s_mode none), as a
    float32 GaussianSet.  Returns (coefficients float32 [4][G^3], kept, construction dict, set)."""
    from oracle import bank as obank
    from oracle import construct as oconstruct
    from oracle import dwt as odwt
    from oracle import select as oselect
    from oracle import tf as otf
    G = vol.shape[0]
    rf = otf.apply(vol, tf.xs, tf.rgba)                       # [4][z][y][x] FP64
    coeffs = np.empty((4, G ** 3), np.float32)
    for c in range(4):
        coeffs[c] = odwt.pack(odwt.dwt3d(rf[c], J, wav), G, J)
    del rf
    Ks = [K] if np.ndim(K) == 0 else list(K)
    out = []
    for k in Ks:
        kept = oselect.topk(coeffs, k)
        ref = oconstruct.construct(coeffs, kept, G, J, obank.build_bank(wav, J), s_mode="none")
        f = np.float32
        gs = vi.GaussianSet(ref["means"].astype(f), ref["scales"].astype(f), ref["quats"].astype(f),
                            ref["opacity"].astype(f), ref["rgb"].astype(f))
        out.append((kept, ref, gs))
    return coeffs, out


def sampled_tile_parity(rp, P, gs, cams, view_scene, scene_offsets, tile, sample_views, n_random, seed):
    """Forward and backward of one planned batch against the oracle on sampled tiles.

    For every sampled view: the oracle's pair lists of the view's scene (float32 decisions) against
    the GPU's, the view's whole list, pair count and every tile's range bit for bit; the images of
    n_random random non-empty tiles and of the view's longest tile against the oracle's FP64
    compositing (at pixels the oracle flags as near a threshold, against every outcome the branch
    there allows).  Then dL/dI is random on those tiles and zero elsewhere, so every Gaussian's
    gradient is the oracle's autodiff over the same tiles (and exactly zero for Gaussians in none of
    them).  Returns the sampled tiles, the GPU gradient [14][N], the involved Gaussians and the
    oracle's gradient of those ({group: [rows][n]})."""
    from oracle import binning, render
    from paper_2601_09417_amd import api
    out = api.render_fwd(rp, P)
    torch.cuda.synchronize()
    assert int(out.status[0]) == 0, "pair capacity overflow"
    N = P.shape[1]
    so = np.asarray(scene_offsets, np.int64)
    toff = binning.tile_grid(cams, tile)
    ioff = binning.item_offsets(view_scene, so)
    n_pairs = int(out.status[1])
    ptile = rp.region("pair_tile", torch.int32).cpu().numpy()[:n_pairs]
    pitem = rp.region("pair_item", torch.int32).cpu().numpy()[:n_pairs] & ITEM_MASK
    ranges = rp.region("ranges", torch.int32).cpu().numpy().reshape(-1, 2)
    assert np.all(np.diff(ptile.view(np.uint32).astype(np.int64)) >= 0)
    imgs = [t.cpu().numpy() for t in api.split_views(out.image, cams)]
    rng = np.random.default_rng(seed)
    dL = [np.zeros((3, c.height, c.width), np.float32) for c in cams]
    tiles = []                  # (view, scene-global Gaussian indices of the list, pixel xs, ys, dL values)
    err_img, img_max = 0.0, 0.0
    flag_err, n_flagged = 0.0, 0
    for v in sample_views:
        cam, s = cams[v], view_scene[v]
        s0, s1 = int(so[s]), int(so[s + 1])
        sub = gs.subset(np.arange(s0, s1))
        ref = binning.pair_lists(sub, [cam], tile)
        TX = -(-cam.width // tile)
        lens = ref["ranges"][:, 1] - ref["ranges"][:, 0]
        # the view's whole list, its pair count and every tile's range
        va, vb = np.searchsorted(ptile, [toff[v], toff[v + 1]])
        assert vb - va == ref["tile"].size, (v, vb - va, ref["tile"].size)
        assert np.array_equal(ptile[va:vb], ref["tile"] + toff[v])
        assert np.array_equal(pitem[va:vb] - ioff[v], ref["item"]), v
        rv = ranges[toff[v]:toff[v + 1]].astype(np.int64)
        ne = lens > 0
        assert np.array_equal(rv[ne] - va, ref["ranges"][ne]), v
        assert np.all(rv[~ne, 1] == rv[~ne, 0]), v
        say(f"  view {v}: {ref['tile'].size} pairs, every tile's list and range bit-exact")
        nonempty = np.nonzero(lens > 0)[0]
        pick = rng.choice(nonempty, min(n_random, nonempty.size), replace=False)
        for lt in np.unique(np.concatenate([pick, [int(np.argmax(lens))]])):
            a, b = ref["ranges"][lt]
            ga, gb = ranges[toff[v] + lt]
            assert gb - ga == b - a, (v, lt, gb - ga, b - a)
            assert np.array_equal(ptile[ga:gb], np.full(b - a, toff[v] + lt))
            local = ref["item"][a:b]
            assert np.array_equal(pitem[ga:gb] - ioff[v], local), (v, lt)
            glob = s0 + local
            xs, ys = render._tile_pixels(cam, tile, int(lt % TX), int(lt // TX))
            it = torch.as_tensor(glob, dtype=torch.int64)
            m2d, con, _ = render.project_fp64(render._t(gs.means)[:, it], render._t(gs.scales)[:, it],
                                              render._t(gs.quats)[:, it], cam)
            pix = torch.stack([render._t(xs + 0.5), render._t(ys + 0.5)], 1)
            col, _, _, fl, _ = render.composite_tile(pix, m2d, con, render._t(gs.opacity)[it],
                                                     render._t(gs.rgb)[:, it].T, render._t(cam.bg))
            col, fl = col.numpy(), fl.numpy()
            gpu_px = imgs[v][:, ys, xs].T
            err_img = max(err_img, float(np.abs(gpu_px - col)[~fl].max(initial=0.0)))
            img_max = max(img_max, float(np.abs(col).max()))
            if fl.any():
                # several results are correct at a flagged pixel: the GPU value must be one of them
                m2n, cn = m2d.numpy(), con.numpy()
                opn, rgbn = np.asarray(gs.opacity, np.float64)[glob], np.asarray(gs.rgb, np.float64)[:, glob].T
                for p_ in np.nonzero(fl)[0]:
                    outs = render.composite_pixel_outcomes(xs[p_] + 0.5, ys[p_] + 0.5, range(glob.size), m2n, cn, opn,
                                                           rgbn, np.asarray(cam.bg, np.float64))
                    e = min(float(np.abs(gpu_px[p_] - np.asarray(o[0])).max()) for o in outs)
                    flag_err = max(flag_err, e)
                    n_flagged += 1
            d = rng.normal(size=(3, xs.size)).astype(np.float32)
            d[:, fl] = 0.0
            dL[v][:, ys, xs] = d
            tiles.append((v, glob, xs, ys, d))
    assert err_img <= IMG_TOL * max(img_max, 1e-6), (err_img, img_max)
    assert flag_err <= IMG_TOL * max(img_max, 1e-6), (flag_err, img_max)
    say(f"  {len(tiles)} sampled tiles in {len(sample_views)} views: image error {err_img / max(img_max, 1e-6):.2e}; "
        f"{n_flagged} flagged pixels, each within {flag_err / max(img_max, 1e-6):.2e} of a correct outcome")

    g = api.render_bwd(rp, P, flat(dL), out).cpu().numpy()
    involved = np.unique(np.concatenate([t[1] for t in tiles]))
    assert np.all(np.delete(g, involved, axis=1) == 0.0)
    inv = torch.as_tensor(involved, dtype=torch.int64)
    leaf = {k: render._t(np.asarray(getattr(gs, k), np.float64))[..., inv].clone().requires_grad_(True)
            for k in ("means", "scales", "quats", "opacity", "rgb")}
    pos = {int(gi): i for i, gi in enumerate(involved)}
    total = 0.0
    for v, glob, xs, ys, d in tiles:
        loc = torch.as_tensor([pos[int(i)] for i in glob], dtype=torch.int64)
        m2d, con, _ = render.project_fp64(leaf["means"][:, loc], leaf["scales"][:, loc], leaf["quats"][:, loc],
                                          cams[v])
        pix = torch.stack([render._t(xs + 0.5), render._t(ys + 0.5)], 1)
        col, _, _, _, _ = render.composite_tile(pix, m2d, con, leaf["opacity"][loc], leaf["rgb"][:, loc].T,
                                                render._t(cams[v].bg))
        total = total + (col * render._t(d.T.astype(np.float64))).sum()
    total.backward()
    oracle_grad = {name: leaf[name].grad.numpy().reshape(rows.stop - rows.start, -1) for name, rows in ROWS.items()}
    for name, rows in ROWS.items():
        r = oracle_grad[name]
        # The rotation of an isotropic Gaussian does not change it, so its quaternion gradient is
        # exactly zero (every Haar bank entry is isotropic); the group is then measured against the
        # size the quaternion gradient has when the Gaussian is anisotropic, max |dL/ds| s, the
        # magnitude of dL/dSigma s^2 that dSigma/dq carries.
        floor = (float(np.abs(oracle_grad["scales"] * np.asarray(gs.scales, np.float64)[:, involved]).max())
                 if name == "quats" else 0.0)
        e = group_error(g[rows][:, involved], r, floor)
        say(f"  grad {name}: {e:.2e} over {involved.size} Gaussians")
        assert e <= GRAD_TOL, name
    return tiles, g, involved, oracle_grad
