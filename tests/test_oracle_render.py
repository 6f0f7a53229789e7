"""Pins of the oracle rasteriser: closed forms, brute force, invariants and finite differences."""
import math

import numpy as np
import pytest

import vbm_inputs as vi
from oracle import binning, render


def _axis_camera(W=65, H=49, f=60.0):
    """Camera at (0, -3, 0) looking along +y (OpenCV axes: x right = +x, y down = -z)."""
    return vi.Camera(width=W, height=H, fx=f, fy=f, cx=W / 2.0, cy=H / 2.0, near=0.2,
                     viewmat=vi.look_at(np.array([0.0, -3.0, 0.0])).astype(np.float32))


def _one(mean, sigma, op, rgb, quat=(1, 0, 0, 0)):
    f = np.float32
    return vi.GaussianSet(np.array(mean, f).reshape(3, 1), np.full((3, 1), sigma, f), np.array(quat, f).reshape(4, 1),
                          np.array([op], f), np.array(rgb, f).reshape(3, 1))


def test_single_isotropic_gaussian_closed_form():
    """On the optical axis at depth z, an isotropic sigma projects to sigma2^2 = f^2 sigma^2 / z^2 + 0.3 and the image
    is c * min(0.99, o exp(-|p - m|^2 / (2 sigma2^2))) wherever alpha >= 1/255 inside the tile rectangle."""
    cam = _axis_camera()
    z, sigma, op, rgb = 3.0, 0.05, 0.8, (0.9, 0.4, 0.2)
    gs = _one((0.0, 0.0, 0.0), sigma, op, rgb)
    b = render.Batch(gs, [cam], 16)
    out = render.render_forward(b)[0]
    s2 = cam.fx ** 2 * float(np.float32(sigma)) ** 2 / z ** 2 + 0.3
    pr = b.pairs["proj"][0]
    x0, x1, y0, y1 = (int(pr[k][0]) for k in ("x0", "x1", "y0", "y1"))
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    d2 = (xs + 0.5 - cam.cx) ** 2 + (ys + 0.5 - cam.cy) ** 2
    a = np.minimum(0.99, float(np.float32(op)) * np.exp(-d2 / (2 * s2)))
    inside = (xs // 16 >= x0) & (xs // 16 < x1) & (ys // 16 >= y0) & (ys // 16 < y1)
    a = np.where(inside & (a >= 1 / 255), a, 0.0)
    for ch in range(3):
        assert np.abs(out["image"][ch] - float(np.float32(rgb[ch])) * a).max() <= 1e-12
    assert np.abs(out["final_T"] - (1 - a)).max() <= 1e-12
    # the rectangle covers at least the 3-sigma disc
    r = 3 * math.sqrt(s2)
    assert x0 * 16 <= cam.cx - r and x1 * 16 >= cam.cx + r and y0 * 16 <= cam.cy - r and y1 * 16 >= cam.cy + r


def test_two_gaussians_over_operator():
    cam = _axis_camera()
    g1 = _one((0.0, -0.5, 0.0), 0.2, 0.6, (1.0, 0.0, 0.0))     # nearer (depth 2.5)
    g2 = _one((0.0, 0.5, 0.0), 0.2, 0.7, (0.0, 1.0, 0.0))      # farther (depth 3.5)
    gs = vi.GaussianSet.concat([g2, g1])
    b = render.Batch(gs, [cam], 16)
    out = render.render_forward(b)[0]
    i, j = cam.height // 2, cam.width // 2
    a1 = min(0.99, float(np.float32(0.6)))       # both centred on the axis: exp(0) at the centre sample
    a2 = min(0.99, float(np.float32(0.7)))
    expect_r = a1 * 1.0
    expect_g = a2 * (1 - a1)
    # the centre pixel samples (W/2, H/2) exactly because W, H are odd
    assert abs(out["image"][0, i, j] - expect_r) <= 1e-12
    assert abs(out["image"][1, i, j] - expect_g) <= 1e-12
    assert abs(out["final_T"][i, j] - (1 - a1) * (1 - a2)) <= 1e-12


def _scene(n=250, seed=4, W=64, H=48, views=2):
    gs = vi.random_gaussians(n, seed, log_scale_mean=-3.0)
    return gs, vi.orbit_cameras(views, W, H)


def test_tiled_equals_bruteforce_per_pixel():
    gs, cams = _scene()
    b = render.Batch(gs, cams, 16)
    out = render.render_forward(b)
    P = b.leaf_params()
    m2d, con, op, rgb = (t.detach().numpy() for t in b.project_items(P))
    for v, cam in enumerate(cams):
        pr = b.pairs["proj"][v]
        ioff = b.pairs["item_offset"][v]
        rng = np.random.default_rng(v)
        for _ in range(60):
            x, y = int(rng.integers(cam.width)), int(rng.integers(cam.height))
            tx, ty = x // 16, y // 16
            rep, rtx, rty = pr["reached"]
            cand = [int(g) for g in rep[(rtx == tx) & (rty == ty)]]
            cand.sort(key=lambda g: (int(pr["depth"][g:g + 1].view(np.uint32)[0]), g))
            items = [ioff + g for g in cand]
            col, T, nc = render.composite_pixel_bruteforce(x + 0.5, y + 0.5, items, m2d, con, op, rgb, cam.bg)
            assert np.abs(np.array(col) - out[v]["image"][:, y, x]).max() <= 1e-12
            assert abs(T - out[v]["final_T"][y, x]) <= 1e-12
            assert nc == out[v]["n_contrib"][y, x]


def test_footprint_culling_drops_only_non_contributing_pairs():
    """Compositing over the full 3-sigma rectangles (no footprint test) gives the same image: every
    dropped (tile, Gaussian) pair has alpha < 1/255 at all pixels of its tile."""
    gs, cams = _scene(n=300, seed=12)
    gs.opacity[:] = np.linspace(0.001, 0.9, gs.n).astype(np.float32)
    b = render.Batch(gs, cams[:1], 16)
    out = render.render_forward(b)[0]
    P = b.leaf_params()
    m2d, con, op, rgb = (t.detach().numpy() for t in b.project_items(P))
    pr = binning.project_fp32(gs.means, gs.scales, gs.quats, cams[0], 16)      # no opacity: full rectangles
    dropped = int(pr["n_tiles"].sum()) - int(b.pairs["tile"].size)
    assert dropped > 0
    cam = cams[0]
    for y in range(0, cam.height, 3):
        for x in range(0, cam.width, 3):
            tx, ty = x // 16, y // 16
            cand = [g for g in range(gs.n) if pr["n_tiles"][g] > 0 and pr["x0"][g] <= tx < pr["x1"][g]
                    and pr["y0"][g] <= ty < pr["y1"][g]]
            cand.sort(key=lambda g: (int(pr["depth"][g:g + 1].view(np.uint32)[0]), g))
            col, T, _ = render.composite_pixel_bruteforce(x + 0.5, y + 0.5, cand, m2d, con, op, rgb, cam.bg)
            assert np.abs(np.array(col) - out["image"][:, y, x]).max() <= 1e-12
            assert abs(T - out["final_T"][y, x]) <= 1e-12


def test_pair_list_invariants():
    gs, cams = _scene(views=3)
    b = render.Batch(gs, cams, 16)
    p = b.pairs
    total = sum(int(pr["n_tiles"].sum()) for pr in p["proj"])
    assert p["tile"].size == total
    key = np.stack([p["tile"], p["depth_bits"], p["item"]], 1)
    assert all(tuple(key[i]) < tuple(key[i + 1]) for i in range(len(key) - 1))
    r = p["ranges"]
    assert r[0, 0] == 0 and r[-1, 1] == total
    assert np.all(r[1:, 0] == r[:-1, 1])
    # a batch of views = the single-view lists concatenated by tile offset
    for v in range(3):
        pv = binning.pair_lists(gs, [cams[v]], 16)
        s, e = r[p["tile_offset"][v]], r[p["tile_offset"][v + 1] - 1]
        sl = slice(s[0], e[1])
        assert np.array_equal(p["tile"][sl] - p["tile_offset"][v], pv["tile"])
        assert np.array_equal(p["item"][sl] - p["item_offset"][v], pv["item"])


def test_transmittance_monotone_and_bounded():
    gs, cams = _scene(n=400, seed=9)
    gs.opacity[:] = 0.95
    b = render.Batch(gs, cams[:1], 16)
    out = render.render_forward(b)[0]
    assert np.all(out["final_T"] <= 1.0) and np.all(out["final_T"] >= 0.0)
    P = b.leaf_params()
    m2d, con, op, rgb = b.project_items(P)
    import torch
    for v, tx, ty, gt, xs, ys, it in b.tiles():
        if len(it) == 0:
            continue
        it_t = torch.as_tensor(it)
        pix = torch.stack([torch.as_tensor(xs + 0.5, dtype=torch.float64), torch.as_tensor(ys + 0.5, dtype=torch.float64)], 1)
        _, tf, nc, _, contrib = render.composite_tile(pix, m2d[it_t].detach(), con[it_t].detach(), op[it_t].detach(),
                                                      rgb[it_t].detach(), torch.zeros(3, dtype=torch.float64))
        assert torch.all(tf >= 1e-4)


def test_manual_reverse_recursion_matches_autodiff():
    gs, cams = _scene(n=150, seed=6, W=48, H=32)
    b = render.Batch(gs, cams, 16)
    dL = [np.random.default_rng(1).normal(size=(3, c.height, c.width)) for c in cams]
    _, g2 = render.render_backward(b, dL)
    gm = render.render_backward_manual(b, dL)
    for k in g2:
        assert np.abs(g2[k] - gm[k]).max() <= 1e-10 * max(1.0, np.abs(g2[k]).max())


def _signature(b):
    """Decisions that finite differences must not cross: per-tile contribution masks and clamp states."""
    import torch
    P = b.leaf_params()
    with torch.no_grad():
        m2d, con, op, rgb = b.project_items(P)
    sig = []
    for v, tx, ty, gt, xs, ys, it in b.tiles():
        if len(it) == 0:
            continue
        it_t = torch.as_tensor(it)
        pix = torch.stack([torch.as_tensor(xs + 0.5, dtype=torch.float64), torch.as_tensor(ys + 0.5, dtype=torch.float64)], 1)
        with torch.no_grad():
            dx = m2d[it_t][None, :, 0] - pix[:, None, 0]
            dy = m2d[it_t][None, :, 1] - pix[:, None, 1]
            c = con[it_t]
            pw = -0.5 * (c[None, :, 0] * dx * dx + c[None, :, 2] * dy * dy) - c[None, :, 1] * dx * dy
            clamped = (op[it_t][None] * torch.exp(pw)) > 0.99
            _, _, _, _, contrib = render.composite_tile(pix, m2d[it_t], c, op[it_t], rgb[it_t],
                                                        torch.zeros(3, dtype=torch.float64))
        sig.append(contrib.numpy().tobytes() + clamped.numpy().tobytes())
    return sig


def test_gradient_matches_central_differences():
    gs = vi.random_gaussians(12, 21, extent=0.3, log_scale_mean=-2.0)
    gs.opacity[:] = np.float32(0.6)
    cams = vi.orbit_cameras(2, 32, 32)
    b = render.Batch(gs, cams, 16)
    rng = np.random.default_rng(2)
    dL = [rng.normal(size=(3, c.height, c.width)) for c in cams]
    grads, _ = render.render_backward(b, dL)
    base = {k: v.copy() for k, v in b.params64.items()}
    base_sig = _signature(b)

    def objective():
        out = render.render_forward(b)
        return sum(float((o["image"] * d).sum()) for o, d in zip(out, dL))

    checked = 0
    for key in ("means", "scales", "quats", "opacity", "rgb"):
        arr = base[key]
        for flat in rng.choice(arr.size, size=min(arr.size, 8), replace=False):
            idx = np.unravel_index(flat, arr.shape)
            h = 1e-6 * max(1.0, abs(arr[idx]))
            vals = []
            ok = True
            for sgn in (1, -1):
                b.params64 = {k: v.copy() for k, v in base.items()}
                b.params64[key][idx] += sgn * h
                if _signature(b) != base_sig:
                    ok = False
                    break
                vals.append(objective())
            b.params64 = {k: v.copy() for k, v in base.items()}
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            scale = max(1.0, np.abs(grads[key]).max())
            assert abs(fd - grads[key][idx]) <= 1e-6 * scale, (key, idx, fd, grads[key][idx])
            checked += 1
    assert checked >= 25


def test_footprint_threshold_bounds_the_log():
    """tau(o) >= 2 ln(255 o) with margin for every representable opacity in [1/255, 1]."""
    o = np.linspace(1 / 255, 1.0, 200001).astype(np.float32)
    o = o[o >= binning.ALPHA_MIN32]
    tau = binning.footprint_tau(o).astype(np.float64)
    exact = 2 * np.log(255 * o.astype(np.float64))
    assert np.all(tau >= exact * 1.005 + 0.005)


def _outcome_set(res):
    return sorted((round(c[0], 12), round(c[1], 12), round(c[2], 12), n) for c, _, n in res)


def test_pixel_outcomes_branch_at_thresholds():
    """At a decision that sits on a threshold both outcomes are correct: a Gaussian whose alpha is
    exactly 1/255 is kept or skipped, and one that takes T to 1e-4 (up to rounding) is added or ends
    the pixel.  Away from the thresholds the only outcome is the plain compositing result."""
    m2d = [(0.5, 0.5)] * 3
    con = [(1.0, 0.0, 1.0)] * 3
    rgb = [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)]
    bg = (0.0, 0.0, 0.0)
    # alpha exactly at 1/255 (centred Gaussian: exp(0) = 1)
    op = [1.0 / 255.0, 0.5, 0.3]
    res = render.composite_pixel_outcomes(0.5, 0.5, [0, 1], m2d, con, op, rgb, bg)
    a0 = 1.0 / 255.0
    want = [([a0, 0.5 * (1 - a0), 0.0], None, 2), ([0.0, 0.5, 0.0], None, 2)]
    assert _outcome_set(res) == _outcome_set(want)
    # the second 0.99 takes T to (1 - 0.99)^2 = 1e-4 up to rounding
    op = [0.99, 0.99, 0.3]
    res = render.composite_pixel_outcomes(0.5, 0.5, [0, 1, 2], m2d, con, op, rgb, bg)
    t1 = 1 - 0.99
    add = ([0.99, 0.99 * t1, 0.0], None, 2)          # the third then takes T below 1e-4: stop
    stop = ([0.99, 0.0, 0.0], None, 1)
    assert _outcome_set(res) == _outcome_set([add, stop])
    # nothing near a threshold: one outcome, the plain result
    op = [0.6, 0.5, 0.3]
    res = render.composite_pixel_outcomes(0.5, 0.5, [0, 1, 2], m2d, con, op, rgb, bg)
    col, T, n = render.composite_pixel_bruteforce(0.5, 0.5, [0, 1, 2], m2d, con, op, rgb, bg)
    assert len(res) == 1 and np.allclose(res[0][0], col, atol=0, rtol=0) and res[0][2] == n


def test_stop_position_bounds_the_contributions():
    """n_visited (the stop position, else the list length) is at least n_contrib (the last
    contributor + 1) and every list entry between them fails the alpha test, so a backward that
    takes entries below n_visited with alpha >= 1/255 visits exactly the contributions."""
    gs, cams = _scene(n=400, seed=19)
    gs.opacity[:] = np.float32(0.9)
    b = render.Batch(gs, cams[:1], 16)
    out = render.render_forward(b)[0]
    assert np.all(out["n_visited"] >= out["n_contrib"])
    assert (out["n_visited"] > out["n_contrib"]).any()
    P = b.leaf_params()
    m2d, con, op, rgb = (t.detach().numpy() for t in b.project_items(P))
    cam = cams[0]
    for v, tx, ty, gt, xs, ys, it in b.tiles():
        for x, y in list(zip(xs, ys))[::7]:
            nc, nv = out["n_contrib"][y, x], out["n_visited"][y, x]
            assert nv <= len(it)
            for pos in range(nc, nv):
                i = it[pos]
                dx, dy = m2d[i, 0] - (x + 0.5), m2d[i, 1] - (y + 0.5)
                A, B, C = con[i]
                a = min(0.99, op[i] * math.exp(-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy))
                assert a < 1 / 255
