"""FP32 projection decisions and the sorted (tile, Gaussian) pair lists.  Test infrastructure.

The paper fine-tunes with the 3DGS rasteriser it cites (Sec. 3, 3D Gaussian Splatting; Sec. 4.4)
without specifying it.  The integer outputs of binning -- which tiles a Gaussian touches and the
depth keys that order them -- are decided in float32 here, each operation written out in a fixed
order with no fused multiply-add, so that an implementation following the same order decides
identically bit for bit.  The reading of the cited rasteriser used throughout:

  camera point     Xc = R mu + t (OpenCV axes); culled unless Zc > near
  rotation         q_hat = q / |q|, R_q the usual unit-quaternion rotation matrix
  EWA (2D cov.)    Sigma2 = V V^T + 0.3 I with V = J R_view R_q diag(s)  (= J W Sigma3 W^T J^T)
  Jacobian         J = [[fx/Z, 0, -fx X~/Z^2], [0, fy/Z, -fy Y~/Z^2]], X~ = Z clamp(X/Z, +-1.3 (W/2)/fx)
  culling          det(Sigma2) > 0
  radius           r = ceil(3 sqrt(lambda_max)), lambda_max = mid + sqrt(max(0.1, mid^2 - det))
  pixel centre     mean2d = (fx X/Z + cx, fy Y/Z + cy); pixel (i, j) samples (i + 0.5, j + 0.5)
  tile rectangle   x0 = clamp(floor((px - r)/T), 0, TX), x1 = clamp(floor((px + r)/T) + 1, 0, TX)
  footprint        a pixel gets alpha = o exp(-q/2) >= 1/255 only where q = d^T Sigma2^-1 d <= 2 ln(255 o);
                   a Gaussian with o < 1/255 is dropped, and a tile of the rectangle is kept only when the
                   minimum of q over the rectangle of its pixel centres is <= tau, an upper bound of
                   2 ln(255 o) computed without transcendental functions:
                   tau = 2 * 32 (x^(1/32) - 1) * 1.01 + 0.01, x = 255 o (ln x <= n (x^(1/n) - 1)).
                   Dropped pairs are exactly those whose alpha stays below 1/255 at every pixel of the
                   tile, so the rendered image does not change.
  pair order       ascending (global tile, depth bits as u32, item index)
"""
from __future__ import annotations

import numpy as np

f32 = np.float32
ONE, TWO, HALF, DIL, LIMK, THREE, EIGMIN = f32(1), f32(2), f32(0.5), f32(0.3), f32(1.3), f32(3), f32(0.1)
ALPHA_MIN32 = f32(1) / f32(255)


def footprint_tau(o):
    """float32 upper bound of 2 ln(255 o) (five square roots, no transcendental function)."""
    y = f32(255) * np.asarray(o, dtype=f32)
    for _ in range(5):
        y = np.sqrt(y)
    u = f32(32) * (y - ONE)
    return (TWO * u) * f32(1.01) + f32(0.01)


def tile_reached(mx, my, A, B, C, tau, tx, ty, T, W, H):
    """Vectorised float32 test: does {q <= tau} reach a pixel centre of tile (tx, ty)?"""
    X0 = (tx * T).astype(f32) + HALF
    X1 = np.minimum((tx + 1) * T, W).astype(f32) - HALF
    Y0 = (ty * T).astype(f32) + HALF
    Y1 = np.minimum((ty + 1) * T, H).astype(f32) - HALF
    dx0, dx1, dy0, dy1 = X0 - mx, X1 - mx, Y0 - my, Y1 - my
    inside = (dx0 <= 0) & (dx1 >= 0) & (dy0 <= 0) & (dy1 >= 0)
    B2 = TWO * B

    def q(dx, dy):
        return ((A * dx) * dx + (B2 * dx) * dy) + (C * dy) * dy

    with np.errstate(all="ignore"):
        # Stationary points of q on the four edges: dy = -(B/C) dx on a vertical edge, dx = -(B/A) dy
        # on a horizontal one, with the two ratios rounded once per Gaussian.
        nBC, nBA = -(B / C), -(B / A)
        ya = np.minimum(np.maximum(dx0 * nBC, dy0), dy1)
        yb = np.minimum(np.maximum(dx1 * nBC, dy0), dy1)
        xa = np.minimum(np.maximum(dy0 * nBA, dx0), dx1)
        xb = np.minimum(np.maximum(dy1 * nBA, dx0), dx1)
        qm = np.minimum(np.minimum(q(dx0, ya), q(dx1, yb)), np.minimum(q(xa, dy0), q(xb, dy1)))
    return inside | (qm <= tau)


def _rot_f32(qw, qx, qy, qz):
    n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz
    nq = np.sqrt(n2)
    w, x, y, z = qw / nq, qx / nq, qy / nq, qz / nq
    xx, yy, zz = x * x, y * y, z * z
    xy, xz, yz = x * y, x * z, y * z
    wx, wy, wz = w * x, w * y, w * z
    return [[ONE - TWO * (yy + zz), TWO * (xy - wz), TWO * (xz + wy)],
            [TWO * (xy + wz), ONE - TWO * (xx + zz), TWO * (yz - wx)],
            [TWO * (xz - wy), TWO * (yz + wx), ONE - TWO * (xx + yy)]]


def project_fp32(means, scales, quats, cam, tile: int, opacity=None) -> dict:
    """Per-Gaussian float32 projection decisions for one camera.

    means/scales [3][N], quats [4][N] float32.  Returns depth (float32), rect x0, y0, x1, y1 (int64),
    n_tiles (int64, 0 when culled), radius, px, py and the 2D covariance entries a, b, c.
    """
    m = np.asarray(means, dtype=f32)
    s = np.asarray(scales, dtype=f32)
    q = np.asarray(quats, dtype=f32)
    V = np.asarray(cam.viewmat, dtype=f32)
    fx, fy, cx, cy = f32(cam.fx), f32(cam.fy), f32(cam.cx), f32(cam.cy)
    W, H, T = cam.width, cam.height, int(tile)
    TX, TY = -(-W // T), -(-H // T)
    with np.errstate(all="ignore"):
        Xc = ((V[0, 0] * m[0] + V[0, 1] * m[1]) + V[0, 2] * m[2]) + V[0, 3]
        Yc = ((V[1, 0] * m[0] + V[1, 1] * m[1]) + V[1, 2] * m[2]) + V[1, 3]
        Zc = ((V[2, 0] * m[0] + V[2, 1] * m[1]) + V[2, 2] * m[2]) + V[2, 3]
        vis = Zc > f32(cam.near)
        Rq = _rot_f32(q[0], q[1], q[2], q[3])
        M = [[Rq[i][k] * s[k] for k in range(3)] for i in range(3)]
        limx = LIMK * ((HALF * f32(W)) / fx)
        limy = LIMK * ((HALF * f32(H)) / fy)
        txz = Xc / Zc
        tyz = Yc / Zc
        Xt = np.minimum(limx, np.maximum(-limx, txz)) * Zc
        Yt = np.minimum(limy, np.maximum(-limy, tyz)) * Zc
        z2 = Zc * Zc
        J00 = fx / Zc
        J02 = -((fx * Xt) / z2)
        J11 = fy / Zc
        J12 = -((fy * Yt) / z2)
        A0 = [J00 * V[0, k] + J02 * V[2, k] for k in range(3)]
        A1 = [J11 * V[1, k] + J12 * V[2, k] for k in range(3)]
        V0 = [(A0[0] * M[0][k] + A0[1] * M[1][k]) + A0[2] * M[2][k] for k in range(3)]
        V1 = [(A1[0] * M[0][k] + A1[1] * M[1][k]) + A1[2] * M[2][k] for k in range(3)]
        a = ((V0[0] * V0[0] + V0[1] * V0[1]) + V0[2] * V0[2]) + DIL
        b = (V0[0] * V1[0] + V0[1] * V1[1]) + V0[2] * V1[2]
        c = ((V1[0] * V1[0] + V1[1] * V1[1]) + V1[2] * V1[2]) + DIL
        det = a * c - b * b
        vis &= det > f32(0)
        mid = HALF * (a + c)
        disc = np.maximum(EIGMIN, mid * mid - det)
        lam = mid + np.sqrt(disc)
        r = np.ceil(THREE * np.sqrt(lam))
        px = fx * txz + cx
        py = fy * tyz + cy
        Tf = f32(T)
        x0 = np.minimum(np.maximum(np.floor((px - r) / Tf), f32(0)), f32(TX))
        x1 = np.minimum(np.maximum(np.floor((px + r) / Tf) + ONE, f32(0)), f32(TX))
        y0 = np.minimum(np.maximum(np.floor((py - r) / Tf), f32(0)), f32(TY))
        y1 = np.minimum(np.maximum(np.floor((py + r) / Tf) + ONE, f32(0)), f32(TY))
        vis &= np.isfinite(px) & np.isfinite(py) & np.isfinite(r)
        ca, cb, cc = c / det, -(b / det), a / det
        if opacity is not None:
            op = np.asarray(opacity, dtype=f32)
            vis &= op >= ALPHA_MIN32
    x0 = np.where(vis, x0, 0).astype(np.int64)
    x1 = np.where(vis, x1, 0).astype(np.int64)
    y0 = np.where(vis, y0, 0).astype(np.int64)
    y1 = np.where(vis, y1, 0).astype(np.int64)
    rect_tiles = np.where(vis, (x1 - x0) * (y1 - y0), 0)
    reached = None
    if opacity is not None:
        # expand every rectangle tile, keep those the opacity-aware footprint reaches
        gidx = np.nonzero(rect_tiles > 0)[0]
        cnt = rect_tiles[gidx]
        rep = np.repeat(gidx, cnt)
        start = np.concatenate([[0], np.cumsum(cnt)[:-1]]) if cnt.size else np.zeros(0, np.int64)
        local = np.arange(rep.size) - np.repeat(start, cnt)
        w = (x1 - x0)[rep]
        tx = x0[rep] + local % np.maximum(w, 1)
        ty = y0[rep] + local // np.maximum(w, 1)
        keep = tile_reached(px[rep], py[rep], ca[rep], cb[rep], cc[rep], footprint_tau(op)[rep], tx, ty, T, W, H)
        reached = (rep[keep], tx[keep], ty[keep])
        n_tiles = np.bincount(rep[keep], minlength=x0.shape[0]).astype(np.int64)
    else:
        n_tiles = rect_tiles
    return dict(depth=Zc.astype(f32), x0=x0, y0=y0, x1=x1, y1=y1, n_tiles=n_tiles, radius=r, px=px, py=py,
                a=a, b=b, c=c, conic=(ca, cb, cc), visible=vis & (n_tiles > 0), TX=TX, TY=TY, reached=reached)


def tile_grid(cams, tile: int):
    """Per-view tile counts and offsets of the global tile index."""
    counts = [(-(-c.width // tile)) * (-(-c.height // tile)) for c in cams]
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def item_offsets(cams_scene, scene_offsets):
    """item index = item_offset[v] + (g - scene_offsets[s]) for the views' scenes."""
    sizes = [scene_offsets[s + 1] - scene_offsets[s] for s in cams_scene]
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def pair_lists(gs, cams, tile: int, view_scene=None, scene_offsets=None) -> dict:
    """All (tile, item) pairs of a batch of views, sorted by (global tile, depth bits, item).

    gs: dict/obj with float32 means, scales, quats ([3|4][N]); views reference scenes through
    ``view_scene`` (default: every view sees scene 0 = all Gaussians).
    """
    means, scales, quats, opacity = (np.asarray(getattr(gs, k) if hasattr(gs, k) else gs[k], dtype=f32)
                                     for k in ("means", "scales", "quats", "opacity"))
    N = means.shape[1]
    if view_scene is None:
        view_scene = [0] * len(cams)
        scene_offsets = np.array([0, N])
    toff = tile_grid(cams, tile)
    ioff = item_offsets(view_scene, scene_offsets)
    keys_t, keys_d, items, projs = [], [], [], []
    for v, cam in enumerate(cams):
        s0, s1 = scene_offsets[view_scene[v]], scene_offsets[view_scene[v] + 1]
        pr = project_fp32(means[:, s0:s1], scales[:, s0:s1], quats[:, s0:s1], cam, tile, opacity[s0:s1])
        projs.append(pr)
        rep, tx, ty = pr["reached"]
        if rep.size == 0:
            continue
        keys_t.append(toff[v] + ty * pr["TX"] + tx)
        keys_d.append(pr["depth"][rep].view(np.uint32).astype(np.int64))
        items.append(ioff[v] + rep)
    if keys_t:
        kt = np.concatenate(keys_t)
        kd = np.concatenate(keys_d)
        it = np.concatenate(items)
    else:
        kt = kd = it = np.zeros(0, dtype=np.int64)
    order = np.lexsort((it, kd, kt))
    kt, kd, it = kt[order], kd[order], it[order]
    n_tiles_total = int(toff[-1])
    starts = np.searchsorted(kt, np.arange(n_tiles_total), side="left")
    ends = np.searchsorted(kt, np.arange(n_tiles_total), side="right")
    return dict(tile=kt, depth_bits=kd, item=it, ranges=np.stack([starts, ends], 1), tile_offset=toff,
                item_offset=ioff, proj=projs)
