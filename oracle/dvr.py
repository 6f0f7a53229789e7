"""Ray-marching direct volume renderer for the supervision images (Sec. 4.4).  Test infrastructure.

The paper renders its targets with a production DVR tool it does not describe further.  The
reading used here: one ray per pixel centre, clipped to the volume box [-1, 1]^3; samples every
half voxel from the entry point; trilinear interpolation of the scalar field (voxel centres at
-1 + h (i + 1/2), clamped at the border), then the transfer function (post-classification); opacity
corrected to the step length, alpha_s = 1 - (1 - alpha)^(step / voxel); front-to-back compositing,
stopping once T < 1e-4; black background.
"""
from __future__ import annotations

import numpy as np

from . import tf as _tf


def ray_dirs(cam):
    V = np.asarray(cam.viewmat, dtype=np.float64)
    R, t = V[:, :3], V[:, 3]
    eye = -R.T @ t
    xs = (np.arange(cam.width) + 0.5 - cam.cx) / cam.fx
    ys = (np.arange(cam.height) + 0.5 - cam.cy) / cam.fy
    Y, X = np.meshgrid(ys, xs, indexing="ij")
    d_cam = np.stack([X, Y, np.ones_like(X)], -1)
    d = d_cam @ R                     # = R^T d_cam per pixel
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return eye, d


def trilinear(vol: np.ndarray, p: np.ndarray) -> np.ndarray:
    """vol [z][y][x]; p [..., 3] world (x, y, z) -> interpolated values."""
    G = vol.shape[0]
    h = 2.0 / G
    u = (p + 1.0) / h - 0.5
    u = np.clip(u, 0.0, G - 1.0)
    i0 = np.minimum(np.floor(u).astype(np.int64), G - 2)
    f = u - i0
    x0, y0, z0 = i0[..., 0], i0[..., 1], i0[..., 2]
    fx, fy, fz = f[..., 0], f[..., 1], f[..., 2]
    out = 0.0
    for dz in (0, 1):
        wz = fz if dz else 1 - fz
        for dy in (0, 1):
            wy = fy if dy else 1 - fy
            for dx in (0, 1):
                wx = fx if dx else 1 - fx
                out = out + wz * wy * wx * vol[z0 + dz, y0 + dy, x0 + dx]
    return out


def render(vol: np.ndarray, xs, rgba, cam, step_vox: float = 0.5, t_min: float = 1e-4, pixels=None,
           flag_rel: float | None = None):
    """Image [3][H][W] and transmittance [H][W]; with ``pixels`` = (px, py) index arrays only those
    rays are marched and the results are [3][n] and [n].  With ``flag_rel`` a third result marks the
    rays on which some sample left T within flag_rel * t_min of the stop threshold t_min, where a
    renderer with other rounding may legitimately stop one sample earlier or later."""
    vol = np.asarray(vol, dtype=np.float64)
    G = vol.shape[0]
    h = 2.0 / G
    dt = step_vox * h
    eye, d = ray_dirs(cam)
    if pixels is not None:
        d = d[np.asarray(pixels[1]), np.asarray(pixels[0])][None]      # [1][n][3]
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t1 = (-1.0 - eye) * inv
        t2 = (1.0 - eye) * inv
    tn = np.max(np.minimum(t1, t2), -1)
    tf = np.min(np.maximum(t1, t2), -1)
    tn = np.maximum(tn, 0.0)
    hit = tf > tn
    H, W = d.shape[0], d.shape[1]
    C = np.zeros((H, W, 3))
    T = np.ones((H, W))
    near = np.zeros((H, W), dtype=bool)
    span = np.where(hit, tf - tn, 0.0)          # rays that miss the cube have non-finite spans
    nsteps = np.where(hit, np.floor(span / dt).astype(np.int64) + 1, 0)
    for k in range(int(nsteps.max()) if nsteps.size else 0):
        act = (k < nsteps) & (T >= t_min)
        if not act.any():
            break
        tk = tn + k * dt
        p = eye[None, None, :] + tk[..., None] * d
        val = trilinear(vol, p[act])
        c = _tf.apply(val, xs, rgba)              # [4][n]
        a = 1.0 - (1.0 - c[3]) ** step_vox
        Ta = T[act]
        C[act] += (Ta * a)[:, None] * c[:3].T
        T[act] = Ta * (1.0 - a)
        if flag_rel is not None:
            near[act] |= np.abs(T[act] - t_min) <= flag_rel * t_min
    out = (C[0].T, T[0], near[0]) if pixels is not None else (C.transpose(2, 0, 1), T, near)
    return out if flag_rel is not None else out[:2]
