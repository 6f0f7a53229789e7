"""Pins of the oracle's geometry against definitions it does not share code with.

The rasteriser is cited, not specified, by the paper (Sec. 3, 3D Gaussian Splatting; Sec. 4.4), so
its EWA projection is pinned to what EWA splatting defines: the 2D covariance is the 3D covariance
pushed through the Jacobian of the pinhole map, here taken by finite differences of that map (and,
independently, estimated by Monte Carlo sampling of the projected points), with the Jacobian
evaluated at the point pulled back into 1.3x the field of view.  The rotation of a quaternion is
pinned to scipy's.  The supervision renderer's trilinear lookup is pinned to the exactness of
trilinear interpolation on affine fields and at voxel centres, and its rays to the rasteriser's
projection of the points they pass through.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import vbm_inputs as vi
from oracle import binning, dvr, render


def _rand_quats(n, seed):
    q = np.random.default_rng(seed).normal(size=(4, n)) * np.random.default_rng(seed + 1).uniform(0.2, 3.0, n)
    return q


def _scipy_rot(q):
    """q [4][N] (w, x, y, z), any norm -> [N][3][3] from scipy (scalar-last convention)."""
    return Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], 1)).as_matrix()


def test_quat_to_rot_matches_scipy():
    q = _rand_quats(300, 11)
    ref = _scipy_rot(q)
    got = render.quat_to_rot(torch.as_tensor(q)).numpy()
    assert np.abs(got - ref).max() <= 1e-13
    q32 = q.astype(np.float32)
    R32 = np.array(binning._rot_f32(q32[0], q32[1], q32[2], q32[3]), dtype=np.float64)   # [3][3][N]
    ref32 = _scipy_rot(q32.astype(np.float64))
    assert np.abs(R32.transpose(2, 0, 1) - ref32).max() <= 2e-6


def _pinhole(cam, Xc):
    """The pinhole map of camera coordinates [..., 3] to pixel coordinates [..., 2] (OpenCV axes)."""
    return np.stack([cam.fx * Xc[..., 0] / Xc[..., 2] + cam.cx, cam.fy * Xc[..., 1] / Xc[..., 2] + cam.cy], -1)


def _pinhole_jacobian_fd(cam, Xc):
    """2x3 Jacobian of the pinhole map at camera point Xc by FP64 central differences."""
    J = np.zeros((2, 3))
    for k in range(3):
        h = 1e-5 * max(1.0, abs(Xc[k]))
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (_pinhole(cam, Xc + e) - _pinhole(cam, Xc - e)) / (2 * h)
    return J


def _expected_sigma2(cam, mean, scale, quat):
    """EWA 2D covariance: Jacobian (finite differences) at the FOV-clamped camera point, 3D covariance
    from scipy's rotation, plus the 0.3 px dilation."""
    V = np.asarray(cam.viewmat, dtype=np.float64)
    Rv, tv = V[:, :3], V[:, 3]
    Xc = Rv @ mean + tv
    limx = 1.3 * (0.5 * cam.width / cam.fx)
    limy = 1.3 * (0.5 * cam.height / cam.fy)
    Xcl = np.array([Xc[2] * np.clip(Xc[0] / Xc[2], -limx, limx), Xc[2] * np.clip(Xc[1] / Xc[2], -limy, limy), Xc[2]])
    J = _pinhole_jacobian_fd(cam, Xcl)
    R = _scipy_rot(quat[:, None])[0]
    S3 = R @ np.diag(scale ** 2) @ R.T
    S2 = J @ Rv @ S3 @ Rv.T @ J.T
    return S2 + 0.3 * np.eye(2), _pinhole(cam, Xc)


def _camera():
    return vi.orbit_cameras(5, 160, 96, azimuth0=0.3)[2]


def _points_at_ratios(cam, rx, ry, depth, seed):
    """World points whose camera coordinates have X/Z = rx, Y/Z = ry at the given depths."""
    V = np.asarray(cam.viewmat, dtype=np.float64)
    Rv, tv = V[:, :3], V[:, 3]
    Xc = np.stack([rx * depth, ry * depth, depth], 0)
    return Rv.T @ (Xc - tv[:, None])


def _gaussian_batch(cam, rx, ry, seed):
    n = rx.size
    r = np.random.default_rng(seed)
    depth = r.uniform(2.0, 5.0, n)
    means = _points_at_ratios(cam, rx, ry, depth, seed)
    scales = np.exp(r.normal(-3.0, 0.6, (3, n)))
    quats = _rand_quats(n, seed + 7)
    return means, scales, quats


def _check_projection(cam, means, scales, quats, rtol64=1e-8, rtol32=2e-4):
    m2d, conic, _ = render.project_fp64(torch.as_tensor(means), torch.as_tensor(scales), torch.as_tensor(quats), cam)
    m2d, conic = m2d.numpy(), conic.numpy()
    f32 = np.float32
    pr = binning.project_fp32(means.astype(f32), scales.astype(f32), quats.astype(f32), cam, 16)
    for i in range(means.shape[1]):
        S2, px = _expected_sigma2(cam, means[:, i], scales[:, i], quats[:, i])
        A, B, C = conic[i]
        inv = np.linalg.inv(np.array([[A, B], [B, C]]))
        scale = np.abs(S2).max()
        assert np.abs(inv - S2).max() <= rtol64 * scale, (i, inv, S2)
        assert np.abs(m2d[i] - px).max() <= 1e-9 * max(1.0, np.abs(px).max())
        got32 = np.array([[pr["a"][i], pr["b"][i]], [pr["b"][i], pr["c"][i]]], dtype=np.float64)
        assert np.abs(got32 - S2).max() <= rtol32 * scale, (i, got32, S2)
        assert abs(pr["px"][i] - px[0]) <= 1e-3 and abs(pr["py"][i] - px[1]) <= 1e-3


def test_projected_covariance_off_axis_matches_pinhole_jacobian():
    """Inside the clamp, off the optical axis in both directions: the EWA covariance equals
    J(X) W Sigma3 W^T J(X)^T + 0.3 I with J the finite-difference Jacobian of the pinhole map."""
    cam = _camera()
    limx = 1.3 * (0.5 * cam.width / cam.fx)
    limy = 1.3 * (0.5 * cam.height / cam.fy)
    r = np.random.default_rng(3)
    rx = r.uniform(-0.95, 0.95, 60) * limx
    ry = r.uniform(-0.95, 0.95, 60) * limy
    # also points just inside the clamp that a clamp at (W/2)/fx instead of 1.3 (W/2)/fx would change
    rx = np.concatenate([rx, [1.2 * 0.5 * cam.width / cam.fx, -1.25 * 0.5 * cam.width / cam.fx, 0.1]])
    ry = np.concatenate([ry, [-0.2, 0.3, 1.2 * 0.5 * cam.height / cam.fy]])
    means, scales, quats = _gaussian_batch(cam, rx, ry, 5)
    _check_projection(cam, means, scales, quats)


def test_projected_covariance_field_of_view_clamp():
    """Outside 1.3x the half field of view the Jacobian is that of the pinhole map at the point pulled
    back onto the clamp (same depth); the projected centre itself is not clamped."""
    cam = _camera()
    hx = 0.5 * cam.width / cam.fx
    hy = 0.5 * cam.height / cam.fy
    rx = np.array([1.35, -1.4, 2.0, -3.0, 0.5, -0.2, 1.8, 1.31]) * hx
    ry = np.array([0.1, -0.4, 0.2, 0.0, 1.5, -2.5, -1.9, 1.33]) * hy
    means, scales, quats = _gaussian_batch(cam, rx, ry, 9)
    _check_projection(cam, means, scales, quats)


def test_projected_covariance_monte_carlo():
    """A small Gaussian's projected sample covariance (world samples through the exact pinhole map)
    matches Sigma2 - 0.3 I, a check that needs no Jacobian at all."""
    cam = _camera()
    limx = 1.3 * (0.5 * cam.width / cam.fx)
    limy = 1.3 * (0.5 * cam.height / cam.fy)
    rx = np.array([0.7, -0.6, 0.3]) * limx
    ry = np.array([-0.5, 0.6, 0.8]) * limy
    means, scales, quats = _gaussian_batch(cam, rx, ry, 21)
    scales = scales * 0.2 / scales.max(0, keepdims=True)        # largest axis 0.2: ~5 px on screen
    scales[:, 1] *= np.array([1.0, 0.3, 0.1])
    m2d, conic, _ = render.project_fp64(torch.as_tensor(means), torch.as_tensor(scales), torch.as_tensor(quats), cam)
    V = np.asarray(cam.viewmat, dtype=np.float64)
    rng = np.random.default_rng(17)
    for i in range(means.shape[1]):
        R = _scipy_rot(quats[:, i:i + 1])[0]
        L = R @ np.diag(scales[:, i])
        scale_lin = 0.02 / scales[:, i].max()            # shrink so the linearisation error is tiny
        n = 400_000
        X = means[:, i][None, :] + (rng.normal(size=(n, 3)) @ L.T) * scale_lin
        Xc = X @ V[:, :3].T + V[:, 3]
        uv = _pinhole(cam, Xc)
        emp = np.cov(uv.T) / scale_lin ** 2
        A, B, C = conic[i].numpy()
        S2 = np.linalg.inv(np.array([[A, B], [B, C]])) - 0.3 * np.eye(2)
        assert np.abs(emp - S2).max() <= 0.02 * np.abs(S2).max(), (i, emp, S2)


def test_fp32_spec_projection_agrees_with_fp64_off_axis():
    """The float32 binning spec and the FP64 projection agree on an orbit scene whose Gaussians fill
    the view (most far off the optical axis, some beyond the clamp)."""
    gs = vi.random_gaussians(3000, 31, extent=1.6, log_scale_mean=-3.0)
    cam = vi.orbit_cameras(3, 200, 120)[1]
    m2d, conic, depth = render.project_fp64(torch.as_tensor(gs.means, dtype=torch.float64),
                                            torch.as_tensor(gs.scales, dtype=torch.float64),
                                            torch.as_tensor(gs.quats, dtype=torch.float64), cam)
    pr = binning.project_fp32(gs.means, gs.scales, gs.quats, cam, 16)
    ok = depth.numpy() > 0.5
    m2d, conic = m2d.numpy()[ok], conic.numpy()[ok]
    assert np.abs(pr["px"][ok] - m2d[:, 0]).max() <= 2e-3
    assert np.abs(pr["py"][ok] - m2d[:, 1]).max() <= 2e-3
    c32 = np.stack([pr["conic"][0], pr["conic"][1], pr["conic"][2]], 1)[ok].astype(np.float64)
    den = np.abs(conic).max(1, keepdims=True)
    assert (np.abs(c32 - conic) / den).max() <= 1e-3


# ----------------------------------------------------------------------------- DVR

def _affine_volume(G, coef):
    """Voxel (i, j, k) = coef . (1, x_c, y_c, z_c) at its centre (-1 + h (i + 1/2), ...)."""
    h = 2.0 / G
    c = -1.0 + h * (np.arange(G) + 0.5)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return coef[0] + coef[1] * x + coef[2] * y + coef[3] * z


def test_trilinear_exact_on_affine_fields():
    G = 12
    coef = np.array([0.3, 0.7, -1.1, 0.45])
    vol = _affine_volume(G, coef)
    h = 2.0 / G
    lo, hi = -1.0 + 0.5 * h, 1.0 - 0.5 * h              # the hull of the voxel centres
    p = np.random.default_rng(2).uniform(lo, hi, (500, 3))
    got = dvr.trilinear(vol, p)
    want = coef[0] + p @ coef[1:]
    assert np.abs(got - want).max() <= 1e-12
    # beyond the centre hull (inside the box) the lookup holds the border value: the clamped point's
    q = np.random.default_rng(3).uniform(-1.0, 1.0, (500, 3))
    want_q = coef[0] + np.clip(q, lo, hi) @ coef[1:]
    assert np.abs(dvr.trilinear(vol, q) - want_q).max() <= 1e-12


def test_trilinear_returns_voxel_values_at_centres():
    G = 9
    vol = np.random.default_rng(4).uniform(size=(G, G, G))
    h = 2.0 / G
    idx = np.random.default_rng(5).integers(0, G, (400, 3))          # (x, y, z) voxel indices
    p = -1.0 + h * (idx + 0.5)
    got = dvr.trilinear(vol, p)
    assert np.abs(got - vol[idx[:, 2], idx[:, 1], idx[:, 0]]).max() <= 1e-13
    # midway between two voxel centres along one axis: the mean of the two
    p2 = p.copy()
    sel = idx[:, 0] < G - 1
    p2[sel, 0] += 0.5 * h
    mid = 0.5 * (vol[idx[sel, 2], idx[sel, 1], idx[sel, 0]] + vol[idx[sel, 2], idx[sel, 1], idx[sel, 0] + 1])
    assert np.abs(dvr.trilinear(vol, p2[sel]) - mid).max() <= 1e-13


def test_dvr_ray_passes_through_the_rasterised_point():
    """The supervision ray of pixel (i, j) runs through exactly the world points that the rasteriser
    projects to that pixel's sample position (i + 0.5, j + 0.5)."""
    cams = []
    for k, eye in enumerate(([3.1, 0.7, 1.2], [-0.4, -2.9, 1.6], [0.3, 2.2, -2.4])):
        f = 70.0 + 9.0 * k
        cams.append(vi.Camera(width=90, height=70, fx=f, fy=f * 1.05, cx=44.0 + k, cy=35.5 - k, near=0.2,
                              viewmat=vi.look_at(np.array(eye))))          # float64: an orthonormal rotation
    for cam in cams:
        eye, d = dvr.ray_dirs(cam)
        r = np.random.default_rng(int(cam.width))
        ii = r.integers(0, cam.width, 40)
        jj = r.integers(0, cam.height, 40)
        t = r.uniform(1.5, 5.0, 40)
        pts = eye[None, :] + t[:, None] * d[jj, ii]
        m2d, _, depth = render.project_fp64(torch.as_tensor(pts.T), torch.full((3, 40), 0.01, dtype=torch.float64),
                                            torch.tensor([[1.0], [0.0], [0.0], [0.0]], dtype=torch.float64).expand(4, 40),
                                            cam)
        m2d = m2d.numpy()
        assert np.abs(m2d[:, 0] - (ii + 0.5)).max() <= 1e-9
        assert np.abs(m2d[:, 1] - (jj + 0.5)).max() <= 1e-9
        assert np.all(depth.numpy() > 0)


def test_dvr_samples_a_slab_at_half_voxel_steps():
    """A ray along +x through a volume that is opaque-coloured only in the slab x in [a, b] composites
    exactly the samples taken every half voxel from the box entry that fall inside the slab."""
    G = 16
    h = 2.0 / G
    c = -1.0 + h * (np.arange(G) + 0.5)
    vol = np.zeros((G, G, G))
    vol[:, :, 5:9] = 1.0                          # voxels 5..8 along x
    cam = vi.Camera(width=1, height=1, fx=1.0, fy=1.0, cx=0.5, cy=0.5, near=0.01,
                    viewmat=vi.look_at(np.array([-3.0, 0.0, 0.0]), target=np.array([0.0, 0.0, 0.0]),
                                       up=np.array([0.0, 0.0, 1.0])).astype(np.float64))
    xs = np.array([0.0, 1.0])
    rgba = np.array([[0.0, 0.0, 0.0, 0.0], [0.2, 0.6, 1.0, 0.3]])
    C, T = dvr.render(vol, xs, rgba, cam)
    # samples at x = -1 + k h/2; value by linear interpolation between centres (y, z on centre planes)
    xk = -1.0 + np.arange(4 * G + 1) * 0.5 * h
    xk = xk[xk <= 1.0 + 1e-12]
    prof = np.interp(xk, c, ((np.arange(G) >= 5) & (np.arange(G) <= 8)).astype(np.float64))
    Tr, Cr = 1.0, np.zeros(3)
    for v in prof:
        a = 1.0 - (1.0 - 0.3 * v) ** 0.5
        Cr += Tr * a * np.array([0.2, 0.6, 1.0]) * v
        Tr *= 1.0 - a
    assert abs(T[0, 0] - Tr) <= 1e-12
    assert np.abs(C[:, 0, 0] - Cr).max() <= 1e-12
