"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only *makes inputs*: scalar volumes, transfer-function control points,
orbit cameras and random Gaussian sets.  It holds none of the method's arithmetic
(no wavelet, bank, projection or compositing code), so the CPU oracle and the HIP
path can both consume its outputs without sharing method code.

Every generator is seeded with ``numpy.random.SeedSequence([config_index, stream])``
with the streams: 0 volume, 1 noise, 2 transfer function, 3 cameras, 4 FD subset,
5 random Gaussian sets, 6 visual-mode transfer functions.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

STREAM_VOLUME, STREAM_NOISE, STREAM_TF, STREAM_CAMERAS, STREAM_FD, STREAM_GAUSS, STREAM_MODES = range(7)


def rng(config_index: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(config_index), int(stream)]))


# ----------------------------------------------------------------------------- volumes

def _quat_to_rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def blob_volume(G: int, n_blobs: int, config_index: int, sigma_scale: float = 1.0) -> np.ndarray:
    """Sum of anisotropic 3D Gaussian blobs on a G^3 grid, float64 [z][y][x].

    Amplitudes U[0.2, 1], per-axis sigmas U[1.5, 5] voxels times ``sigma_scale``,
    rotations from a normalised N(0, I4) quaternion, centres U[0.2G, 0.8G].
    """
    r = rng(config_index, STREAM_VOLUME)
    vol = np.zeros((G, G, G), dtype=np.float64)
    for _ in range(n_blobs):
        amp = r.uniform(0.2, 1.0)
        sig = r.uniform(1.5, 5.0, size=3) * sigma_scale
        R = _quat_to_rot(r.normal(size=4))
        c = r.uniform(0.2 * G, 0.8 * G, size=3)            # (x, y, z) voxel-index coordinates
        prec = R @ np.diag(1.0 / sig ** 2) @ R.T
        ext = int(math.ceil(4.0 * sig.max()))
        lo = np.maximum(np.floor(c).astype(int) - ext, 0)
        hi = np.minimum(np.floor(c).astype(int) + ext + 1, G)
        xs = np.arange(lo[0], hi[0]) - c[0]
        ys = np.arange(lo[1], hi[1]) - c[1]
        zs = np.arange(lo[2], hi[2]) - c[2]
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        q = (prec[0, 0] * X * X + prec[1, 1] * Y * Y + prec[2, 2] * Z * Z
             + 2 * prec[0, 1] * X * Y + 2 * prec[0, 2] * X * Z + 2 * prec[1, 2] * Y * Z)
        vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += amp * np.exp(-0.5 * q)
    return vol


def spectral_noise(G: int, rgen: np.random.Generator, kmax: float, mode_exponent: float,
                   dtype=np.float64) -> np.ndarray:
    """Random-phase field with per-mode amplitude |k|^-mode_exponent for 1 <= |k| <= kmax.

    Shell-integrated spectrum E(k) ~ k^2 * |amp|^2, so E(k) ~ k^-2 needs mode_exponent = 2
    and E(k) ~ k^-5/3 needs mode_exponent = 11/6.  Returned with zero mean, unit std.
    """
    k1 = np.fft.fftfreq(G, d=1.0 / G).astype(dtype)
    k3 = np.fft.rfftfreq(G, d=1.0 / G).astype(dtype)
    kz = k1[:, None, None]
    ky = k1[None, :, None]
    kx = k3[None, None, :]
    kk = np.sqrt(kz * kz + ky * ky + kx * kx)
    with np.errstate(divide="ignore"):
        amp = np.where((kk >= 1.0) & (kk <= kmax), kk ** (-mode_exponent), 0.0).astype(dtype)
    del kk
    ctype = np.complex64 if dtype == np.float32 else np.complex128
    spec = (rgen.standard_normal(amp.shape, dtype=dtype)
            + 1j * rgen.standard_normal(amp.shape, dtype=dtype)).astype(ctype)
    spec *= amp
    del amp
    field = np.fft.irfftn(spec, s=(G, G, G))
    del spec
    field = field - field.mean()
    sd = field.std()
    return (field / sd).astype(dtype) if sd > 0 else field.astype(dtype)


def minmax(v: np.ndarray) -> np.ndarray:
    lo, hi = float(v.min()), float(v.max())
    return (v - lo) / (hi - lo) if hi > lo else np.zeros_like(v)


def volume_for_config(config_index: int) -> np.ndarray:
    """The scalar volume of a named workload, float32 [z][y][x], min-max normalised to [0, 1].

    0: 32^3, 8 blobs.   1: 128^3, 64 blobs + k^-2 noise (k <= 16, std 0.05).
    2: 256^3 blobs + noise.   3: 512^3 turbulence (E(k) ~ k^-5/3, 1 <= k <= 64).
    """
    if config_index == 0:
        v = blob_volume(32, 8, 0)
    elif config_index in (1, 2):
        G = 128 if config_index == 1 else 256
        v = blob_volume(G, 64, config_index, sigma_scale=G / 32)
        v = v + 0.05 * spectral_noise(G, rng(config_index, STREAM_NOISE), 16.0, 2.0)
    elif config_index == 3:
        v = spectral_noise(512, rng(3, STREAM_VOLUME), 64.0, 11.0 / 6.0, dtype=np.float32)
    else:
        raise ValueError(f"no volume recipe for config {config_index}")
    return minmax(v).astype(np.float32)


def scene_volume(config_index: int, scene: int, G: int) -> np.ndarray:
    """Uneven multi-scene batch volumes: blobs + k^-2 noise on a G^3 grid (seed per scene)."""
    ci = 100 * config_index + scene
    v = blob_volume(G, 64, ci, sigma_scale=G / 32)
    v = v + 0.05 * spectral_noise(G, rng(ci, STREAM_NOISE), 16.0, 2.0)
    return minmax(v).astype(np.float32)


# ----------------------------------------------------------------------------- transfer function

@dataclasses.dataclass
class TransferFunction:
    """Piecewise-linear 1D transfer function: ``xs`` ascending in [0, 1], ``rgba`` [n][4]."""
    xs: np.ndarray
    rgba: np.ndarray


def transfer_function(config_index: int, n_points: int = 6) -> TransferFunction:
    """6 seeded control points: x = [0, sorted U(0,1) x 4, 1]; RGB ~ U[0,1]; alpha ~ U[0,0.5], alpha(x0)=0."""
    r = rng(config_index, STREAM_TF)
    inner = np.sort(r.uniform(0.0, 1.0, size=n_points - 2))
    xs = np.concatenate([[0.0], inner, [1.0]]).astype(np.float32)
    rgb = r.uniform(0.0, 1.0, size=(n_points, 3))
    a = r.uniform(0.0, 0.5, size=n_points)
    a[0] = 0.0
    rgba = np.concatenate([rgb, a[:, None]], axis=1).astype(np.float32)
    return TransferFunction(xs=xs, rgba=rgba)


def mode_intervals(vol: np.ndarray, n_modes: int = 5, q_lo: float = 0.5) -> np.ndarray:
    """Value intervals of the visual modes: edges at n_modes + 1 equally spaced quantiles of the
    volume's values from q_lo to 1, so each mode covers the same number of voxels of the upper
    part of the value distribution.  float32 [n_modes + 1], strictly increasing."""
    e = np.quantile(np.asarray(vol, np.float64).reshape(-1), np.linspace(q_lo, 1.0, n_modes + 1))
    e = e.astype(np.float32)
    if not np.all(np.diff(e) > 0):
        raise ValueError("mode intervals collapse: the volume has too few distinct values")
    return e


def mode_transfer_functions(vol: np.ndarray, config_index: int, n_modes: int = 5,
                            q_lo: float = 0.5) -> list:
    """One transfer function per visual mode, each zero outside its own value interval [a, b].

    Four control points per mode: (a, 0), two seeded interior points at a + (b - a) u with sorted
    u ~ U(0.15, 0.85), RGB ~ U(0.2, 1), alpha ~ U(0.1, 0.5), and (b, 0); the map is constant (zero)
    beyond the end points.
    """
    edges = mode_intervals(vol, n_modes, q_lo)
    r = rng(config_index, STREAM_MODES)
    out = []
    for h in range(n_modes):
        a, b = float(edges[h]), float(edges[h + 1])
        u = np.sort(r.uniform(0.15, 0.85, size=2))
        xs = np.array([a, a + (b - a) * u[0], a + (b - a) * u[1], b], dtype=np.float32)
        rgba = np.zeros((4, 4), dtype=np.float32)
        rgba[1:3, :3] = r.uniform(0.2, 1.0, size=(2, 3))
        rgba[1:3, 3] = r.uniform(0.1, 0.5, size=2)
        if not np.all(np.diff(xs) > 0):
            raise ValueError("mode interval too narrow for float32 control points")
        out.append(TransferFunction(xs=xs, rgba=rgba))
    return out


def union_transfer_function(tfs: list) -> TransferFunction:
    """The sum of transfer functions with disjoint supports, each zero at its end points: the control
    points of all of them in order, a shared end point (zero in both) taken once."""
    xs, rgba = [], []
    for tf in sorted(tfs, key=lambda t: float(t.xs[0])):
        if float(tf.rgba[0].max()) != 0.0 or float(tf.rgba[-1].max()) != 0.0:
            raise ValueError("a mode transfer function must be zero at its end points")
        for x, c in zip(tf.xs, tf.rgba):
            if xs and float(x) < xs[-1]:
                raise ValueError("mode transfer functions overlap")
            if xs and float(x) == xs[-1]:
                continue                     # shared end point, zero on both sides
            xs.append(float(x))
            rgba.append(np.asarray(c, np.float32))
    return TransferFunction(xs=np.array(xs, np.float32), rgba=np.array(rgba, np.float32))


# ----------------------------------------------------------------------------- cameras

@dataclasses.dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    ``viewmat`` is the world->camera [R | t] matrix, 3x4 row-major; pixel (i, j) samples the
    image plane at (i + 0.5, j + 0.5).
    """
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    near: float
    viewmat: np.ndarray  # float32 [3][4]
    bg: tuple = (0.0, 0.0, 0.0)


def look_at(eye: np.ndarray, target=np.zeros(3), up=np.array([0.0, 0.0, 1.0])) -> np.ndarray:
    f = target - eye
    f = f / np.linalg.norm(f)
    right = np.cross(f, up)
    right = right / np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f])
    t = -R @ eye
    return np.concatenate([R, t[:, None]], axis=1)


def orbit_cameras(n_views: int, width: int, height: int, distance: float = 3.5,
                  elevation_deg: float = 20.0, fov_y_deg: float = 45.0, near: float = 0.2,
                  azimuth0: float = 0.0) -> list:
    """View v of V at azimuth 2*pi*v/V, fixed elevation and distance, looking at the origin, +z up."""
    f = height / (2.0 * math.tan(math.radians(fov_y_deg) / 2.0))
    el = math.radians(elevation_deg)
    cams = []
    for v in range(n_views):
        az = azimuth0 + 2.0 * math.pi * v / n_views
        eye = distance * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
        cams.append(Camera(width=width, height=height, fx=f, fy=f, cx=width / 2.0, cy=height / 2.0,
                           near=near, viewmat=look_at(eye).astype(np.float32)))
    return cams


# ----------------------------------------------------------------------------- random Gaussian sets

@dataclasses.dataclass
class GaussianSet:
    """Activated 3DGS parameters, float32 SoA: means [3][N], scales [3][N] (>0),
    quats [4][N] (w, x, y, z; unnormalised), opacity [N] in (0, 1), rgb [3][N]."""
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacity: np.ndarray
    rgb: np.ndarray

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    def subset(self, idx) -> "GaussianSet":
        return GaussianSet(self.means[:, idx].copy(), self.scales[:, idx].copy(), self.quats[:, idx].copy(),
                           self.opacity[idx].copy(), self.rgb[:, idx].copy())

    @staticmethod
    def concat(sets) -> "GaussianSet":
        return GaussianSet(np.concatenate([s.means for s in sets], 1), np.concatenate([s.scales for s in sets], 1),
                           np.concatenate([s.quats for s in sets], 1), np.concatenate([s.opacity for s in sets]),
                           np.concatenate([s.rgb for s in sets], 1))


def random_gaussians(n: int, seed: int, extent: float = 0.8, log_scale_mean: float = -3.5,
                     log_scale_std: float = 0.5, opacity_range=(0.05, 0.95)) -> GaussianSet:
    """A seeded random Gaussian set inside [-extent, extent]^3 (for render-only tests)."""
    r = rng(seed, STREAM_GAUSS)
    means = r.uniform(-extent, extent, size=(3, n))
    scales = np.exp(r.normal(log_scale_mean, log_scale_std, size=(3, n)))
    quats = r.normal(size=(4, n))
    opacity = r.uniform(opacity_range[0], opacity_range[1], size=n)
    rgb = r.uniform(0.0, 1.0, size=(3, n))
    f32 = np.float32
    return GaussianSet(means.astype(f32), scales.astype(f32), quats.astype(f32), opacity.astype(f32),
                       rgb.astype(f32))


# ----------------------------------------------------------------------------- named workloads

@dataclasses.dataclass
class Workload:
    name: str
    G: int
    J: int
    wavelet: str          # "haar" | "bior4.4"
    K: int
    n_views: int
    width: int
    height: int
    tile: int
    loss: str             # "l1" | "l1_dssim"


WORKLOADS = {
    "c0": Workload("c0: 32^3, Haar J=1, K=2048, 1x64^2", 32, 1, "haar", 2048, 1, 64, 64, 16, "l1"),
    "c1": Workload("c1: 128^3, Haar J=3, K=100000, 16x800^2", 128, 3, "haar", 100_000, 16, 800, 800, 16, "l1"),
    "c2": Workload("c2: 256^3, bior4.4 J=4, K=500000, 8x1024^2", 256, 4, "bior4.4", 500_000, 8, 1024, 1024, 16,
                   "l1_dssim"),
    "H": Workload("H: 512^3 turbulence, bior4.4 J=5, K=1000000, 8x1920x1080", 512, 5, "bior4.4", 1_000_000, 8,
                  1920, 1080, 16, "l1_dssim"),
}
