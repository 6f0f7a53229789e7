"""Visual modes (Sec. 4.4): each transfer function TF_h is zero outside its own value interval of
the field.  Pins of the mode inputs and of what the oracle computes from them: the union of the
modes is their sum, the oracle's DWT (a linear map) of the union is the sum of the per-mode
DWTs, and a mode whose interval holds none of the field's values renders nothing."""
import os
import re

import numpy as np

import vbm_inputs as vi
from oracle import dvr, dwt, tf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tf_max_points() -> int:
    with open(os.path.join(ROOT, "include", "vbm.h")) as f:
        return int(re.search(r"#define VBM_TF_MAX_POINTS (\d+)", f.read()).group(1))


def _modes(config=0, n=5):
    vol = vi.volume_for_config(config)
    return vol, vi.mode_transfer_functions(vol, config, n)


def test_each_mode_vanishes_outside_its_interval():
    vol, tfs = _modes()
    edges = vi.mode_intervals(vol)
    x = np.unique(np.concatenate([np.linspace(0.0, 1.0, 20001), edges.astype(np.float64)]))
    for h, t in enumerate(tfs):
        a, b = float(edges[h]), float(edges[h + 1])
        assert t.xs[0] == edges[h] and t.xs[-1] == edges[h + 1]
        c = tf.apply(x, t.xs, t.rgba)
        outside = (x <= a) | (x >= b)
        assert np.all(c[:, outside] == 0.0), h
        assert np.all(c[3, ~outside] > 0.0), h          # alpha positive on the open interval
        assert np.all(c >= 0.0)


def test_intervals_hold_equal_voxel_counts():
    vol, _ = _modes(n=5)
    e = vi.mode_intervals(vol, 5, 0.5)
    v = vol.reshape(-1)
    counts = np.array([np.count_nonzero((v >= e[h]) & (v < e[h + 1])) for h in range(5)])
    counts[-1] += np.count_nonzero(v == e[-1])
    assert counts.sum() == np.count_nonzero(v >= e[0])
    assert counts.max() - counts.min() <= 2 + 1e-3 * v.size, counts
    assert abs(counts.sum() - 0.5 * v.size) <= 2 + 1e-3 * v.size


def test_union_is_the_sum_of_the_modes():
    for config in (0, 1):
        vol, tfs = _modes(config)
        u = vi.union_transfer_function(tfs)
        assert 2 <= len(u.xs) <= _tf_max_points()
        assert np.all(np.diff(u.xs) > 0)
        x = np.linspace(-0.1, 1.1, 40001)
        total = sum(tf.apply(x, t.xs, t.rgba) for t in tfs)
        assert np.abs(tf.apply(x, u.xs, u.rgba) - total).max() <= 1e-12


def test_dwt_of_the_union_is_the_sum_of_mode_dwts():
    vol, tfs = _modes()
    u = vi.union_transfer_function(tfs)
    for J, wav in ((1, "haar"), (2, "bior4.4")):
        whole = dwt.dwt3d_rgba(tf.apply(vol, u.xs, u.rgba), J, wav)
        parts = sum(dwt.dwt3d_rgba(tf.apply(vol, t.xs, t.rgba), J, wav) for t in tfs)
        assert np.abs(whole - parts).max() <= 1e-12 * np.abs(whole).max()


def test_mode_outside_the_fields_values_renders_nothing():
    """A volume whose values all lie below the first interval: every mode is transparent there,
    so the DVR leaves colour 0 and transmittance 1; moved into one interval, that mode alone
    renders as the union does."""
    vol, tfs = _modes()
    edges = vi.mode_intervals(vol)
    cam = vi.orbit_cameras(1, 12, 10, distance=3.0)[0]
    rng = np.random.default_rng(3)
    low = (float(edges[0]) * rng.uniform(0.0, 0.99, size=(8, 8, 8))).astype(np.float32)
    for t in tfs:
        img, T = dvr.render(low, t.xs, t.rgba, cam)
        assert np.all(img == 0.0) and np.all(T == 1.0)
    h = 3
    a, b = float(edges[h]), float(edges[h + 1])
    inside = (a + (b - a) * rng.uniform(0.05, 0.95, size=(8, 8, 8))).astype(np.float32)
    u = vi.union_transfer_function(tfs)
    img_h, T_h = dvr.render(inside, tfs[h].xs, tfs[h].rgba, cam)
    img_u, T_u = dvr.render(inside, u.xs, u.rgba, cam)
    assert np.abs(img_h - img_u).max() <= 1e-12 and np.abs(T_h - T_u).max() <= 1e-12
    assert img_h.max() > 0.0 and T_h.min() < 1.0
