"""Pins of the oracle loss, optimiser and volume renderer."""
import math

import numpy as np
import torch

import vbm_inputs as vi
from oracle import adam, dvr, loss, tf


def test_ssim_identity_and_bruteforce():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(3, 20, 17))
    y = np.clip(x + 0.1 * rng.normal(size=x.shape), 0, 1)
    m = loss.ssim_map(torch.as_tensor(x), torch.as_tensor(x)).numpy()
    assert np.abs(m - 1).max() <= 1e-12
    m = loss.ssim_map(torch.as_tensor(x), torch.as_tensor(y)).numpy()
    for (c, i, j) in [(0, 0, 0), (1, 10, 8), (2, 19, 16), (0, 5, 16)]:
        assert abs(m[c, i, j] - loss.ssim_pixel_bruteforce(x, y, c, i, j)) <= 1e-12


def test_l1_gradient_is_sign_over_count():
    rng = np.random.default_rng(1)
    x = [rng.uniform(size=(3, 4, 5)), rng.uniform(size=(3, 6, 2))]
    y = [a.copy() for a in x]
    y[0][0, 0, 0] += 0.5
    y[1][2, 1, 1] -= 0.25
    val, g = loss.loss_and_grad(x, y, "l1")
    count = 60 + 36
    assert abs(val - 0.75 / count) <= 1e-15
    assert g[0][0, 0, 0] == -1.0 / count and g[1][2, 1, 1] == 1.0 / count
    assert np.count_nonzero(g[0]) == 1 and np.count_nonzero(g[1]) == 1


def test_dssim_gradient_central_differences():
    rng = np.random.default_rng(2)
    x = [rng.uniform(size=(3, 14, 13))]
    y = [np.clip(x[0] + 0.2 * rng.normal(size=x[0].shape), 0, 1)]
    val, g = loss.loss_and_grad(x, y, "l1_dssim")
    for (c, i, j) in [(0, 3, 4), (1, 0, 12), (2, 13, 6), (0, 7, 7)]:
        h = 1e-6
        xp = [x[0].copy()]
        xp[0][c, i, j] += h
        xm = [x[0].copy()]
        xm[0][c, i, j] -= h
        fd = (loss.loss_and_grad(xp, y, "l1_dssim")[0] - loss.loss_and_grad(xm, y, "l1_dssim")[0]) / (2 * h)
        assert abs(fd - g[0][c, i, j]) <= 1e-7


def test_adam_matches_torch_and_first_step_sign():
    rng = np.random.default_rng(3)
    raw = {k: rng.normal(size=(3, 5)) for k in adam.GROUPS}
    m = {k: np.zeros_like(v) for k, v in raw.items()}
    v = {k: np.zeros_like(v) for k, v in raw.items()}
    params = {k: torch.tensor(raw[k], requires_grad=True) for k in adam.GROUPS}
    opt = torch.optim.Adam([{"params": [params[k]], "lr": adam.DEFAULT_LR[k]} for k in adam.GROUPS],
                           betas=(0.9, 0.999), eps=1e-15)
    for t in range(1, 4):
        g = {k: rng.normal(size=(3, 5)) for k in adam.GROUPS}
        new_raw, m, v = adam.step(raw, g, m, v, t)
        if t == 1:
            for k in adam.GROUPS:
                assert np.allclose(new_raw[k] - raw[k], -adam.DEFAULT_LR[k] * np.sign(g[k]), atol=1e-12)
        raw = new_raw
        for k in adam.GROUPS:
            params[k].grad = torch.tensor(g[k])
        opt.step()
        for k in adam.GROUPS:
            assert np.abs(params[k].detach().numpy() - raw[k]).max() <= 1e-12


def test_chain_grads_through_activations():
    raw = dict(log_scales=np.array([[0.1, -2.0]]), logit_opacity=np.array([0.3, -1.0]))
    act = dict(means=0, quats=0, rgb=0, scales=np.array([[2.0, 3.0]]), opacity=np.array([1.0, 2.0]))
    g = adam.chain_grads(act, raw)
    assert np.allclose(g["log_scales"], act["scales"] * np.exp(raw["log_scales"]))
    sig = 1 / (1 + np.exp(-raw["logit_opacity"]))
    assert np.allclose(g["logit_opacity"], act["opacity"] * sig * (1 - sig))


def test_tf_exact_at_control_points_and_linear_between():
    t = vi.transfer_function(0)
    vals = tf.apply(t.xs, t.xs, t.rgba)
    assert np.allclose(vals.T, t.rgba.astype(np.float64), atol=1e-7)
    mid = 0.5 * (t.xs[1:] + t.xs[:-1])
    vm = tf.apply(mid, t.xs, t.rgba)
    assert np.allclose(vm.T, 0.5 * (t.rgba[1:].astype(np.float64) + t.rgba[:-1]), atol=1e-6)


def test_dvr_constant_medium():
    """A constant medium over a path of n half-voxel samples leaves T = (1 - a)^(n/2) and colour c (1 - T)."""
    G = 32
    vol = np.full((G, G, G), 0.5)
    xs = np.array([0.0, 1.0])
    rgba = np.array([[0.2, 0.6, 0.9, 0.1], [0.2, 0.6, 0.9, 0.1]])
    cam = vi.Camera(width=7, height=5, fx=10.0, fy=10.0, cx=3.5, cy=2.5, near=0.2,
                    viewmat=vi.look_at(np.array([3.5, 0.0, 0.0])).astype(np.float32))
    C, T = dvr.render(vol, xs, rgba, cam)
    t = T[2, 3]
    ok = [abs(t - (1 - 0.1) ** (n / 2.0)) <= 1e-12 for n in (64, 65)]
    assert any(ok)
    assert np.allclose(C[:, 2, 3], rgba[0, :3] * (1 - t), atol=1e-12)
    # rays that miss the box stay transparent
    cam2 = vi.Camera(width=3, height=3, fx=10.0, fy=10.0, cx=1.5, cy=1.5, near=0.2,
                     viewmat=vi.look_at(np.array([3.5, 0.0, 5.0]), target=np.array([3.5, 0.0, 10.0]),
                                        up=np.array([1.0, 0.0, 0.0])).astype(np.float32))
    C2, T2 = dvr.render(vol, xs, rgba, cam2)
    assert np.all(T2 == 1.0) and np.all(C2 == 0.0)
