"""Image losses of the fine-tuning loop (Sec. 4.4: the loss of the cited 3DGS).  Test infrastructure.

  L1      mean |I - I_ref| over views, channels and pixels; dL/dI = sign(I - I_ref) / count, sign(0) = 0
  SSIM    per channel, 11x11 Gaussian window (sigma 1.5, normalised), zero-padded "same" filtering,
          C1 = 0.01^2, C2 = 0.03^2, mean of the SSIM map
  mixed   (1 - lam) L1 + lam (1 - SSIM), lam = 0.2
Gradients are exact (reverse-mode differentiation in float64).
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as Fn

F64 = torch.float64
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def gaussian_window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    x = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-x * x / (2 * sigma * sigma))
    return g / g.sum()


def _blur(x, g1):
    """x [C][H][W] -> separable zero-padded 'same' filtering with the 1D window g1."""
    C = x.shape[0]
    k = g1.shape[0]
    w2 = (g1[:, None] * g1[None, :])[None, None].expand(C, 1, k, k).contiguous()
    return Fn.conv2d(x[None], w2, padding=k // 2, groups=C)[0]


def ssim_map(x, y, size=11, sigma=1.5):
    g1 = torch.as_tensor(gaussian_window(size, sigma), dtype=F64)
    mx, my = _blur(x, g1), _blur(y, g1)
    sxx = _blur(x * x, g1) - mx * mx
    syy = _blur(y * y, g1) - my * my
    sxy = _blur(x * y, g1) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def loss_and_grad(images: list, targets: list, kind: str = "l1", lam: float = 0.2):
    """images/targets: lists of [3][H][W] arrays.  Returns (loss, [dL/dI per view])."""
    xs = [torch.as_tensor(np.asarray(i, dtype=np.float64)).clone().requires_grad_(True) for i in images]
    ys = [torch.as_tensor(np.asarray(t, dtype=np.float64)) for t in targets]
    count = sum(x.numel() for x in xs)
    l1 = sum((x - y).abs().sum() for x, y in zip(xs, ys)) / count
    if kind == "l1":
        loss = l1
    elif kind == "l1_dssim":
        ssim = sum(ssim_map(x, y).sum() for x, y in zip(xs, ys)) / count
        loss = (1 - lam) * l1 + lam * (1 - ssim)
    elif kind == "ssim":
        loss = sum(ssim_map(x, y).sum() for x, y in zip(xs, ys)) / count
    else:
        raise ValueError(kind)
    loss.backward()
    return float(loss.detach()), [x.grad.numpy() for x in xs]


def ssim_pixel_bruteforce(x: np.ndarray, y: np.ndarray, c: int, i: int, j: int, size=11, sigma=1.5) -> float:
    """SSIM map value at one pixel by explicit window sums (zero outside the image)."""
    g1 = gaussian_window(size, sigma)
    h = size // 2
    H, W = x.shape[1:]
    mx = my = sxx = syy = sxy = 0.0
    for di in range(-h, h + 1):
        for dj in range(-h, h + 1):
            ii, jj = i + di, j + dj
            if 0 <= ii < H and 0 <= jj < W:
                w = g1[di + h] * g1[dj + h]
                a, b = float(x[c, ii, jj]), float(y[c, ii, jj])
                mx += w * a
                my += w * b
                sxx += w * a * a
                syy += w * b * b
                sxy += w * a * b
    vx, vy, cxy = sxx - mx * mx, syy - my * my, sxy - mx * my
    return ((2 * mx * my + C1) * (2 * cxy + C2)) / ((mx * mx + my * my + C1) * (vx + vy + C2))
