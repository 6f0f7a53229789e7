"""Adam on the raw fine-tuning parameters (Sec. 5, Implementation Details: Adam).  Test infrastructure.

Raw parameters per Gaussian: means (3), log_scales (3), quats (4), logit_opacity (1), rgb (3);
activated scales = exp(log_scales), opacity = sigmoid(logit_opacity).  Gradients of the activated
parameters are chained through the activations, then the textbook Adam update with bias correction
is applied per parameter group with its own learning rate.
"""
from __future__ import annotations

import numpy as np

GROUPS = ("means", "log_scales", "quats", "logit_opacity", "rgb")
DEFAULT_LR = dict(means=1e-3, log_scales=5e-3, quats=1e-3, logit_opacity=5e-3, rgb=2.5e-3)


def raw_from_activated(scales, opacity):
    op = np.asarray(opacity, dtype=np.float64)
    return np.log(np.asarray(scales, dtype=np.float64)), np.log(op / (1.0 - op))


def chain_grads(act_grads: dict, raw: dict) -> dict:
    """Activated-parameter grads -> raw-parameter grads."""
    scales = np.exp(raw["log_scales"])
    op = 1.0 / (1.0 + np.exp(-raw["logit_opacity"]))
    return dict(means=act_grads["means"], log_scales=act_grads["scales"] * scales, quats=act_grads["quats"],
                logit_opacity=act_grads["opacity"] * op * (1.0 - op), rgb=act_grads["rgb"])


def step(raw: dict, grads: dict, m: dict, v: dict, t: int, lr: dict = None, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (t is the 1-based step count).  Returns new (raw, m, v) dicts (FP64)."""
    lr = lr or DEFAULT_LR
    new_raw, new_m, new_v = {}, {}, {}
    for k in GROUPS:
        g = np.asarray(grads[k], dtype=np.float64)
        mk = beta1 * m[k] + (1 - beta1) * g
        vk = beta2 * v[k] + (1 - beta2) * g * g
        mhat = mk / (1 - beta1 ** t)
        vhat = vk / (1 - beta2 ** t)
        new_raw[k] = raw[k] - lr[k] * mhat / (np.sqrt(vhat) + eps)
        new_m[k], new_v[k] = mk, vk
    return new_raw, new_m, new_v
