"""Joint-norm global top-K coefficient selection.  Test infrastructure.

The joint magnitude of a coefficient location is the 2-norm over its four RGBA channels
(Supp. A, Joint Multi-Channel Sparsification), so a location is kept or dropped coherently across
channels.  The workloads keep the K locations with the largest joint norm over all subbands
(the paper's per-subband MAD filter is a separate, later step).  Ties go to the lower packed
index.  The norm is evaluated in float32 in the fixed order sqrt(((R^2 + G^2) + B^2) + A^2) so that
the integer decision is taken in the same precision on both sides.
"""
from __future__ import annotations

import numpy as np


def joint_norm_f32(coeffs: np.ndarray) -> np.ndarray:
    """coeffs [4][M] float32 -> v [M] float32."""
    c = np.asarray(coeffs, dtype=np.float32)
    r, g, b, a = c[0], c[1], c[2], c[3]
    return np.sqrt(((r * r + g * g) + b * b) + a * a)


def topk(coeffs: np.ndarray, K: int) -> np.ndarray:
    """Indices of the K largest joint norms (ties -> lower index), returned in ascending index order.

    With t the K-th largest value, that set is every index with v > t plus the lowest-index entries
    with v == t until K are taken.
    """
    v = joint_norm_f32(coeffs)
    M = v.shape[0]
    K = min(int(K), M)
    if K == 0:
        return np.zeros(0, dtype=np.int64)
    t = np.partition(v, M - K)[M - K]
    above = np.nonzero(v > t)[0]
    ties = np.nonzero(v == t)[0][:K - above.size]
    return np.sort(np.concatenate([above, ties])).astype(np.int64)


def topk_bruteforce(coeffs: np.ndarray, K: int) -> np.ndarray:
    """Same set by a full lexicographic sort on (-v, index); for small inputs."""
    v = joint_norm_f32(coeffs)
    order = np.lexsort((np.arange(v.shape[0]), -v))
    return np.sort(order[:K]).astype(np.int64)
