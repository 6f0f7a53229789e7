"""FP64 EWA projection, front-to-back compositing and its exact gradient.  Test infrastructure.

Fine-tuning renders the Gaussian set G = {(mu, Sigma, c, alpha)} (Sec. 3, 3D Gaussian Splatting)
with the cited 3DGS rasteriser and back-propagates an image loss (Sec. 4.4).  The values here are
computed in float64 from the float32 parameters over the float32 pair lists of ``binning``:

  per pixel p = (i + 0.5, j + 0.5), over its tile's list in order:
    d = mean2d - p;  power = -1/2 (A dx^2 + C dy^2) - B dx dy   with [[A, B], [B, C]] = Sigma2^-1
    skip if power > 0;  alpha = min(0.99, o exp(power));  skip if alpha < 1/255
    T' = T (1 - alpha);  stop (without adding) if T' < 1e-4
    C += c alpha T;  T = T';  n_contrib = position + 1
  output C + T bg, final T, n_contrib.

The gradient is the exact derivative of this definition (taken by reverse-mode automatic
differentiation in float64 on the CPU, tile by tile), including zero derivative where the 0.99
clamp or the field-of-view clamp of the Jacobian is active.  ``render_backward_manual`` restates
the same gradient as the reverse-order recursion that recomputes T by division from the final
transmittance; the two agree to rounding (a test pins this).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import binning

F64 = torch.float64
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), dtype=F64)


def quat_to_rot(q):
    """q [4][N] (unnormalised) -> R [N][3][3] (torch, differentiable)."""
    qn = q / torch.sqrt((q * q).sum(0, keepdim=True))
    w, x, y, z = qn[0], qn[1], qn[2], qn[3]
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)
    return R


def project_fp64(means, scales, quats, cam):
    """EWA projection in float64 (torch, differentiable).

    means/scales [3][N], quats [4][N] -> mean2d [N][2], conic [N][3] = (A, B, C), depth [N].
    """
    V = _t(cam.viewmat)
    Rv, tv = V[:, :3], V[:, 3]
    Xc = Rv @ means + tv[:, None]                     # [3][N]
    X, Y, Z = Xc[0], Xc[1], Xc[2]
    fx, fy = float(cam.fx), float(cam.fy)
    limx = 1.3 * (0.5 * cam.width / fx)
    limy = 1.3 * (0.5 * cam.height / fy)
    Xt = torch.clamp(X / Z, -limx, limx) * Z
    Yt = torch.clamp(Y / Z, -limy, limy) * Z
    zero = torch.zeros_like(Z)
    Jm = torch.stack([torch.stack([fx / Z, zero, -fx * Xt / (Z * Z)], -1),
                      torch.stack([zero, fy / Z, -fy * Yt / (Z * Z)], -1)], -2)      # [N][2][3]
    Rq = quat_to_rot(quats)                                                         # [N][3][3]
    M = Rq * scales.T[:, None, :]                                                   # R_q diag(s)
    Vm = Jm @ Rv[None] @ M                                                          # [N][2][3]
    S2 = Vm @ Vm.transpose(1, 2)
    a = S2[:, 0, 0] + 0.3
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + 0.3
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det], -1)
    mean2d = torch.stack([fx * (X / Z) + cam.cx, fy * (Y / Z) + cam.cy], -1)
    return mean2d, conic, Z


def _tile_pixels(cam, tile, tx, ty):
    xs = np.arange(tx * tile, min((tx + 1) * tile, cam.width))
    ys = np.arange(ty * tile, min((ty + 1) * tile, cam.height))
    YY, XX = np.meshgrid(ys, xs, indexing="ij")
    return XX.reshape(-1), YY.reshape(-1)


def composite_tile(pix, m2d, con, op, rgb, bg, rel_alpha=1e-4, rel_t=1e-3, return_stop=False):
    """Vectorised compositing of one tile.  pix [P][2] sample points, list tensors of length L.

    Returns (color [P][3], final_T [P], n_contrib [P], flagged [P], contrib mask [P][L]), and with
    ``return_stop`` also the stop position [P]: the list position of the Gaussian that would have
    taken T below 1e-4, or L when none does (the number of list entries the pixel takes into account).
    ``flagged`` marks pixels where an evaluated Gaussian sits within a relative window of a decision
    threshold (1/255, 0.99 or the 1e-4 stop), where float32 and float64 may legitimately branch apart.
    """
    P, L = pix.shape[0], m2d.shape[0]
    if L == 0:
        z = torch.zeros(P, dtype=torch.bool)
        out = (bg[None, :].expand(P, 3).clone(), torch.ones(P, dtype=F64), torch.zeros(P, dtype=torch.int64), z,
               torch.zeros(P, 0, dtype=torch.bool))
        return out + (torch.zeros(P, dtype=torch.int64),) if return_stop else out
    dx = m2d[None, :, 0] - pix[:, None, 0]
    dy = m2d[None, :, 1] - pix[:, None, 1]
    power = -0.5 * (con[None, :, 0] * dx * dx + con[None, :, 2] * dy * dy) - con[None, :, 1] * dx * dy
    og = op[None, :] * torch.exp(power)
    alpha = torch.clamp(og, max=ALPHA_MAX)
    with torch.no_grad():
        valid = (power <= 0) & (alpha >= ALPHA_MIN)
        ae = torch.where(valid, alpha, torch.zeros_like(alpha))
        t_after = torch.cumprod(1 - ae, 1)
        stop = valid & (t_after < T_MIN)
        idx = torch.arange(L)
        s = torch.where(stop.any(1), stop.to(torch.int64).argmax(1), torch.full((P,), L, dtype=torch.int64))
        contrib = valid & (idx[None, :] < s[:, None])
        last = L - 1 - contrib.flip(1).to(torch.int64).argmax(1)
        n_contrib = torch.where(contrib.any(1), last + 1, torch.zeros_like(last))
        evaluated = idx[None, :] <= s[:, None]
        near = ((og - ALPHA_MIN).abs() <= rel_alpha * ALPHA_MIN) | ((og - ALPHA_MAX).abs() <= rel_alpha * ALPHA_MAX)
        near = near | (valid & ((t_after - T_MIN).abs() <= rel_t * T_MIN))
        flagged = (near & evaluated).any(1)
    a_c = torch.where(contrib, alpha, torch.zeros_like(alpha))
    cp = torch.cumprod(1 - a_c, 1)
    t_before = torch.cat([torch.ones(P, 1, dtype=F64), cp[:, :-1]], 1)
    t_final = cp[:, -1]
    color = (a_c * t_before) @ rgb + t_final[:, None] * bg[None, :]
    if return_stop:
        return color, t_final, n_contrib, flagged, contrib, s
    return color, t_final, n_contrib, flagged, contrib


class Batch:
    """A batch of views over one concatenated Gaussian set (optionally several scenes)."""

    def __init__(self, gs, cams, tile, view_scene=None, scene_offsets=None):
        self.gs = gs
        self.cams = list(cams)
        self.tile = int(tile)
        N = np.asarray(gs.opacity).shape[0]
        self.view_scene = list(view_scene) if view_scene is not None else [0] * len(self.cams)
        self.scene_offsets = np.asarray(scene_offsets if scene_offsets is not None else [0, N], dtype=np.int64)
        self.pairs = binning.pair_lists(gs, self.cams, self.tile, self.view_scene, self.scene_offsets)
        # float64 parameter values used for the image and gradient (default: the float32 inputs);
        # the pair lists stay those decided from the float32 inputs.
        self.params64 = {k: np.asarray(getattr(gs, k), dtype=np.float64)
                         for k in ("means", "scales", "quats", "opacity", "rgb")}

    def item_gaussian(self):
        """Scene-global Gaussian index of every item."""
        out = []
        for v in range(len(self.cams)):
            s = self.view_scene[v]
            out.append(np.arange(self.scene_offsets[s], self.scene_offsets[s + 1]))
        return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)

    def leaf_params(self):
        return {k: _t(v).clone().requires_grad_(True) for k, v in self.params64.items()}

    def project_items(self, P):
        """Per-item FP64 mean2d, conic, opacity, rgb (differentiable in the leaf params P)."""
        m2d, con, op, rgb = [], [], [], []
        for v, cam in enumerate(self.cams):
            s = self.view_scene[v]
            s0, s1 = int(self.scene_offsets[s]), int(self.scene_offsets[s + 1])
            mm, cc, _ = project_fp64(P["means"][:, s0:s1], P["scales"][:, s0:s1], P["quats"][:, s0:s1], cam)
            m2d.append(mm)
            con.append(cc)
            op.append(P["opacity"][s0:s1])
            rgb.append(P["rgb"][:, s0:s1].T)
        return torch.cat(m2d), torch.cat(con), torch.cat(op), torch.cat(rgb)

    def tiles(self):
        """Yields (view, tx, ty, global tile, pixel xs, pixel ys, item list)."""
        toff = self.pairs["tile_offset"]
        rng_ = self.pairs["ranges"]
        items = self.pairs["item"]
        for v, cam in enumerate(self.cams):
            TX = -(-cam.width // self.tile)
            TY = -(-cam.height // self.tile)
            for ty in range(TY):
                for tx in range(TX):
                    gt = int(toff[v] + ty * TX + tx)
                    s, e = rng_[gt]
                    xs, ys = _tile_pixels(cam, self.tile, tx, ty)
                    yield v, tx, ty, gt, xs, ys, items[s:e]


def render_forward(batch: Batch, rel_alpha=1e-4, rel_t=1e-3):
    """Returns per view: image [3][H][W], final_T [H][W], n_contrib [H][W], flagged [H][W] and
    n_visited [H][W] (the stop position of composite_tile) (numpy)."""
    with torch.no_grad():
        P = batch.leaf_params()
        m2d, con, op, rgb = batch.project_items(P)
    out = []
    for cam in batch.cams:
        out.append(dict(image=np.zeros((3, cam.height, cam.width)), final_T=np.ones((cam.height, cam.width)),
                        n_contrib=np.zeros((cam.height, cam.width), dtype=np.int64),
                        flagged=np.zeros((cam.height, cam.width), dtype=bool),
                        n_visited=np.zeros((cam.height, cam.width), dtype=np.int64)))
    with torch.no_grad():
        for v, tx, ty, gt, xs, ys, it in batch.tiles():
            cam = batch.cams[v]
            it_t = torch.as_tensor(it, dtype=torch.int64)
            pix = torch.stack([_t(xs + 0.5), _t(ys + 0.5)], 1)
            col, tf, nc, fl, _, stop = composite_tile(pix, m2d[it_t], con[it_t], op[it_t], rgb[it_t], _t(cam.bg),
                                                      rel_alpha, rel_t, return_stop=True)
            o = out[v]
            o["image"][:, ys, xs] = col.T.numpy()
            o["final_T"][ys, xs] = tf.numpy()
            o["n_contrib"][ys, xs] = nc.numpy()
            o["flagged"][ys, xs] = fl.numpy()
            o["n_visited"][ys, xs] = stop.numpy()
    return out


def render_backward(batch: Batch, dL_dimg: list):
    """Exact FP64 gradient of sum_v <dL_dimg[v], image_v> w.r.t. the activated parameters.

    Returns (grads dict with means [3][N], scales [3][N], quats [4][N], opacity [N], rgb [3][N];
    per-item 2D grads dict mean2d [I][2], conic [I][3], opacity [I], rgb [I][3]).
    """
    P = batch.leaf_params()
    m2d, con, op, rgb = batch.project_items(P)
    L2 = {k: t.detach().clone().requires_grad_(True) for k, t in
          (("mean2d", m2d), ("conic", con), ("opacity", op), ("rgb", rgb))}
    for v, tx, ty, gt, xs, ys, it in batch.tiles():
        if len(it) == 0:
            continue
        cam = batch.cams[v]
        it_t = torch.as_tensor(it, dtype=torch.int64)
        pix = torch.stack([_t(xs + 0.5), _t(ys + 0.5)], 1)
        col, _, _, _, _ = composite_tile(pix, L2["mean2d"][it_t], L2["conic"][it_t], L2["opacity"][it_t],
                                         L2["rgb"][it_t], _t(cam.bg))
        g = _t(np.asarray(dL_dimg[v])[:, ys, xs].T)
        (col * g).sum().backward()
    grads2d = {k: (t.grad if t.grad is not None else torch.zeros_like(t)) for k, t in L2.items()}
    torch.autograd.backward([m2d, con, op, rgb],
                            [grads2d["mean2d"], grads2d["conic"], grads2d["opacity"], grads2d["rgb"]])
    grads = {k: (t.grad if t.grad is not None else torch.zeros_like(t)).numpy() for k, t in P.items()}
    return grads, {k: t.numpy() for k, t in grads2d.items()}


def render_backward_manual(batch: Batch, dL_dimg: list):
    """Per-item 2D gradients by the reverse-order recursion with T recomputed by division.

    For each pixel, walking its list from n_contrib - 1 down to 0 over contributing Gaussians:
      T_i = T_{i+1} / (1 - alpha_i)                     (starting from the final transmittance)
      A_i = c_{i+1} alpha_{i+1} + (1 - alpha_{i+1}) A_{i+1}, A_last = bg   (colour behind i, per unit T)
      dC/dc_i = alpha_i T_i,   dC/dalpha_i = T_i (c_i - A_i)
      dalpha/do = G, dalpha/dpower = alpha (both 0 where the 0.99 clamp holds)
    Pure-Python loops: for small cases only.
    """
    with torch.no_grad():
        P = batch.leaf_params()
        m2d, con, op, rgb = (t.numpy() for t in batch.project_items(P))
    I = m2d.shape[0]
    g_m = np.zeros((I, 2))
    g_c = np.zeros((I, 3))
    g_o = np.zeros(I)
    g_rgb = np.zeros((I, 3))
    fwd = render_forward(batch)
    for v, tx, ty, gt, xs, ys, it in batch.tiles():
        cam = batch.cams[v]
        bg = np.asarray(cam.bg, dtype=np.float64)
        for x, y in zip(xs, ys):
            px, py = x + 0.5, y + 0.5
            T = fwd[v]["final_T"][y, x]
            n = fwd[v]["n_contrib"][y, x]
            dC = np.asarray(dL_dimg[v])[:, y, x].astype(np.float64)
            acc = bg.copy()
            last_a, last_c = 0.0, np.zeros(3)
            for pos in range(n - 1, -1, -1):
                i = it[pos]
                dx, dy = m2d[i, 0] - px, m2d[i, 1] - py
                A, B, C = con[i]
                power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy
                if power > 0:
                    continue
                G = math.exp(power)
                og = op[i] * G
                a = min(ALPHA_MAX, og)
                if a < ALPHA_MIN:
                    continue
                T = T / (1.0 - a)
                acc = last_a * last_c + (1.0 - last_a) * acc
                c = rgb[i]
                g_rgb[i] += a * T * dC
                dL_da = float(np.dot(dC, T * (c - acc)))
                last_a, last_c = a, c
                if og > ALPHA_MAX:
                    continue
                g_o[i] += dL_da * G
                dL_dp = dL_da * a
                g_m[i, 0] += dL_dp * (-(A * dx + B * dy))
                g_m[i, 1] += dL_dp * (-(C * dy + B * dx))
                g_c[i, 0] += dL_dp * (-0.5 * dx * dx)
                g_c[i, 1] += dL_dp * (-dx * dy)
                g_c[i, 2] += dL_dp * (-0.5 * dy * dy)
    return dict(mean2d=g_m, conic=g_c, opacity=g_o, rgb=g_rgb)


def composite_pixel_bruteforce(px, py, cand, m2d, con, op, rgb, bg):
    """Pure-Python sequential compositing of one pixel over an explicit candidate order."""
    T = 1.0
    C = [0.0, 0.0, 0.0]
    n_contrib = 0
    for pos, i in enumerate(cand):
        dx, dy = m2d[i][0] - px, m2d[i][1] - py
        A, B, Cc = con[i]
        power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
        if power > 0:
            continue
        a = min(ALPHA_MAX, op[i] * math.exp(power))
        if a < ALPHA_MIN:
            continue
        Tn = T * (1.0 - a)
        if Tn < T_MIN:
            break
        for ch in range(3):
            C[ch] += rgb[i][ch] * a * T
        T = Tn
        n_contrib = pos + 1
    return [C[ch] + T * bg[ch] for ch in range(3)], T, n_contrib


def composite_pixel_outcomes(px, py, cand, m2d, con, op, rgb, bg, rel_alpha=1e-4, rel_t=1e-3, max_branches=64):
    """Every correct result of compositing one pixel when some decisions sit at a threshold.

    Follows ``composite_pixel_bruteforce``, but where an evaluation lies within the flagging window
    of ``composite_tile`` -- o G within rel_alpha of 1/255 (skip or keep), or the transmittance after
    it within rel_t of 1e-4 (stop or add) -- the other decision is followed as well, since a float32
    renderer may take either there.  (The 0.99 clamp needs no branch: the clamped alpha is
    continuous.)  Returns the list of (colour [3], T, n_contrib) over all branch combinations, the
    FP64 decisions' own among them; at most max_branches are followed.
    """
    results = []

    def finish(T, C, n):
        results.append(([C[ch] + T * bg[ch] for ch in range(3)], T, n))

    def keep(pos, i, a, T, C, n):
        """Adds Gaussian i at list position pos unless the stop rule ends the pixel there; returns
        (T, C, n, ended)."""
        Tn = T * (1.0 - a)
        stop = Tn < T_MIN
        if abs(Tn - T_MIN) <= rel_t * T_MIN and len(results) + 1 < max_branches:
            if stop:
                run(pos + 1, Tn, [C[ch] + rgb[i][ch] * a * T for ch in range(3)], pos + 1)
            else:
                finish(T, C, n)
        if stop:
            finish(T, C, n)
            return T, C, n, True
        return Tn, [C[ch] + rgb[i][ch] * a * T for ch in range(3)], pos + 1, False

    def run(pos, T, C, n):
        while pos < len(cand):
            i = cand[pos]
            dx, dy = m2d[i][0] - px, m2d[i][1] - py
            A, B, Cc = con[i]
            power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
            if power > 0:
                pos += 1
                continue
            og = op[i] * math.exp(power)
            a = min(ALPHA_MAX, og)
            valid = a >= ALPHA_MIN
            if abs(og - ALPHA_MIN) <= rel_alpha * ALPHA_MIN and len(results) + 1 < max_branches:
                if valid:
                    run(pos + 1, T, list(C), n)
                else:
                    T2, C2, n2, ended = keep(pos, i, a, T, list(C), n)
                    if not ended:
                        run(pos + 1, T2, C2, n2)
            if valid:
                T, C, n, ended = keep(pos, i, a, T, C, n)
                if ended:
                    return
            pos += 1
        finish(T, C, n)

    run(0, 1.0, [0.0, 0.0, 0.0], 0)
    return results
