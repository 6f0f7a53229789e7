"""Torch-tensor front end of libvbm.  PyTorch supplies device memory and streams; every step of the
fine-tuning path runs in the library's HIP kernels.

Gaussian parameters live in one float32 tensor ``P`` of shape [14, stride] on the GPU with rows
means 0-2, scales 3-5, quats 6-9 (w, x, y, z), opacity 10, rgb 11-13 (activated values); raw
optimiser parameters use the same rows with log scales and logit opacity.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np
import torch

from . import _lib as L

ROWS = dict(means=slice(0, 3), scales=slice(3, 6), quats=slice(6, 10), opacity=slice(10, 11), rgb=slice(11, 14))
N_ROWS = 14


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _require_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libvbm operates on GPU tensors only")


def gaussians_struct(P: torch.Tensor, offset: int = 0) -> L.vbm_gaussians:
    """SoA pointer struct over a [14, stride] float32 tensor, starting at column ``offset``."""
    assert P.dtype == torch.float32 and P.dim() == 2 and P.shape[0] == N_ROWS and P.is_contiguous()
    assert 0 <= offset <= P.shape[1]
    base, stride = P.data_ptr() + 4 * int(offset), P.shape[1]
    row = lambda r: base + 4 * r * stride  # noqa: E731
    return L.vbm_gaussians(row(0), row(3), row(6), row(10), row(11), stride)


def pack_params(means, scales, quats, opacity, rgb, device="cuda") -> torch.Tensor:
    arr = np.concatenate([np.asarray(means, np.float32), np.asarray(scales, np.float32), np.asarray(quats, np.float32),
                          np.asarray(opacity, np.float32)[None], np.asarray(rgb, np.float32)], 0)
    return torch.from_numpy(np.ascontiguousarray(arr)).to(device)


def make_tf(xs, rgba) -> L.vbm_tf:
    xs = np.asarray(xs, np.float32)
    rgba = np.asarray(rgba, np.float32)
    if xs.shape[0] > L.VBM_TF_MAX_POINTS:
        raise ValueError("too many transfer-function control points")
    t = L.vbm_tf()
    t.n_points = xs.shape[0]
    for i in range(xs.shape[0]):
        t.x[i] = float(xs[i])
        for c in range(4):
            t.rgba[i][c] = float(rgba[i, c])
    return t


# ----------------------------------------------------------------------------- DWT + construction

def dwt3d(vol: torch.Tensor, J: int, wavelet: str, tf=None) -> torch.Tensor:
    """vol float32 [G, G, G] (with tf = (xs, rgba)) or [4, G^3] RGBA (tf None) -> coefficients [4, G^3]."""
    lib = L.load()
    _require_cuda(vol)
    G = vol.shape[-1] if tf is not None else round(vol.shape[1] ** (1 / 3))
    coeffs = torch.empty(4, G ** 3, dtype=torch.float32, device=vol.device)
    ws = torch.empty(lib.vbm_dwt3d_workspace_size(G, J), dtype=torch.uint8, device=vol.device)
    tfs = make_tf(*tf) if tf is not None else None
    st = lib.vbm_dwt3d(vol.contiguous().data_ptr(), G, J, L.WAVELETS[wavelet], C.byref(tfs) if tfs else None,
                       coeffs.data_ptr(), ws.data_ptr(), ws.numel(), _stream(vol.device))
    L.check(st, "vbm_dwt3d")
    return coeffs


def bank_build(wavelet: str, J: int, tau: float = 0.1, lam: float = 1e-8):
    """Returns (list of entry dicts, packed float32 numpy [7J+1, 12]) from the host FP64 bank build."""
    lib = L.load()
    n = lib.vbm_bank_size(J)
    arr = (L.vbm_bank_entry * n)()
    L.check(lib.vbm_bank_build(L.WAVELETS[wavelet], J, tau, lam, arr), "vbm_bank_build")
    packed = np.zeros((n, L.VBM_BANK_FLOATS), np.float32)
    L.check(lib.vbm_bank_pack(arr, n, packed.ctypes.data_as(C.POINTER(C.c_float))), "vbm_bank_pack")
    entries = [dict(j=e.j, o=e.o, w=e.w, u=np.array(e.u[:]), sigma=np.array(e.sigma[:]), scale=np.array(e.scale[:]),
                    quat=np.array(e.quat[:]), roi_size=e.roi_size) for e in arr]
    return entries, packed


def build_gaussians(coeffs: torch.Tensor, G: int, J: int, bank_packed, K: int, s_mode: str = "paper",
                    delta: float = 0.5, opacity_min: float = 1e-3, opacity_max: float = 0.99, stride: int | None = None,
                    isotropic: bool = False, unit_weight: bool = False, out: torch.Tensor | None = None,
                    offset: int = 0):
    """Top-K + construction.  Returns (P [14, stride] activated parameters, kept int64 [K]).
    With ``out`` given, the K Gaussians are written into its columns [offset, offset + K) and
    ``out`` is returned as P (the other columns are left as they are)."""
    lib = L.load()
    _require_cuda(coeffs)
    dev = coeffs.device
    bank = torch.as_tensor(np.ascontiguousarray(bank_packed, dtype=np.float32)).to(dev)
    if out is None:
        P = torch.zeros(N_ROWS, stride or K, dtype=torch.float32, device=dev)
    else:
        _require_cuda(out)
        if not 0 <= offset or offset + K > out.shape[1]:
            raise ValueError(f"columns [{offset}, {offset + K}) do not fit an output of {out.shape[1]}")
        P = out
    kept = torch.empty(K, dtype=torch.int64, device=dev)
    ws = torch.empty(lib.vbm_build_workspace_size(G, J), dtype=torch.uint8, device=dev)
    opts = L.vbm_build_opts(0 if s_mode == "paper" else 1, delta, opacity_min, opacity_max, int(isotropic),
                            int(unit_weight))
    st = lib.vbm_build_gaussians(coeffs.data_ptr(), G, J, bank.data_ptr(), K, C.byref(opts),
                                 gaussians_struct(P, offset), kept.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev))
    L.check(st, "vbm_build_gaussians")
    return P, kept


def adaptive_select(coeffs: torch.Tensor, G: int, J: int, K_tot: int, alpha: float = 0.5, beta: float = 0.5,
                    lam: float = 3.0, ref: int = 3, min_band: int = 10, capacity: int | None = None):
    """Adaptive per-subband selection.  Returns (kept int64 [count] ascending packed indices,
    band statistics float64 [7J+1][12] with columns L.ADAPTIVE_STATS).  One host sync reads the count;
    a count above the capacity (default: G^3) raises."""
    lib = L.load()
    _require_cuda(coeffs)
    dev = coeffs.device
    cap = G ** 3 if capacity is None else int(capacity)
    kept = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    stats = torch.zeros(7 * J + 1, L.VBM_ADAPTIVE_STATS, dtype=torch.float64, device=dev)
    ws = torch.empty(lib.vbm_adaptive_workspace_size(G, J), dtype=torch.uint8, device=dev)
    opts = L.vbm_adaptive_opts(int(K_tot), float(alpha), float(beta), float(lam), int(ref), int(min_band))
    st = lib.vbm_adaptive_select(coeffs.data_ptr(), G, J, C.byref(opts), cap, kept.data_ptr(), count.data_ptr(),
                                 stats.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev))
    L.check(st, "vbm_adaptive_select")
    n = int(count.item())
    if n > cap:
        raise L.VBMError(f"vbm_adaptive_select kept {n} > capacity {cap}")
    return kept[:n], stats


def construct_gaussians(coeffs: torch.Tensor, G: int, J: int, bank_packed, kept: torch.Tensor, s_mode: str = "paper",
                        delta: float = 0.5, opacity_min: float = 1e-3, opacity_max: float = 0.99,
                        stride: int | None = None, isotropic: bool = False, unit_weight: bool = False):
    """Construction for a given list of packed indices (int64, device).  Returns P [14, stride]."""
    lib = L.load()
    _require_cuda(coeffs)
    dev = coeffs.device
    n = int(kept.numel())
    kept = kept.to(device=dev, dtype=torch.int64).contiguous()
    bank = torch.as_tensor(np.ascontiguousarray(bank_packed, dtype=np.float32)).to(dev)
    stride = stride or max(n, 1)
    P = torch.zeros(N_ROWS, stride, dtype=torch.float32, device=dev)
    opts = L.vbm_build_opts(0 if s_mode == "paper" else 1, delta, opacity_min, opacity_max, int(isotropic),
                            int(unit_weight))
    st = lib.vbm_construct_gaussians(coeffs.data_ptr(), G, J, bank.data_ptr(), kept.data_ptr(), n, C.byref(opts),
                                     gaussians_struct(P), _stream(dev))
    L.check(st, "vbm_construct_gaussians")
    return P


# ----------------------------------------------------------------------------- rendering

def make_view(cam, scene: int = 0) -> L.vbm_view:
    v = L.vbm_view()
    v.scene = scene
    v.width, v.height = int(cam.width), int(cam.height)
    v.fx, v.fy, v.cx, v.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    v.near_plane = float(cam.near)
    vm = np.asarray(cam.viewmat, np.float32).reshape(-1)
    for i in range(12):
        v.viewmat[i] = float(vm[i])
    for i in range(3):
        v.bg[i] = float(cam.bg[i])
    return v


@dataclasses.dataclass
class RenderPlan:
    """A planned batch: host plan struct, device view table and the render workspace."""
    plan: L.vbm_plan
    views: object
    table: torch.Tensor
    ws: torch.Tensor
    cams: list
    view_scene: list
    scene_offsets: np.ndarray
    # Forwards enqueued on this plan so far.  The workspace holds the state of the latest one only
    # (pair lists, lane-group marks, ranges, launch order, per-item records), so a backward must
    # name that forward: render_bwd refuses a FwdOut whose generation is older.
    generation: int = 0

    @property
    def n_pixels(self) -> int:
        return int(self.plan.n_pixels)

    def view_dims(self) -> np.ndarray:
        return np.array([[c.width, c.height] for c in self.cams], dtype=np.int32)

    def pixel_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([c.width * c.height for c in self.cams])]).astype(np.int64)

    def region(self, name: str, dtype=torch.uint8) -> torch.Tensor:
        r = L.REGION[name]
        off, nb = int(self.plan.region_offset[r]), int(self.plan.region_bytes[r])
        return self.ws[off:off + nb].view(dtype)


def plan_batch(cams, scene_offsets=None, view_scene=None, tile: int = 16, sort_bits: int = 8,
               pair_capacity: int = 1 << 20, mode: str = "batched", device="cuda", lds_batch: int = 0,
               lds_batch_bwd: int = 0) -> RenderPlan:
    lib = L.load()
    V = len(cams)
    view_scene = list(view_scene) if view_scene is not None else [0] * V
    scene_offsets = np.asarray(scene_offsets, dtype=np.int64)
    S = scene_offsets.shape[0] - 1
    views = (L.vbm_view * V)(*[make_view(c, s) for c, s in zip(cams, view_scene)])
    sch = L.vbm_schedule(tile, sort_bits, int(pair_capacity), L.MODE_EXACT if mode == "exact" else L.MODE_BATCHED,
                         int(lds_batch), int(lds_batch_bwd))
    plan = L.vbm_plan()
    so = np.ascontiguousarray(scene_offsets)
    L.check(lib.vbm_plan_make(views, V, so.ctypes.data_as(C.POINTER(C.c_int64)), S, C.byref(sch), C.byref(plan), None),
            "vbm_plan_make")
    host = np.zeros(plan.view_table_bytes, dtype=np.uint8)
    L.check(lib.vbm_plan_make(views, V, so.ctypes.data_as(C.POINTER(C.c_int64)), S, C.byref(sch), C.byref(plan),
                              host.ctypes.data), "vbm_plan_make")
    table = torch.from_numpy(host).to(device)
    ws = torch.empty(plan.ws_bytes, dtype=torch.uint8, device=device)
    return RenderPlan(plan, views, table, ws, list(cams), view_scene, scene_offsets)


@dataclasses.dataclass
class FwdOut:
    image: torch.Tensor      # float32 [3 * n_pixels] (per view [3][H][W], concatenated)
    final_T: torch.Tensor    # float32 [n_pixels]
    n_contrib: torch.Tensor  # int32 [n_pixels]
    status: torch.Tensor     # int32 [4]: overflow, pairs, visible items, overflow count
    generation: int = -1     # the plan's forward count after the forward that wrote this output


def render_fwd(rp: RenderPlan, P: torch.Tensor, out: FwdOut | None = None) -> FwdOut:
    lib = L.load()
    _require_cuda(P)
    dev = P.device
    if out is None:
        out = FwdOut(torch.empty(3 * rp.n_pixels, dtype=torch.float32, device=dev),
                     torch.empty(rp.n_pixels, dtype=torch.float32, device=dev),
                     torch.empty(rp.n_pixels, dtype=torch.int32, device=dev),
                     torch.zeros(4, dtype=torch.int32, device=dev))
    st = lib.vbm_render_fwd(C.byref(rp.plan), rp.table.data_ptr(), gaussians_struct(P), out.image.data_ptr(),
                            out.final_T.data_ptr(), out.n_contrib.data_ptr(), out.status.data_ptr(), rp.ws.data_ptr(),
                            rp.ws.numel(), _stream(dev))
    L.check(st, "vbm_render_fwd")
    rp.generation += 1
    out.generation = rp.generation
    return out


def render_bwd(rp: RenderPlan, P: torch.Tensor, dL_dimg: torch.Tensor, fwd: FwdOut, grads: torch.Tensor | None = None,
               accumulate: bool = False) -> torch.Tensor:
    lib = L.load()
    _require_cuda(P, dL_dimg)
    if fwd.generation != rp.generation:
        raise L.VBMError(f"render_bwd: the plan's workspace holds forward {rp.generation}, not forward "
                         f"{fwd.generation} whose output was passed (a later forward on the same plan replaced "
                         "its pair lists); run the forward again first")
    if grads is None:
        grads = torch.zeros_like(P)
    st = lib.vbm_render_bwd(C.byref(rp.plan), rp.table.data_ptr(), gaussians_struct(P), dL_dimg.data_ptr(),
                            fwd.final_T.data_ptr(), fwd.n_contrib.data_ptr(), gaussians_struct(grads),
                            1 if accumulate else 0, rp.ws.data_ptr(), rp.ws.numel(), _stream(P.device))
    L.check(st, "vbm_render_bwd")
    return grads


def split_views(flat: torch.Tensor, cams, channels: int = 3) -> list:
    """Concatenated per-view planar buffer -> list of [channels, H, W] views."""
    out, off = [], 0
    for c in cams:
        n = channels * c.width * c.height
        out.append(flat[off:off + n].view(channels, c.height, c.width) if channels > 1 else
                   flat[off:off + n].view(c.height, c.width))
        off += n
    return out


# ----------------------------------------------------------------------------- loss, optimiser, DVR

class ImageLoss:
    """Preallocated loss workspace for a fixed set of view sizes."""

    def __init__(self, view_dims, kind: str = "l1", lam: float = 0.2, device="cuda"):
        lib = L.load()
        self.dims = np.ascontiguousarray(np.asarray(view_dims, dtype=np.int32).reshape(-1, 2))
        self.kind = 0 if kind == "l1" else 1
        self.lam = float(lam)
        nb = lib.vbm_image_loss_workspace_size(self.dims.ctypes.data_as(C.POINTER(C.c_int32)), self.dims.shape[0],
                                               self.kind)
        self.ws = torch.empty(max(int(nb), 1), dtype=torch.uint8, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)

    def __call__(self, image: torch.Tensor, target: torch.Tensor, grad: torch.Tensor) -> torch.Tensor:
        lib = L.load()
        st = lib.vbm_image_loss(image.data_ptr(), target.data_ptr(), self.dims.ctypes.data_as(C.POINTER(C.c_int32)),
                                self.dims.shape[0], self.kind, self.lam, grad.data_ptr(), self.loss.data_ptr(),
                                self.ws.data_ptr(), self.ws.numel(), _stream(image.device))
        L.check(st, "vbm_image_loss")
        return self.loss


def image_loss_static(image: torch.Tensor, target: torch.Tensor, view_dims, kind: str = "l1", lam: float = 0.2,
                      grad: torch.Tensor | None = None, loss: torch.Tensor | None = None):
    """The image loss through vbm_image_loss_static (no workspace: the library's fixed scratch array).
    Returns (loss float32 [1], dL/dI); pass ``grad`` and ``loss`` to write into existing tensors."""
    lib = L.load()
    _require_cuda(image, target)
    dims = np.ascontiguousarray(np.asarray(view_dims, dtype=np.int32).reshape(-1, 2))
    if grad is None:
        grad = torch.empty_like(image)
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float32, device=image.device)
    st = lib.vbm_image_loss_static(image.data_ptr(), target.data_ptr(), dims.ctypes.data_as(C.POINTER(C.c_int32)),
                                   dims.shape[0], 0 if kind == "l1" else 1, float(lam), grad.data_ptr(),
                                   loss.data_ptr(), _stream(image.device))
    L.check(st, "vbm_image_loss_static")
    return loss, grad


LR_DEFAULT = (1e-3, 5e-3, 1e-3, 5e-3, 2.5e-3)  # means, log scales, quats, logit opacity, rgb


def adam_init(act: torch.Tensor, n: int | None = None):
    """Optimiser state at the start of fine-tuning (vbm_adam_init): returns (raw, m, v), each
    [14, stride] like ``act``; raw holds log scales and logit opacity, m = v = 0."""
    lib = L.load()
    _require_cuda(act)
    raw = torch.empty_like(act)
    m = torch.empty_like(act)
    v = torch.empty_like(act)
    n = act.shape[1] if n is None else int(n)
    st = lib.vbm_adam_init(n, raw.shape[1], gaussians_struct(act), raw.data_ptr(), m.data_ptr(), v.data_ptr(),
                           _stream(act.device))
    L.check(st, "vbm_adam_init")
    return raw, m, v


def adam_step(raw, m, v, grads, act, lr=LR_DEFAULT, step: int = 1, step_dev: torch.Tensor | None = None,
              betas=(0.9, 0.999), eps=1e-15, n: int | None = None):
    lib = L.load()
    o = L.vbm_adam_opts()
    for k in range(5):
        o.lr[k] = float(lr[k])
    o.beta1, o.beta2, o.eps, o.step = betas[0], betas[1], eps, int(step)
    n = raw.shape[1] if n is None else n
    st = lib.vbm_adam_step(n, raw.shape[1], raw.data_ptr(), m.data_ptr(), v.data_ptr(), gaussians_struct(grads),
                           gaussians_struct(act), C.byref(o), _ptr(step_dev), _stream(raw.device))
    L.check(st, "vbm_adam_step")


def dvr_render(vol: torch.Tensor, tf, cams, step_vox: float = 0.5, out: torch.Tensor | None = None) -> torch.Tensor:
    """Ray-marched images of vol [G, G, G] for each camera, concatenated planar [3][H][W] per view
    (written into ``out`` when given)."""
    lib = L.load()
    _require_cuda(vol)
    G = vol.shape[0]
    views = (L.vbm_view * len(cams))(*[make_view(c) for c in cams])
    n = sum(3 * c.width * c.height for c in cams)
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=vol.device)
    elif out.numel() != n or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError(f"dvr_render: out must be {n} contiguous float32 values")
    t = make_tf(*tf)
    st = lib.vbm_dvr_render(vol.contiguous().data_ptr(), G, C.byref(t), views, len(cams), step_vox, out.data_ptr(),
                            _stream(vol.device))
    L.check(st, "vbm_dvr_render")
    return out


# ----------------------------------------------------------------------------------- visual modes
# Sec. 4.4: a series of transfer functions TF_h, each non-zero only on its own value interval of F,
# gives one radiance field RF_h = TF_h(F) per visual mode and one Gaussian set G_h per field.  The
# sets live side by side in one parameter buffer as the scenes of one batch, so all modes are
# fine-tuned in the same launches; afterwards they are rendered separately (one scene per mode) or
# concatenated (one scene holding every column).

def build_mode_sets(vol: torch.Tensor, tfs, J: int, wavelet: str, K, s_mode: str = "paper", **build_kw):
    """One Gaussian set per transfer function (each given as (xs, rgba)), built from the wavelet
    coefficients of TF_h(vol) and written into consecutive columns of one buffer.  K is one count
    for every mode or one per mode.  Returns (P [14, sum K], scene_offsets int64 [n_modes + 1],
    kept: list of int64 [K_h] packed indices)."""
    _require_cuda(vol)
    G = vol.shape[-1]
    Ks = [int(K)] * len(tfs) if np.ndim(K) == 0 else [int(k) for k in K]
    if len(Ks) != len(tfs) or not tfs:
        raise ValueError("one count per transfer function")
    offsets = np.concatenate([[0], np.cumsum(Ks)]).astype(np.int64)
    _, packed = bank_build(wavelet, J)
    P = torch.zeros(N_ROWS, int(offsets[-1]), dtype=torch.float32, device=vol.device)
    kept = []
    for h, tf in enumerate(tfs):
        coeffs = dwt3d(vol, J, wavelet, tf)
        _, kh = build_gaussians(coeffs, G, J, packed, Ks[h], s_mode=s_mode, out=P, offset=int(offsets[h]),
                                **build_kw)
        kept.append(kh)
        del coeffs
    return P, offsets, kept


def mode_views(cams, n_modes: int):
    """Views of a mode batch: every camera once per mode, mode-major.  Returns (cams, view_scene)."""
    return [c for _ in range(n_modes) for c in cams], [h for h in range(n_modes) for _ in cams]


def dvr_render_modes(vol: torch.Tensor, tfs, cams, step_vox: float = 0.5) -> torch.Tensor:
    """Supervision images of a mode batch: the DVR of every RF_h from every camera, mode-major (the
    view order of mode_views)."""
    n = sum(3 * c.width * c.height for c in cams)
    out = torch.empty(len(tfs) * n, dtype=torch.float32, device=vol.device)
    for h, tf in enumerate(tfs):
        dvr_render(vol, tf, cams, step_vox, out=out[h * n:(h + 1) * n])
    return out
