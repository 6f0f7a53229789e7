"""Fine-tuning step runners (Sec. 4.4: render, image loss, backward, Adam) on top of libvbm.

* ``VBMRender``  -- torch.autograd.Function around vbm_render_fwd / vbm_render_bwd (the backward
  recomputes each pixel's transmittance instead of storing per-Gaussian state).
* ``FineTuner``  -- one fine-tuning iteration in three schedules:
    plain    one view per launch: per view a forward (which synchronises once to size the sort
             exactly), one loss over all views, per view a backward; then Adam
    batched  every view (and scene) in one launch per phase, counts kept on the device; or, with
             size classes, one launch per phase for each class of views (consecutive views of one
             size), each with its own tile edge and radix digit width
    graph    the batched step captured once in a HIP graph and replayed
  All three produce identical pair lists and images; gradients agree up to float atomics order.
  Images do not depend on the tile edge either: a tile's list differs from another tiling's only
  in Gaussians that reach none of its pixels, which every pixel skips.
* ``render_images`` -- a forward-only batch render with exactly counted pair lists (used to render
  the visual-mode sets concatenated or separately after fine-tuning).
* ``autotune``   -- times the batched step for each (tile, radix digit) candidate and picks the
  fastest; run before capture, on a copy of the parameters.  ``autotune_classes`` does so for
  each size class of a batch on its own; ``autotune_schedule`` keeps one schedule for the batch
  or one per size class, whichever step is faster.
* ``size_classes`` -- the runs of consecutive views of equal size.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import api


class VBMRender(torch.autograd.Function):
    """image = render(P) for a planned batch; P is the [14, N] activated parameter tensor.

    The forward reads the plan's overflow flag (one host sync) and raises when the pair lists did
    not fit the plan's capacity, since the image would be incomplete.  The backward needs the pair
    lists and per-item state that the forward left in the plan's workspace; when another forward
    has run on the same plan since (a second loss, a re-render), the backward first re-runs this
    call's forward from the saved P, which rebuilds the same lists and transmittances bit for bit
    (every step of the forward is deterministic), so each backward gets its own forward's state.
    """

    @staticmethod
    def forward(ctx, P: torch.Tensor, rp: api.RenderPlan):
        fwd = api.render_fwd(rp, P.detach().contiguous())
        if int(fwd.status[0].item()) != 0:
            raise api.L.VBMError(f"VBMRender: {int(fwd.status[1].item())} pairs exceed the plan's capacity of "
                                 f"{int(rp.plan.pair_capacity)}; plan the batch with a larger pair_capacity")
        ctx.rp = rp
        ctx.generation = fwd.generation
        ctx.save_for_backward(P, fwd.final_T, fwd.n_contrib)
        return fwd.image

    @staticmethod
    def backward(ctx, grad_image):
        P, final_T, n_contrib = ctx.saved_tensors
        rp = ctx.rp
        Pd = P.detach().contiguous()
        if ctx.generation == rp.generation:
            fwd = api.FwdOut(None, final_T, n_contrib, None, ctx.generation)
        else:
            fwd = api.render_fwd(rp, Pd)
        g = api.render_bwd(rp, Pd, grad_image.contiguous(), fwd)
        return g, None


def size_classes(cams) -> list:
    """Runs of consecutive views with the same (width, height), as [(v0, v1), ...]."""
    out, v0 = [], 0
    for v in range(1, len(cams) + 1):
        if v == len(cams) or (cams[v].width, cams[v].height) != (cams[v0].width, cams[v0].height):
            out.append((v0, v))
            v0 = v
    return out


class FineTuner:
    def __init__(self, P: torch.Tensor, cams, targets: torch.Tensor, scene_offsets=None, view_scene=None,
                 tile: int = 16, sort_bits: int = 8, loss: str = "l1", lam: float = 0.2, lr=api.LR_DEFAULT,
                 schedule: str = "batched", pair_capacity: int | None = None, capacity_margin: float = 1.25,
                 classes=None, class_schedules=None, lds_batch: int = 0, lds_batch_bwd: int = 0):
        """``classes``: consecutive view ranges [(v0, v1), ...] covering every view, each rendered by
        its own launches with (tile, sort_bits[, lds_batch[, lds_batch_bwd]]) from ``class_schedules``
        (default: one class, the whole batch, with ``tile``, ``sort_bits``, ``lds_batch`` and
        ``lds_batch_bwd``)."""
        assert schedule in ("plain", "batched", "graph")
        self.dev = P.device
        self.cams = list(cams)
        self.N = P.shape[1]
        self.scene_offsets = np.asarray(scene_offsets if scene_offsets is not None else [0, self.N], np.int64)
        self.view_scene = list(view_scene) if view_scene is not None else [0] * len(self.cams)
        self.tile, self.sort_bits = tile, sort_bits
        self.classes = [tuple(c) for c in classes] if classes is not None else [(0, len(self.cams))]
        if [v for c in self.classes for v in range(c[0], c[1])] != list(range(len(self.cams))):
            raise ValueError("classes must be consecutive view ranges covering every view once, in order")
        self.class_schedules = ([(tuple(x) + (0, 0))[:4] for x in class_schedules] if class_schedules is not None
                                else [(tile, sort_bits, lds_batch, lds_batch_bwd)] * len(self.classes))
        if len(self.class_schedules) != len(self.classes):
            raise ValueError("one schedule (tile, sort_bits[, lds_batch[, lds_batch_bwd]]) per class")
        self.view_schedule = [self.class_schedules[c] for c, (a, b) in enumerate(self.classes) for _ in range(a, b)]
        self.schedule = schedule
        self.lr = lr
        self.margin = capacity_margin
        self.act = P.contiguous().clone()
        self.raw, self.m, self.v = api.adam_init(self.act)
        self.grads = torch.zeros_like(self.raw)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.targets = targets
        npx = sum(c.width * c.height for c in self.cams)
        self.image = torch.zeros(3 * npx, dtype=torch.float32, device=self.dev)
        self.final_T = torch.zeros(npx, dtype=torch.float32, device=self.dev)
        self.n_contrib = torch.zeros(npx, dtype=torch.int32, device=self.dev)
        self.dL = torch.zeros(3 * npx, dtype=torch.float32, device=self.dev)
        self.loss_fn = api.ImageLoss([[c.width, c.height] for c in self.cams], loss, lam, self.dev)
        self.pix_off = np.concatenate([[0], np.cumsum([c.width * c.height for c in self.cams])]).astype(np.int64)
        self.graph = None
        self.overflows = 0
        self._plan(pair_capacity)

    # -- planning ------------------------------------------------------------------------------
    def _measure_pairs(self) -> list:
        """Exact pair count per view from one exact-mode forward (planning only)."""
        counts = []
        for v, cam in enumerate(self.cams):
            tile, bits, lds, lds_bwd = self.view_schedule[v]
            rp = api.plan_batch([cam], self.scene_offsets, [self.view_scene[v]], tile, bits, 1, "exact", self.dev, lds,
                                lds_bwd)
            out = api.render_fwd(rp, self.act)
            torch.cuda.synchronize(self.dev)
            counts.append(int(out.status[1].item()))
        return counts

    def _plan(self, capacity):
        if capacity is None:
            counts = self._measure_pairs()
        else:
            counts = [capacity] * len(self.cams)
        self.view_caps = [max(1, int(c * self.margin) + 1024) for c in counts]
        if self.schedule == "plain":
            groups = [(v, v + 1, *self.view_schedule[v], self.view_caps[v], "exact") for v in range(len(self.cams))]
        else:
            groups = [(a, b, *self.class_schedules[c], sum(self.view_caps[a:b]) if capacity is None else capacity,
                       "batched") for c, (a, b) in enumerate(self.classes)]
        self.plans, self.outs = [], []
        for a, b, tile, bits, lds, lds_bwd, cap, mode in groups:
            self.plans.append(api.plan_batch(self.cams[a:b], self.scene_offsets, self.view_scene[a:b], tile, bits, cap,
                                             mode, self.dev, lds, lds_bwd))
            pa, pb = int(self.pix_off[a]), int(self.pix_off[b])
            self.outs.append(api.FwdOut(self.image[3 * pa:3 * pb], self.final_T[pa:pb], self.n_contrib[pa:pb],
                                        torch.zeros(4, dtype=torch.int32, device=self.dev)))
        self.graph = None

    # -- one iteration ---------------------------------------------------------------------------
    def _step_body(self):
        # plain: one plan per view (exact mode); batched / graph: one plan per class of views
        for rp, out in zip(self.plans, self.outs):
            api.render_fwd(rp, self.act, out)
        self.loss_fn(self.image, self.targets, self.dL)
        pix = 0
        for k, (rp, out) in enumerate(zip(self.plans, self.outs)):
            n = rp.n_pixels
            api.render_bwd(rp, self.act, self.dL[3 * pix:3 * (pix + n)], out, self.grads, accumulate=k > 0)
            pix += n
        api.adam_step(self.raw, self.m, self.v, self.grads, self.act, self.lr, step_dev=self.step_dev)

    def step(self):
        if self.schedule == "graph":
            if self.graph is None:
                self._capture()
            self.graph.replay()
        else:
            self._step_body()

    def _capture(self):
        # Every buffer of the step is preallocated and the library allocates nothing, so the step
        # is captured directly; the capture executes nothing, the first replay is the first step.
        torch.cuda.synchronize(self.dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step_body()

    def overflowed(self) -> bool:
        """True if any forward since the last check dropped pairs (reads the device counts, one host
        sync, and clears them)."""
        hit = any(int(o.status[0].item()) != 0 or int(o.status[3].item()) != 0 for o in self.outs)
        for o in self.outs:
            o.status[3].zero_()
        return hit

    def check_capacity(self) -> bool:
        """Reads the overflow flags (one host sync).  If a forward dropped pairs, re-plans with the
        exact counts of the current parameters, so the next step renders complete lists (its graph is
        captured again); returns True when it re-planned."""
        if not self.overflowed():
            return False
        self.overflows += 1
        self._plan(None)
        return True

    def pair_count(self) -> int:
        return sum(int(o.status[1].item()) for o in self.outs)

    def loss(self) -> float:
        return float(self.loss_fn.loss.item())


def render_images(P: torch.Tensor, cams, scene_offsets=None, view_scene=None, tile: int = 16,
                  sort_bits: int = 8) -> torch.Tensor:
    """Forward render of a batch with complete pair lists: counts every view's pairs exactly (one
    exact-mode forward per view), then renders all views in one batched forward planned for that
    count.  Returns the images, planar [3][H][W] per view, concatenated."""
    N = P.shape[1]
    so = np.asarray(scene_offsets if scene_offsets is not None else [0, N], np.int64)
    vs = list(view_scene) if view_scene is not None else [0] * len(cams)
    total = 0
    for v, cam in enumerate(cams):
        rp = api.plan_batch([cam], so, [vs[v]], tile, sort_bits, 1, "exact", P.device)
        out = api.render_fwd(rp, P)
        torch.cuda.synchronize(P.device)
        total += int(out.status[1].item())
    rp = api.plan_batch(cams, so, vs, tile, sort_bits, max(total, 1), "batched", P.device)
    out = api.render_fwd(rp, P)
    torch.cuda.synchronize(P.device)
    if int(out.status[0].item()) != 0:
        raise RuntimeError("render_images: the batched forward dropped pairs")
    return out.image


# (tile edge, tile-sort digit width, LDS batch depth of the forward and of the backward compositing
# list walk; 0 = scalar cache), in order of preference: the tuner keeps the first one within
# TUNE_MARGIN of the fastest
TUNE_CANDIDATES = ((16, 8, 0, 0), (16, 4, 0, 0), (8, 8, 0, 0), (32, 8, 0, 0), (16, 8, 32, 0), (16, 8, 64, 0),
                   (16, 8, 32, 32))
TUNE_MARGIN = 0.01


def _pixel_range(cams, a, b):
    off = np.concatenate([[0], np.cumsum([c.width * c.height for c in cams])]).astype(np.int64)
    return int(off[a]), int(off[b])


def autotune_classes(P: torch.Tensor, cams, targets: torch.Tensor, scene_offsets=None, view_scene=None,
                     classes=None, loss: str = "l1", lam: float = 0.2, candidates=TUNE_CANDIDATES, steps: int = 5,
                     warmup: int = 2) -> dict:
    """Picks a schedule (tile, sort_bits, lds_batch, lds_batch_bwd) for each size class of a batch on its own (default classes: the runs
    of equal-size views): every candidate runs the batched step of that class's views alone (their
    targets, all Gaussians, Adam included) and the fastest is kept.  Returns dict(classes,
    schedules [(tile, sort_bits, lds_batch, lds_batch_bwd)] per class, tables [per-class candidate
    tables])."""
    classes = size_classes(cams) if classes is None else [tuple(c) for c in classes]
    vs = list(view_scene) if view_scene is not None else [0] * len(cams)
    schedules, tables = [], []
    for a, b in classes:
        pa, pb = _pixel_range(cams, a, b)
        r = autotune(P, cams[a:b], targets[3 * pa:3 * pb], scene_offsets, vs[a:b], loss=loss, lam=lam,
                     candidates=candidates, steps=steps, warmup=warmup)
        schedules.append((r["tile"], r["sort_bits"], r["lds_batch"], r["lds_batch_bwd"]))
        tables.append(r["table"])
    return dict(classes=classes, schedules=schedules, tables=tables)


def autotune(P: torch.Tensor, cams, targets: torch.Tensor, scene_offsets=None, view_scene=None, loss: str = "l1",
             lam: float = 0.2, candidates=TUNE_CANDIDATES, steps: int = 5, warmup: int = 2,
             margin: float = TUNE_MARGIN) -> dict:
    """Chooses the tile edge, the radix digit width of the tile sort and the LDS batch depth of the
    compositing list walk for a batch.

    Each candidate (tile, sort_bits, lds_batch, lds_batch_bwd) gets its own plan (exact pair counts, capacity
    margin) and runs ``warmup`` + ``steps`` eager batched iterations on a copy of P (FineTuner
    clones it), timed with a device synchronisation on both sides.  The pick is the first candidate,
    in the given order of preference, whose time is within ``margin`` (a fraction) of the fastest,
    so that differences at the level of timing noise do not change the schedule from run to run.
    Returns it as dict(tile, sort_bits, lds_batch, lds_batch_bwd, ms) plus the table of every
    candidate's ms per step.
    """
    table = []
    for cand in candidates:
        tile, bits, lds, lds_bwd = (tuple(cand) + (0, 0))[:4]
        ft = FineTuner(P, cams, targets, scene_offsets, view_scene, tile=tile, sort_bits=bits, lds_batch=lds,
                       lds_batch_bwd=lds_bwd, loss=loss, lam=lam, schedule="batched")
        table.append(dict(tile=tile, sort_bits=bits, lds_batch=lds, lds_batch_bwd=lds_bwd,
                          ms=_time_steps(ft, steps, warmup)))
        del ft
    fastest = min(d["ms"] for d in table)
    best = next(d for d in table if d["ms"] <= fastest * (1.0 + margin))
    return dict(tile=best["tile"], sort_bits=best["sort_bits"], lds_batch=best["lds_batch"],
                lds_batch_bwd=best["lds_batch_bwd"], ms=best["ms"], table=table)


def _time_steps(ft: "FineTuner", steps: int, warmup: int) -> float:
    """ms per eager step after ``warmup`` steps (device-synchronised on both sides); inf when a
    step overflowed its pair capacity."""
    for _ in range(warmup):
        ft.step()
    torch.cuda.synchronize(ft.dev)
    t0 = time.perf_counter()
    for _ in range(steps):
        ft.step()
    torch.cuda.synchronize(ft.dev)
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return float("inf") if ft.overflowed() else ms


def autotune_schedule(P: torch.Tensor, cams, targets: torch.Tensor, scene_offsets=None, view_scene=None,
                      loss: str = "l1", lam: float = 0.2, candidates=TUNE_CANDIDATES, steps: int = 5,
                      warmup: int = 2) -> dict:
    """The step schedule of a batch: the best single schedule for the whole batch and, when
    the batch holds views of several sizes, the best per size class (autotune_classes); the per-class
    schedule (one launch per class and phase) is taken when its whole step is faster by more than
    TUNE_MARGIN.  Returns the FineTuner keywords (tile, sort_bits, lds_batch, lds_batch_bwd, classes,
    class_schedules) plus the measurements (single_ms: the single schedule's step)."""
    whole = autotune(P, cams, targets, scene_offsets, view_scene, loss=loss, lam=lam, candidates=candidates,
                     steps=steps, warmup=warmup)
    out = dict(tile=whole["tile"], sort_bits=whole["sort_bits"], lds_batch=whole["lds_batch"],
               lds_batch_bwd=whole["lds_batch_bwd"], classes=None,
               class_schedules=None, ms=whole["ms"], single_ms=whole["ms"], table=whole["table"])
    classes = size_classes(cams)
    if len(classes) > 1:
        ct = autotune_classes(P, cams, targets, scene_offsets, view_scene, classes, loss=loss, lam=lam,
                              candidates=candidates, steps=steps, warmup=warmup)
        ft = FineTuner(P, cams, targets, scene_offsets, view_scene, loss=loss, lam=lam, schedule="batched",
                       classes=classes, class_schedules=ct["schedules"])
        ms = _time_steps(ft, steps, warmup)
        del ft
        out.update(class_tables=ct["tables"], per_class=dict(classes=classes, schedules=ct["schedules"], ms=ms))
        if ms < whole["ms"] * (1.0 - TUNE_MARGIN):
            out.update(classes=classes, class_schedules=ct["schedules"], ms=ms)
    return out
