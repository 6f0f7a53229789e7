#!/usr/bin/env python
"""Fine-tuning throughput of the VBM fine-tuning loop on one MI355X.

One step = one image-space fine-tuning iteration (Sec. 4.4): EWA projection of every Gaussian in
every view, binning with the depth-keyed radix sort, front-to-back compositing, the image loss
(0.8 L1 + 0.2 D-SSIM) and its gradient, the reverse-order backward through compositing and
projection, and one Adam step -- all in libvbm's HIP kernels.  The Gaussians come from the method's
own initialisation (TF -> 3D DWT -> top-K by joint norm -> transition-bank construction), run once
on the GPU before timing, and the targets from the GPU ray marcher, also before timing.

Workload (default "H"): 512^3 synthetic turbulence volume (random phases, E(k) ~ k^-5/3 for
1 <= k <= 64, min-max normalised), bior4.4 J=5, the top 1,000,000 coefficients, 8 orbit views at
1920x1080, 16x16 tiles.  Reported value: iterations/sec of the batched schedule (every view in one
launch per phase, captured in a HIP graph), with the plain one-view-per-launch schedule timed
alongside, the compositing kernels' roofline and the CPU oracle timed on a bounded sample.

Prints exactly one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fine-tune iters/sec (fwd+bwd, 1M Gaussians, 1080p, 8 views) batched vs plain"
HBM_PEAK_GBS = 8000.0
# MI355X vector ALU: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz issue 39.3e12 lane-operations/s; an FMA
# counts 2 flops, so 78.6 TFLOP/s of float32 without packed instructions (which every device compile
# here disables); AMD's published 157.3 TFLOP/s counts the packed (two-wide) FMA.
CU, SIMD_PER_CU, LANES_PER_SIMD, CLOCK_GHZ = 256, 4, 16, 2.4
FP32_ALU_PEAK_TFLOPS = round(CU * SIMD_PER_CU * LANES_PER_SIMD * 2 * CLOCK_GHZ / 1e3, 1)
FP32_PUBLISHED_PACKED_TFLOPS = 157.3
# Algorithmic cost per (pixel, Gaussian) evaluation of the compositing kernels.
FLOPS_FWD_EVAL, FLOPS_FWD_USED = 17, 8
FLOPS_BWD_EVAL, FLOPS_BWD_USED = 17, 40
# Algorithmic HBM bytes.  Forward: per pair the 4-byte item id and the 36-byte record (32-byte
# compositing record + blue); per pixel the image (12), final T (4) and contribution count (4)
# written.  Backward: per pair the same 40 bytes read plus nine 4-byte gradient sums added; per
# pixel dL/dI (12), final T (4) and the count (4) read -- it reads no image and writes nothing per
# pixel.  (The lane-group marks the forward writes back into visited pair values are not counted.)
BYTES_PER_PAIR_FWD, BYTES_PER_PIXEL_FWD = 40, 20
BYTES_PER_PAIR_BWD, BYTES_PER_PIXEL_BWD = 76, 20
# adaptive selection: 16 B read + 4 B key written, eight select passes (the median and the
# K_band-th largest share four) and three count/flag/write passes over the 4-byte keys, per coefficient
ADAPTIVE_BYTES_PER_COEF = 16 + 4 + 8 * 4 + 3 * 4

WORKLOADS = {
    "c0": dict(config=0, G=32, J=1, wavelet="haar", K=2048, views=1, W=64, H=64, tile=16, loss="l1",
               desc="32^3 blobs, Haar J=1, top-2048 Gaussians, one 64x64 view, L1, Adam"),
    "c3": dict(config=3, G=512, J=5, wavelet="bior4.4", K=2_000_000, views=16, W=1920, H=1080, tile=16,
               loss="l1_dssim", desc="512^3 turbulence (E(k)~k^-5/3, kmax 64), bior4.4 J=5, top-2M Gaussians, "
                                     "16 orbit views 1920x1080, loss 0.8 L1 + 0.2 D-SSIM, Adam"),
    "c4": dict(config=4, wavelet="bior4.4", tile=16, loss="l1_dssim", views_per_scene=4,
               scenes=[dict(G=64, J=3, K=50_000, W=512, H=512), dict(G=128, J=3, K=200_000, W=800, H=800),
                       dict(G=256, J=4, K=800_000, W=1280, H=720), dict(G=384, J=5, K=1_500_000, W=1920, H=1080)],
               desc="4 scenes (64^3/128^3/256^3/384^3 blobs + k^-2 noise, one transfer function, bior4.4 "
                    "J=3/3/4/5, top 50k/200k/800k/1.5M Gaussians), 4 orbit views each at 512x512/800x800/"
                    "1280x720/1920x1080, all 16 in one batch, loss 0.8 L1 + 0.2 D-SSIM, Adam"),
    "H": dict(config=3, G=512, J=5, wavelet="bior4.4", K=1_000_000, views=8, W=1920, H=1080, tile=16,
              loss="l1_dssim", desc="512^3 turbulence (E(k)~k^-5/3, kmax 64), bior4.4 J=5, top-1M Gaussians, "
                                    "8 orbit views 1920x1080, loss 0.8 L1 + 0.2 D-SSIM, Adam"),
    "c1": dict(config=1, G=128, J=3, wavelet="haar", K=100_000, views=16, W=800, H=800, tile=16, loss="l1",
               desc="128^3 blobs + k^-2 noise, Haar J=3, top-100k Gaussians, 16 orbit views 800x800, L1, Adam"),
    "c2": dict(config=2, G=256, J=4, wavelet="bior4.4", K=500_000, views=8, W=1024, H=1024, tile=16,
               loss="l1_dssim", desc="256^3 blobs + k^-2 noise, bior4.4 J=4, top-500k Gaussians, 8 orbit views "
                                     "1024x1024, loss 0.8 L1 + 0.2 D-SSIM, Adam"),
}
# checkpoints (steps) of the --convergence ablation runs
CONVERGENCE_AT = (1, 10, 25, 50, 100, 200, 400, 800, 1000)


def workload_shape(wl) -> str:
    if "scenes" in wl:
        sc = wl["scenes"]
        return (f"{sum(x['K'] for x in sc)} Gaussians in {len(sc)} scenes, {wl['views_per_scene'] * len(sc)} views "
                + "/".join(f"{x['W']}x{x['H']}" for x in sc))
    return f"{wl['K']} Gaussians, {wl['W']}x{wl['H']}, {wl['views']} views"


def n_views_of(wl) -> int:
    return wl["views_per_scene"] * len(wl["scenes"]) if "scenes" in wl else wl["views"]


def workload_config(wl) -> dict:
    if "scenes" in wl:
        return {"gaussians": [x["K"] for x in wl["scenes"]], "views": [wl["views_per_scene"]] * len(wl["scenes"]),
                "width": [x["W"] for x in wl["scenes"]], "height": [x["H"] for x in wl["scenes"]]}
    return {"gaussians": wl["K"], "views": wl["views"], "width": wl["W"], "height": wl["H"]}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------- CPU oracle baseline

def host_cpu() -> dict:
    """The host's logical CPUs available to this process and the CPU model."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count()
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:  # pragma: no cover
        pass
    return dict(nproc=n, cpu_count=os.cpu_count(), model=model)


def cpu_baseline_worker(queue, go, workload: str, n_tiles: int, threads: int) -> None:
    """Times the CPU oracle's per-iteration work on a bounded sample of the same workload.  Waits for
    ``go`` before doing anything, so that none of its work overlaps the GPU measurements."""
    if not go.wait(timeout=3600):
        queue.put(dict(ok=False, error="never released"))
        return
    try:
        import torch
        torch.set_num_threads(threads)
        import vbm_inputs as vi
        from oracle import adam as oadam
        from oracle import bank as obank
        from oracle import binning, construct, dvr, dwt, loss, render, select
        from oracle import tf as otf

        wl = WORKLOADS[workload]
        t_init = time.perf_counter()
        vol = vi.volume_for_config(wl["config"])
        tfn = vi.transfer_function(wl["config"])
        rgba = otf.apply(vol, tfn.xs, tfn.rgba)
        coeffs = dwt.dwt3d_rgba(rgba, wl["J"], wl["wavelet"])
        del rgba
        kept = select.topk(coeffs.astype(np.float32), wl["K"])
        bank = obank.build_bank(wl["wavelet"], wl["J"])
        g = construct.construct(coeffs, kept, wl["G"], wl["J"], bank, s_mode="none")
        del coeffs
        gs = vi.GaussianSet(*(g[k].astype(np.float32) for k in ("means", "scales", "quats", "opacity", "rgb")))
        cams = vi.orbit_cameras(wl["views"], wl["W"], wl["H"])
        init_s = time.perf_counter() - t_init

        # (1) projection + binning of view 0, every Gaussian (scaled by the view count)
        t0 = time.perf_counter()
        batch = render.Batch(gs, [cams[0]], wl["tile"])
        t_bin = time.perf_counter() - t0
        # (2) FP64 projection forward + backward of view 0 (scaled by the view count)
        t0 = time.perf_counter()
        P = batch.leaf_params()
        m2d, con, op, rgb = batch.project_items(P)
        torch.autograd.backward([m2d, con, op, rgb], [torch.ones_like(m2d), torch.ones_like(con),
                                                      torch.ones_like(op), torch.ones_like(rgb)])
        t_proj = time.perf_counter() - t0
        # (3) compositing forward + backward of sampled tiles (scaled by tiles per step)
        cam = cams[0]
        TX, TY = -(-cam.width // wl["tile"]), -(-cam.height // wl["tile"])
        rng = np.random.default_rng(12345)
        sample = rng.choice(TX * TY, size=min(n_tiles, TX * TY), replace=False)
        m2d_d, con_d, op_d, rgb_d = (t.detach() for t in (m2d, con, op, rgb))
        ranges, items = batch.pairs["ranges"], batch.pairs["item"]
        t_comp = 0.0
        pairs_sampled = 0
        for gt in sample:
            ty, tx = divmod(int(gt), TX)
            xs, ys = render._tile_pixels(cam, wl["tile"], tx, ty)
            tgt, _ = dvr.render(vol, tfn.xs, tfn.rgba, cam, pixels=(xs, ys))      # supervision: not timed
            s, e = ranges[gt]
            it = torch.as_tensor(items[s:e])
            pairs_sampled += int(e - s)
            t0 = time.perf_counter()
            leaves = [t[it].clone().requires_grad_(True) for t in (m2d_d, con_d, op_d, rgb_d)]
            pix = torch.stack([torch.as_tensor(xs + 0.5, dtype=torch.float64),
                               torch.as_tensor(ys + 0.5, dtype=torch.float64)], 1)
            col, _, _, _, _ = render.composite_tile(pix, *leaves, torch.zeros(3, dtype=torch.float64))
            l1 = (col - torch.as_tensor(tgt.T)).abs().sum()
            if l1.requires_grad:          # empty tiles have nothing to differentiate
                l1.backward()
            t_comp += time.perf_counter() - t0
        # (4) loss with SSIM on one 256x256 crop (scaled by pixels per step)
        crop = np.random.default_rng(1).uniform(size=(3, 256, 256))
        t0 = time.perf_counter()
        loss.loss_and_grad([crop], [np.clip(crop + 0.05, 0, 1)], wl["loss"])
        t_loss = time.perf_counter() - t0
        # (5) Adam over all Gaussians
        raw = dict(means=gs.means.astype(np.float64), log_scales=np.log(gs.scales.astype(np.float64)),
                   quats=gs.quats.astype(np.float64), logit_opacity=np.zeros(gs.n), rgb=gs.rgb.astype(np.float64))
        zeros = {k: np.zeros_like(v) for k, v in raw.items()}
        t0 = time.perf_counter()
        oadam.step(raw, raw, zeros, {k: v.copy() for k, v in zeros.items()}, 1)
        t_adam = time.perf_counter() - t0
        n_views = wl["views"]
        tiles_total = n_views * TX * TY
        px_total = n_views * cam.width * cam.height
        sec = (n_views * (t_bin + t_proj) + t_comp * tiles_total / len(sample)
               + t_loss * px_total / (256 * 256) + t_adam)
        queue.put(dict(ok=True, sec_per_iter=sec, init_s=init_s, t_bin=t_bin, t_proj=t_proj, t_comp=t_comp,
                       tiles=len(sample), pairs_sampled=pairs_sampled, t_loss=t_loss, t_adam=t_adam,
                       threads=torch.get_num_threads()))
    except Exception as exc:  # pragma: no cover - reported in the JSON line
        import traceback
        queue.put(dict(ok=False, error=f"{exc!r}", tb=traceback.format_exc()[-2000:]))


# ----------------------------------------------------------------------------- GPU side

def traffic_from_profiles(kernel_src: str):
    """HBM traffic of one launch of the backward compositing kernel from committed rocprofv3 counter
    runs, as dict(bytes_per_launch, algorithmic_bytes, pairs) of the profiled launch, or None when
    absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "composite_bwd_H_counters.md")
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        if line.startswith("traffic_json:"):
            d = json.loads(line.split(":", 1)[1])
            if d.get("kernel_sha") == digest:
                return d
    return None


def run_gpu(args, wl):
    import torch

    import vbm_inputs as vi
    from paper_2601_09417_amd import _lib as L
    from paper_2601_09417_amd import api

    dev = torch.device("cuda:0")
    L.load()          # fails loudly when the HIP library is not built
    out = {}
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if "scenes" in wl:
        return run_gpu_scenes(args, wl, out, timed_step_runs)
    t0 = time.perf_counter()
    vol = vi.volume_for_config(wl["config"])
    tfn = vi.transfer_function(wl["config"])
    out["volume_gen_s"] = time.perf_counter() - t0
    vol_d = torch.from_numpy(vol).to(dev)
    del vol
    cams = vi.orbit_cameras(wl["views"], wl["W"], wl["H"])

    # initialisation (once per scene; not part of the iteration)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    coeffs = api.dwt3d(vol_d, wl["J"], wl["wavelet"], (tfn.xs, tfn.rgba))
    _, packed = api.bank_build(wl["wavelet"], wl["J"])
    P, _ = api.build_gaussians(coeffs, wl["G"], wl["J"], packed, wl["K"], s_mode="none")
    torch.cuda.synchronize()
    out["init_ms"] = (time.perf_counter() - t0) * 1e3
    # the supplement's adaptive per-subband selection on the same coefficients (an alternative to the
    # global top-K; once per scene): time of vbm_adaptive_select with HIP events, after one warm call
    api.adaptive_select(coeffs, wl["G"], wl["J"], wl["K"])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 3
    ev[0].record()
    for _ in range(reps):
        kept_a, _ = api.adaptive_select(coeffs, wl["G"], wl["J"], wl["K"])
    ev[1].record()
    torch.cuda.synchronize()
    ams = ev[0].elapsed_time(ev[1]) / reps
    M = wl["G"] ** 3
    out["adaptive_select"] = dict(ms=round(ams, 3), kept=int(kept_a.numel()), budget=wl["K"],
                                  algorithmic_gbs=round(ADAPTIVE_BYTES_PER_COEF * M / (ams * 1e-3) / 1e9, 1))
    del coeffs, kept_a
    targets = api.dvr_render(vol_d, (tfn.xs, tfn.rgba), cams)
    torch.cuda.synchronize()
    log(f"init {out['init_ms']:.1f} ms; targets ready")

    loss_kind = timed_step_runs(args, out, P, cams, targets, wl, None, None)
    if args.convergence > 0:
        out["convergence"] = run_convergence(args, wl, vol_d, tfn, cams, targets, loss_kind)
    if args.modes > 0:
        del targets
        out["modes"] = run_modes(args, wl, vol_d, loss_kind)
    return out


def run_modes(args, wl, vol_d, loss_kind):
    """Visual modes (Sec. 4.4): n transfer functions, each zero outside its own interval of the
    field's values, one Gaussian set per mode (the workload's K split evenly), every set fine-tuned
    against the DVR of its own radiance field from the same orbit cameras, all modes as the scenes
    of one batched step (one HIP graph).  Reports the step rate and PSNR over training of every
    mode rendered separately against its own DVR, and of all sets rendered concatenated against
    the DVR of the union of the transfer functions."""
    import torch

    import vbm_inputs as vi
    from paper_2601_09417_amd import api, trainer

    n, V, R = args.n_modes, args.mode_views, args.mode_size
    vol = vol_d.cpu().numpy()
    tfs = vi.mode_transfer_functions(vol, wl["config"], n)
    edges = vi.mode_intervals(vol, n)
    union = vi.union_transfer_function(tfs)
    del vol
    pairs = [(t.xs, t.rgba) for t in tfs]
    Kh = wl["K"] // n
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P, offs, _ = api.build_mode_sets(vol_d, pairs, wl["J"], wl["wavelet"], Kh, s_mode="none")
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    cams = vi.orbit_cameras(V, R, R)
    cams_all, view_scene = api.mode_views(cams, n)
    targets = api.dvr_render_modes(vol_d, pairs, cams)
    union_targets = api.dvr_render(vol_d, (union.xs, union.rgba), cams)
    torch.cuda.synchronize()
    log(f"modes: {n} sets of {Kh} Gaussians built in {build_ms:.1f} ms; {n} x {V} targets {R}x{R} ready")
    per = targets.numel() // n
    npx = 3 * R * R

    def psnr(img, tgt):
        vals = [10.0 * np.log10(1.0 / max(torch.mean((img[v * npx:(v + 1) * npx] - tgt[v * npx:(v + 1) * npx]) ** 2)
                                          .item(), 1e-12)) for v in range(tgt.numel() // npx)]
        return float(np.mean(vals))

    ft = trainer.FineTuner(P, cams_all, targets, offs, view_scene, loss=loss_kind, lam=0.2, tile=wl["tile"],
                           schedule="graph")
    at = [t for t in CONVERGENCE_AT if t <= args.modes]
    sep = {h: [] for h in range(n)}
    concat = []
    t_train = 0.0
    for t in range(1, args.modes + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ft.step()
        torch.cuda.synchronize()
        if t > 1:                  # the first step includes the graph capture
            t_train += time.perf_counter() - t0
        if t in at:
            for h in range(n):
                sep[h].append(round(psnr(ft.image[h * per:(h + 1) * per], targets[h * per:(h + 1) * per]), 3))
            # the parameters after t updates, all sets in one scene
            concat.append(round(psnr(trainer.render_images(ft.act, cams, tile=wl["tile"]), union_targets), 3))
            log(f"modes step {t}: separate " + " ".join(f"{sep[h][-1]:.2f}" for h in range(n)) +
                f" dB, concatenated {concat[-1]:.2f} dB")
        if t % 10 == 0:
            ft.check_capacity()
    pairs_end, replans = ft.pair_count(), ft.overflows
    del ft
    # reference point, not the paper's procedure: the same initial sets concatenated into one scene
    # and fine-tuned against the union's DVR directly
    fj = trainer.FineTuner(P, cams, union_targets, loss=loss_kind, lam=0.2, tile=wl["tile"], schedule="graph")
    joint = []
    for t in range(1, args.modes + 1):
        fj.step()
        if t in at:
            torch.cuda.synchronize()
            joint.append(round(psnr(fj.image, union_targets), 3))
        if t % 10 == 0:
            fj.check_capacity()
    log("modes joint (concatenated sets fitted to the union's DVR): " +
        ", ".join(f"{t}:{p:.2f}" for t, p in zip(at, joint)))
    del fj
    return dict(n_modes=n, intervals=[round(float(e), 5) for e in edges], gaussians_per_mode=Kh,
                views_per_mode=V, size=[R, R], build_ms=round(build_ms, 1),
                step_ms=round(1e3 * t_train / max(args.modes - 1, 1), 3), pairs_at_end=pairs_end, re_plans=replans,
                steps=at, psnr_db_separate=sep, psnr_db_concatenated=concat, psnr_db_joint=joint,
                note="separate: each mode's views against the DVR of its own transfer function (the image of "
                     "step t, i.e. after t - 1 updates); concatenated: all sets in one scene after t updates "
                     "against the DVR of the union of the transfer functions; joint: the initial sets "
                     "concatenated and fine-tuned against the union's DVR (a reference point)")


def timed_step_runs(args, out, P, cams, targets, wl, scene_offsets, view_scene):
    """Autotune (optional), the graph-captured batched step (the reported value), the compositing
    kernels' event times and counts on the eager batched step, and the plain schedule."""
    import torch

    from paper_2601_09417_amd import _lib as L
    from paper_2601_09417_amd import trainer

    dev = P.device
    lib = L.load()
    so, vs = scene_offsets, view_scene

    def timed(ft, steps, warmup):
        for _ in range(warmup):
            ft.step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t = time.perf_counter()
        e0.record()
        for _ in range(steps):
            ft.step()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        return wall, e0.elapsed_time(e1) / 1e3

    # schedule knobs: the autotuner times each (tile, radix digit) candidate on the eager batched
    # step before anything is captured or timed
    loss_kind = wl["loss"] if args.loss == "default" else args.loss
    ckw = {}       # per-size-class schedule, when the autotuner keeps one
    if args.tile == "auto":
        tune = trainer.autotune_schedule(P, cams, targets, so, vs, loss=loss_kind, lam=0.2)
        tile, bits, lds, lds_bwd = tune["tile"], tune["sort_bits"], tune["lds_batch"], tune["lds_batch_bwd"]
        out["autotune"] = [dict(tile=d["tile"], sort_bits=d["sort_bits"], lds_batch=d["lds_batch"],
                                lds_batch_bwd=d["lds_batch_bwd"], ms=round(d["ms"], 3)) for d in tune["table"]]
        log("autotune: " + ", ".join(f"tile {d['tile']}/{d['sort_bits']}b/lds{d['lds_batch']}/{d['lds_batch_bwd']} "
                                     f"{d['ms']:.2f} ms" for d in tune["table"])
            + f" -> tile {tile}, {bits}-bit digits, LDS batch {lds} forward / {lds_bwd} backward")
        if "per_class" in tune:
            pc = tune["per_class"]
            out["autotune_classes"] = dict(classes=pc["classes"], schedules=pc["schedules"], step_ms=round(pc["ms"], 3),
                                           single_schedule_step_ms=round(tune["single_ms"], 3),
                                           kept=tune["classes"] is not None,
                                           tables=[[dict(tile=d["tile"], sort_bits=d["sort_bits"],
                                                         lds_batch=d["lds_batch"], lds_batch_bwd=d["lds_batch_bwd"],
                                                         ms=round(d["ms"], 3))
                                                    for d in t] for t in tune["class_tables"]])
            log(f"autotune per size class: {pc['schedules']} -> step {pc['ms']:.2f} ms "
                f"({'kept' if tune['classes'] is not None else 'one schedule is faster'})")
        if tune["classes"] is not None:
            ckw = dict(classes=tune["classes"], class_schedules=tune["class_schedules"])
    else:
        tile, bits, lds, lds_bwd = int(args.tile), args.sort_bits, args.lds_batch, args.lds_batch_bwd
    out["tile"], out["sort_bits"], out["loss_kind"] = tile, bits, loss_kind
    out["lds_batch"], out["lds_batch_bwd"] = lds, lds_bwd
    out["class_schedules"] = ckw.get("class_schedules")

    # batched schedule, captured as a graph: the reported value
    ft = trainer.FineTuner(P, cams, targets, so, vs, loss=loss_kind, lam=0.2,
                           tile=tile, sort_bits=bits, lds_batch=lds, lds_batch_bwd=lds_bwd, schedule="graph", **ckw)
    wall, ev = timed(ft, args.steps, args.warmup)
    if ft.overflowed():
        raise RuntimeError("pair capacity overflow during the timed region")
    out["batched_wall_s"], out["batched_event_s"] = wall, ev
    out["pairs_per_step"] = ft.pair_count()
    out["loss"] = ft.loss()
    log(f"batched(graph): {args.steps / wall:.2f} it/s, pairs {out['pairs_per_step']}")
    del ft
    # spread: the same measurement repeated (fresh step runner from the same initial parameters, W
    # warm-up steps, K timed steps); not part of `value`
    reps = [args.steps / wall]
    for _ in range(max(args.repeats - 1, 0)):
        fr = trainer.FineTuner(P, cams, targets, so, vs, loss=loss_kind, lam=0.2,
                               tile=tile, sort_bits=bits, lds_batch=lds, lds_batch_bwd=lds_bwd, schedule="graph", **ckw)
        w2, _ = timed(fr, args.steps, args.warmup)
        if not fr.overflowed():
            reps.append(args.steps / w2)
        del fr
    out["repeats"] = reps

    # kernel-level timing of the compositing kernels on the eager batched schedule
    # (one launch per phase: with a per-class schedule the kernels are timed on the whole batch with
    # the best single schedule, since the library's profiling events bracket one launch)
    fb = trainer.FineTuner(P, cams, targets, so, vs, loss=loss_kind, lam=0.2,
                           tile=tile, sort_bits=bits, lds_batch=lds, lds_batch_bwd=lds_bwd, schedule="batched")
    for _ in range(args.warmup):
        fb.step()
    # one untimed step with the counting kernel variants (evaluations and contributions) ...
    counters = torch.zeros(4, dtype=torch.int64, device=dev)
    lib.vbm_profile_counters(counters.data_ptr())
    fb.step()
    lib.vbm_profile_counters(None)
    # ... then K steps of the timing variants, each compositing launch bracketed by HIP events
    evs = []
    torch.cuda.synchronize()
    for i in range(args.steps):
        quad = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        for e in quad:
            e.record()  # creates the underlying event
        lib.vbm_profile_events(*[e.cuda_event for e in quad])
        fb.step()
        evs.append(quad)
    lib.vbm_profile_events(None, None, None, None)
    torch.cuda.synchronize()
    fwd_ms = float(np.mean([q[0].elapsed_time(q[1]) for q in evs]))
    bwd_ms = float(np.mean([q[2].elapsed_time(q[3]) for q in evs]))
    c = counters.cpu().numpy().astype(np.float64)
    npx = sum(cc.width * cc.height for cc in cams)
    P_pairs = out["pairs_per_step"]
    out["kernels"] = {
        "composite_fwd": dict(ms=fwd_ms, evals=c[0], contrib=c[1],
                              tflops=(FLOPS_FWD_EVAL * c[0] + FLOPS_FWD_USED * c[1]) / (fwd_ms * 1e-3) / 1e12,
                              bytes=BYTES_PER_PAIR_FWD * P_pairs + BYTES_PER_PIXEL_FWD * npx),
        "composite_bwd": dict(ms=bwd_ms, evals=c[2], contrib=c[3],
                              tflops=(FLOPS_BWD_EVAL * c[2] + FLOPS_BWD_USED * c[3]) / (bwd_ms * 1e-3) / 1e12,
                              bytes=BYTES_PER_PAIR_BWD * P_pairs + BYTES_PER_PIXEL_BWD * npx),
    }
    for d in out["kernels"].values():
        d["gbs"] = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    out["pixels_per_step"] = npx
    log(f"composite fwd {fwd_ms:.2f} ms, bwd {bwd_ms:.2f} ms per launch")
    del fb

    # plain schedule: one view per launch, one host sync per view forward
    if not args.skip_plain:
        fp = trainer.FineTuner(P, cams, targets, so, vs, loss=loss_kind, lam=0.2,
                               tile=tile, sort_bits=bits, lds_batch=lds, lds_batch_bwd=lds_bwd, schedule="plain")
        wall_p, _ = timed(fp, args.steps, args.warmup)
        out["plain_wall_s"] = wall_p
        log(f"plain: {args.steps / wall_p:.2f} it/s")
        del fp

    return loss_kind


def run_gpu_scenes(args, wl, out, step_runs):
    """The uneven multi-scene batch: every scene's volume, DWT and top-K build written into one
    parameter buffer, each scene seen by its own orbit views at its own resolution, DVR targets per
    view, all views in one batch."""
    import torch

    import vbm_inputs as vi
    from paper_2601_09417_amd import api

    if args.convergence or args.modes:
        raise SystemExit("--convergence and --modes take a single-scene workload")
    dev = torch.device("cuda:0")
    tfn = vi.transfer_function(wl["config"])
    Ks = [sc["K"] for sc in wl["scenes"]]
    so = np.concatenate([[0], np.cumsum(Ks)]).astype(np.int64)
    P = torch.zeros(api.N_ROWS, int(so[-1]), dtype=torch.float32, device=dev)
    cams, view_scene, targets = [], [], []
    init_ms = 0.0
    for s_, sc in enumerate(wl["scenes"]):
        vol_d = torch.from_numpy(vi.scene_volume(wl["config"], s_, sc["G"])).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        coeffs = api.dwt3d(vol_d, sc["J"], wl["wavelet"], (tfn.xs, tfn.rgba))
        _, packed = api.bank_build(wl["wavelet"], sc["J"])
        api.build_gaussians(coeffs, sc["G"], sc["J"], packed, sc["K"], s_mode="none", out=P, offset=int(so[s_]))
        torch.cuda.synchronize()
        init_ms += (time.perf_counter() - t0) * 1e3
        del coeffs
        c = vi.orbit_cameras(wl["views_per_scene"], sc["W"], sc["H"], azimuth0=0.4 * s_)
        targets.append(api.dvr_render(vol_d, (tfn.xs, tfn.rgba), c))
        cams += c
        view_scene += [s_] * len(c)
        del vol_d
    targets = torch.cat(targets)
    torch.cuda.synchronize()
    out["init_ms"] = init_ms
    log(f"init {init_ms:.1f} ms for {len(Ks)} scenes; targets ready")
    step_runs(args, out, P, cams, targets, wl, so, view_scene)
    return out


def run_convergence(args, wl, vol_d, tfn, cams, targets, loss_kind):
    """PSNR against the DVR targets over training for the method and its ablation variants (Sec. 5):
    without the transition bank's covariances, without the energy projection, with Haar instead of
    bior4.4, and from random parameters.  The PSNR after checkpoint step t is that of the image
    rendered in step t (the parameters after t - 1 updates), averaged over the views."""
    import torch

    import vbm_inputs as vi
    from paper_2601_09417_amd import api, trainer

    dev = vol_d.device
    npx = [c.width * c.height for c in cams]
    offs = np.concatenate([[0], np.cumsum(npx)]) * 3

    def psnr(img):
        vals = []
        for v in range(len(cams)):
            mse = torch.mean((img[offs[v]:offs[v + 1]] - targets[offs[v]:offs[v + 1]]) ** 2).item()
            vals.append(10.0 * np.log10(1.0 / max(mse, 1e-12)))
        return float(np.mean(vals))

    def built(wavelet, **flags):
        coeffs = api.dwt3d(vol_d, wl["J"], wavelet, (tfn.xs, tfn.rgba))
        _, packed = api.bank_build(wavelet, wl["J"])
        P, _ = api.build_gaussians(coeffs, wl["G"], wl["J"], packed, wl["K"], s_mode="none", **flags)
        return P

    variants = {"vbm": lambda: built(wl["wavelet"]),
                "no_transition_bank": lambda: built(wl["wavelet"], isotropic=True),
                "no_energy_projection": lambda: built(wl["wavelet"], unit_weight=True),
                "haar": lambda: built("haar")}
    # random initialisation: seeded uniform centres in the volume, isotropic log-normal scales around
    # the method's mean extent, random rotations, opacity U(0.05, 0.5), colour U(0, 1)
    sigma = float(built(wl["wavelet"], isotropic=True)[3, 0].item())
    rnd = vi.random_gaussians(wl["K"], 7 + wl["config"], extent=0.95, log_scale_mean=float(np.log(sigma)),
                              log_scale_std=0.3, opacity_range=(0.05, 0.5))
    variants["random_init"] = lambda: api.pack_params(rnd.means, rnd.scales, rnd.quats, rnd.opacity, rnd.rgb, dev)
    at = [t for t in CONVERGENCE_AT if t <= args.convergence]
    res = {}
    for name, make in variants.items():
        P = make()
        ft = trainer.FineTuner(P, cams, targets, loss=loss_kind, lam=0.2, tile=wl["tile"], schedule="graph")
        curve = []
        for t in range(1, args.convergence + 1):
            ft.step()
            if t in at:
                torch.cuda.synchronize()
                curve.append(round(psnr(ft.image), 3))
            if t % 10 == 0:
                ft.check_capacity()   # parameters move: re-plan when the pair lists outgrow the plan
        res[name] = curve
        log(f"convergence {name}: " + ", ".join(f"{t}:{p:.2f}" for t, p in zip(at, curve)) +
            f"  (pairs at the end {ft.pair_count()}, re-plans {ft.overflows})")
        del ft, P
    return dict(steps=at, psnr_db=res, workload=wl["desc"])


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="H", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", default="auto", choices=["auto", "8", "16", "32"],
                    help="tile edge; auto = pick (tile, radix digit) by timing each before the timed run")
    ap.add_argument("--sort-bits", type=int, default=8, choices=[4, 8],
                    help="radix digit width of the tile sort when --tile is fixed")
    ap.add_argument("--lds-batch", type=int, default=0, choices=[0, 32, 64],
                    help="forward compositing list entries staged in LDS per wave when --tile is fixed (8 and 16 only)")
    ap.add_argument("--lds-batch-bwd", type=int, default=0, choices=[0, 32, 64],
                    help="the same for the backward compositing")
    ap.add_argument("--loss", default="default", choices=["default", "l1", "l1_dssim"],
                    help="image loss; default = the workload's")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--cpu-tiles", type=int, default=256, help="tiles in the CPU oracle sample")
    ap.add_argument("--cpu-threads", type=int, default=0, help="threads of the CPU oracle (0 = every host CPU)")
    ap.add_argument("--convergence", type=int, default=0,
                    help="also train each ablation variant (Sec. 5) for this many steps and report PSNR")
    ap.add_argument("--modes", type=int, default=0,
                    help="also fine-tune the visual-mode sets (Sec. 4.4) together for this many steps and report PSNR")
    ap.add_argument("--n-modes", type=int, default=5, help="transfer functions (visual modes) per volume")
    ap.add_argument("--mode-views", type=int, default=64, help="supervision views per mode")
    ap.add_argument("--mode-size", type=int, default=512, help="edge of the square mode views")
    ap.add_argument("--repeats", type=int, default=5,
                    help="times the graph measurement is made in all, each from the initial parameters (the "
                         "first gives `value`; all give the spread)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (scales HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs the fine-tuning path on one GPU only; multi-GPU sharding is a design note, "
              "not a measured configuration (use --gpus 1).", file=sys.stderr)
        return 2
    wl = WORKLOADS[args.workload]
    rank0 = int(os.environ.get("RANK", "0")) == 0

    # start the CPU oracle before anything touches the GPU in this process; it waits until every GPU
    # measurement (autotune, graph, kernel events, plain) has finished
    proc = queue = go = None
    if rank0 and not args.no_cpu_baseline and "scenes" not in wl:
        ctx = mp.get_context("spawn")
        queue = ctx.Queue()
        go = ctx.Event()
        threads = args.cpu_threads or host_cpu()["nproc"]
        proc = ctx.Process(target=cpu_baseline_worker,
                           args=(queue, go, args.workload, args.cpu_tiles, threads), daemon=True)
        proc.start()
        log(f"CPU oracle baseline process started (pid {proc.pid}); it runs after the GPU measurements")

    gpu = run_gpu(args, wl)

    cpu = None
    if proc is not None:
        go.set()
        log("GPU measurements done; running the CPU oracle baseline")
        try:
            cpu = queue.get(timeout=900)
        except Exception as exc:
            cpu = dict(ok=False, error=f"no result: {exc!r}")
        proc.join(timeout=30)

    value = args.steps / gpu["batched_wall_s"]
    plain = args.steps / gpu["plain_wall_s"] if "plain_wall_s" in gpu else None
    k = gpu["kernels"]["composite_bwd"]
    kf = gpu["kernels"]["composite_fwd"]
    # the committed counter run covers the 16x16-tile kernel of the workload's own loss only
    traffic = (traffic_from_profiles(os.path.join(ROOT, "paper_2601_09417_amd", "csrc", "raster.hip"))
               if args.workload == "H" and gpu["tile"] == 16 and gpu["lds_batch_bwd"] == 0
               and gpu["loss_kind"] == wl["loss"] else None)
    result = {
        "metric": (METRIC if args.workload == "H" else
                   "fine-tune iters/sec (fwd+bwd, " + workload_shape(wl) + ") batched vs plain"),
        "value": round(value, 4),
        "unit": "iters/sec",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 / value, 3),
        "views_per_sec": round(value * n_views_of(wl), 2),
        "repeat_windows": {"n": len(gpu["repeats"]), "median": round(float(np.median(gpu["repeats"])), 3),
                           "min": round(min(gpu["repeats"]), 3), "max": round(max(gpu["repeats"]), 3)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}", **workload_config(wl), "tile": gpu["tile"],
                   "sort_bits": gpu["sort_bits"], "lds_batch": gpu["lds_batch"],
                   "lds_batch_bwd": gpu["lds_batch_bwd"], "loss": gpu["loss_kind"],
                   "schedule": ("batched per size class " + str(gpu["class_schedules"]) if gpu.get("class_schedules")
                                else "batched") + ", HIP graph"},
        "autotune": gpu.get("autotune"),
        "autotune_classes": gpu.get("autotune_classes"),
        "plain_value": None if plain is None else round(plain, 4),
        "batched_over_plain": None if plain is None else round(value / plain, 3),
        "pairs_per_step": gpu["pairs_per_step"],
        "pixels_per_step": gpu["pixels_per_step"],
        "init_ms": round(gpu["init_ms"], 2),
        "adaptive_select": gpu.get("adaptive_select"),
        "convergence": gpu.get("convergence"),
        "modes": gpu.get("modes"),
        "kernels_ms": {n: round(d["ms"], 3) for n, d in gpu["kernels"].items()},
        "composite_evals": {n: [int(d["evals"]), int(d["contrib"])] for n, d in gpu["kernels"].items()},
        "roofline": {
            "bound": "alu",
            "kernel": "composite_bwd",
            "achieved": round(k["tflops"], 3),
            "peak": FP32_ALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(k["tflops"] / FP32_ALU_PEAK_TFLOPS, 4),
            # measured on the profiled launch (its own pair count), not re-measured here
            "traffic": None if traffic is None else traffic["bytes_per_launch"],
            "traffic_over_algorithmic": (None if traffic is None else
                                         round(traffic["bytes_per_launch"] / traffic["algorithmic_bytes"], 3)),
            "traffic_pairs": None if traffic is None else traffic["pairs"],
            "peak_published_packed": FP32_PUBLISHED_PACKED_TFLOPS,
            "frac_of_published_packed": round(k["tflops"] / FP32_PUBLISHED_PACKED_TFLOPS, 4),
            "hbm": {name: {"algorithmic_bytes": int(d["bytes"]), "ms": round(d["ms"], 4),
                           "gbs": round(d["gbs"], 1), "frac": round(d["gbs"] / HBM_PEAK_GBS, 4)}
                    for name, d in (("composite_fwd", kf), ("composite_bwd", k))},
        },
    }
    if cpu is not None and cpu.get("ok"):
        hc = host_cpu()
        result["cpu_baseline"] = {
            "value": round(1.0 / cpu["sec_per_iter"], 6), "unit": "iters/sec", "cores": cpu["threads"],
            "kind": "oracle", "host_nproc": hc["nproc"], "host_cpu_count": hc["cpu_count"], "cpu_model": hc["model"],
            "ran": "after the GPU measurements, alone on the host",
            "sample": (f"FP64 oracle on the same workload: projection+binning and FP64 projection fwd/bwd of all "
                       f"{wl['K']} Gaussians for view 0 (x{wl['views']} views), compositing fwd+bwd of "
                       f"{cpu['tiles']} random tiles of view 0 ({cpu['pairs_sampled']} pairs; scaled to all tiles), "
                       f"loss on a 256x256 crop (scaled to all pixels), Adam on all Gaussians; "
                       f"oracle-built Gaussians, init {cpu['init_s']:.0f}s untimed"),
            "sec_per_iter": round(cpu["sec_per_iter"], 2),
        }
    elif cpu is not None:
        result["cpu_baseline"] = {"value": None, "error": cpu.get("error")}
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
