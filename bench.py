#!/usr/bin/env python3
"""Throughput of the MI355X 2D-surfel renderer.

Headline: forward rays/s on the driving-scene camera workload (1920x1080
pinhole, f = 960, 1M surfels on a synthetic road corridor, degree-3 SH colour,
FP32), one step = one complete pass of the render path (pose composition,
projection and binning, depth sort, pair emission, tile sort, tile ranges,
compositing) over that frame with the inputs resident in HBM.

Also reported (in "extra"): forward+backward rays/s on the same frame (L1
loss gradient, adjoint compositing, per-surfel adjoint), the per-stage time
split, pair counts, and the algorithmic HBM bytes of a forward step; and, on
the other workloads:
  - neural-Gaussian training step (1280x720 camera, 50k anchors x 10): BF16
    MFMA decode -> render -> L1 loss -> adjoint render -> adjoint decode, with
    the decode's MFMA fraction;
  - LiDAR range image (128 x 1800, 200k anchors x 10 = 2M surfels): decode +
    render forward and forward+backward rays/s;
  - six-camera + LiDAR step (9.2M rays, 3.4M surfels per sensor): the batched
    path (BF16 MFMA decode, one record space, one persistent compositing
    launch, whole step replayed as one HIP graph) against the plain
    per-sensor FP32 path (FP32 VALU decode, one sensor at a time, no graph,
    16x16 tiles, no list splitting), ms per step forward and forward+backward.

roofline: the dominant kernel is the forward compositing kernel; it is bound
by plain FP32 ALU work, so "achieved" is its algorithmic FLOP per launch (the
counted ray-surfel evaluations times the per-pair FLOP of the solve, plus the
composited pairs times the per-pair FLOP of blending) over its average
duration, timed with HIP events around each stage on the render stream during
a second run of the same number of frames (the frame rate itself is timed
without the per-stage events, which cost the frame a few microseconds each).

cpu_baseline: the FP64 oracle on every 8th row and column of the same frame.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Non-packed FP32 VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz.
PEAK_ALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic FLOP per ray-surfel pair of the forward compositing kernel:
# evaluation (offsets, solve, rho, low-pass, exponent) and, for composited
# pairs, transmittance update, weight and 8-channel accumulation.
FLOP_EVAL = 33
FLOP_COMPOSITE = 20

BLEND_SOURCES = ("paper_2503_11731_amd/csrc/blend.hip", "paper_2503_11731_amd/csrc/gs_internal.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "blend_pinhole_1080p_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for p in BLEND_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per blend launch from committed rocprofv3 counters, if they match this source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash():
        return None
    return t.get("bytes_per_launch")


def forward_bytes(n, n_touch, pairs, rays, sh_coeffs):
    """Algorithmic HBM bytes of one forward step (inputs once, records, pairs, sorts, outputs)."""
    inputs = n * (12 + 16 + 8 + 4 + 4 * sh_coeffs)
    per_splat = n * (4 + 4 + 4 + 4 + 4) + n_touch * (64 + 32 + 16)  # keys, vals, tiles, visible + records
    depth_sort = 4 * n * 8 * 2                                       # 4 passes, read + write 8 B
    emit = pairs * 8
    tile_sort = 2 * pairs * 8 * 2
    gather = pairs * (4 + 64 + 32)                                   # surfel id + record per pair
    outputs = rays * (8 * 4 + 8)
    return inputs + per_splat + depth_sort + emit + tile_sort + gather + outputs


def cpu_baseline(scene, cam, stride):
    import torch

    from oracle import raster
    t0 = time.perf_counter()
    out = raster.render(scene, cam, raster.make_opts(), rays=("grid", stride))
    dt = time.perf_counter() - t0
    n = int(out["alpha"].size)
    return dict(value=n / dt, unit="rays/s", cores=int(torch.get_num_threads()), kind="oracle",
                sample=f"every {stride}th row and column of the 1920x1080 frame ({n} rays), FP64, "
                       f"{dt:.1f} s including per-surfel setup of all 1M surfels")


def _timed(fn, steps, warmup):
    """Mean ms per call of fn over `steps` calls after `warmup`, HIP events on the current stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _zero(dicts):
    for d in dicts:
        for v in d.values():
            v.zero_()


def _decode_flops(n_anchors, n_out):
    """Algorithmic FLOP of one decode: 2 A (35*32 + 32*out) (two dense layers)."""
    return 2.0 * n_anchors * (35 * 32 + 32 * n_out)


PEAK_BF16_TFLOPS = 2500.0


def bench_train720p(steps, warmup):
    """Decode (BF16 MFMA) -> render -> L1 -> adjoint render -> adjoint decode, 1280x720, 500k surfels."""
    import torch

    import paper_2503_11731_amd as gs
    from gen import scenes as S
    dev = torch.device("cuda:0")
    sc, sens = S.config3()
    cam = sens[0]
    dec = gs.Decoder.from_gen(sc, dev)
    tgt = gs.Decoder.from_gen(sc, dev, feat_bits=S.target_features(sc, 33))
    sp = gs.poses_tensor([cam["pose"]], dev)
    gp = gs.poses_tensor(sc.group_poses, dev)
    n = sc.n_anchors * sc.k
    offs = tuple(int(x) * sc.k for x in sc.group_offsets)
    r = gs.Renderer([gs.SceneShape(n, -1, False, offs)], [cam], opts=gs.PRODUCTION, device=dev)
    target = r.forward([tgt.forward(sp[0], gp)], sp, gp)[0][:3].clone()
    d = dec.new_decoded()
    outs = r.new_outputs()
    gsurf = [{k: torch.zeros_like(v) for k, v in d.items()}]
    ag = None
    g_out = torch.zeros_like(outs[0])
    rays = cam["width"] * cam["height"]

    def fwd():
        dec.forward(sp[0], gp, out=d)
        r.forward([d], sp, gp, outputs=outs)

    def step():
        nonlocal ag
        fwd()
        o = outs[0]
        g_out[:3] = torch.sign(o[:3] - target) / target.numel()
        _zero(gsurf)
        if ag is not None:
            _zero([ag])
        r.backward([d], sp, gp, outs, [g_out], grads=gsurf)
        ag = dec.backward(sp[0], gp, gsurf[0], grads=ag)

    fwd_ms = _timed(fwd, steps, warmup)
    step_ms = _timed(step, steps, warmup)
    dec_ms = _timed(lambda: dec.forward(sp[0], gp, out=d), steps, warmup)
    dflop = _decode_flops(sc.n_anchors, 100)
    st = r.status()
    return {"workload": "1280x720 pinhole f=640, 50k corridor anchors x 10 offsets = 500k surfels, camera MLP "
                        "35->32->100 (BF16 MFMA, FP32 accumulate), L1 loss vs a perturbed-feature target",
            "fwd_ms": fwd_ms, "fwd_rays_per_s": rays / (fwd_ms / 1e3),
            "train_step_ms": step_ms, "fwd_bwd_rays_per_s": rays / (step_ms / 1e3),
            "decode_ms": dec_ms, "decode_tflops": dflop / (dec_ms / 1e3) / 1e12,
            "decode_mfma_frac": dflop / (dec_ms / 1e3) / 1e12 / PEAK_BF16_TFLOPS,
            "pairs": st["pairs"][0], "segments": st["segments"],
            "grad_finite": bool(all(torch.isfinite(v).all() for v in ag.values()))}


def bench_lidar(steps, warmup):
    """128 x 1800 LiDAR, 200k anchors x 10 = 2M surfels: decode + render, forward and forward+backward."""
    import torch

    import paper_2503_11731_amd as gs
    from gen import scenes as S
    dev = torch.device("cuda:0")
    sc, sens = S.config4()
    lid = sens[0]
    dec = gs.Decoder.from_gen(sc, dev)
    tgt = gs.Decoder.from_gen(sc, dev, feat_bits=S.target_features(sc, 44))
    sp = gs.poses_tensor([lid["pose"]], dev)
    gp = gs.poses_tensor(sc.group_poses, dev)
    n = sc.n_anchors * sc.k
    offs = tuple(int(x) * sc.k for x in sc.group_offsets)
    r = gs.Renderer([gs.SceneShape(n, -1, True, offs)], [lid], opts=gs.PRODUCTION, device=dev)
    target = r.forward([tgt.forward(sp[0], gp)], sp, gp)[0][:2].clone()
    d = dec.new_decoded()
    outs = r.new_outputs()
    gsurf = [{k: torch.zeros_like(v) for k, v in d.items()}]
    ag = None
    g_out = torch.zeros_like(outs[0])
    rays = lid["width"] * lid["height"]
    z_far = 120.0

    def fwd():
        dec.forward(sp[0], gp, out=d)
        r.forward([d], sp, gp, outputs=outs)

    def step():
        nonlocal ag
        fwd()
        o = outs[0]
        g_out[0] = torch.sign(o[0] - target[0]) / (z_far * rays)
        g_out[1] = torch.sign(o[1] - target[1]) / rays
        _zero(gsurf)
        if ag is not None:
            _zero([ag])
        r.backward([d], sp, gp, outs, [g_out], grads=gsurf)
        ag = dec.backward(sp[0], gp, gsurf[0], grads=ag)

    fwd_ms = _timed(fwd, steps, warmup)
    step_ms = _timed(step, steps, warmup)
    st = r.status()
    return {"workload": "128-beam x 1800 spinning LiDAR (elevations uniform in [-25, 15] deg), 200k corridor "
                        "anchors x 10 = 2M surfels, LiDAR MLP 35->32->80; L1 on range / 120 m + intensity",
            "fwd_ms": fwd_ms, "fwd_rays_per_s": rays / (fwd_ms / 1e3),
            "fwd_bwd_ms": step_ms, "fwd_bwd_rays_per_s": rays / (step_ms / 1e3),
            "pairs": st["pairs"][0], "segments": st["segments"], "overflow": st["overflow"]}


def bench_affinity(steps, warmup):
    """Inpainting affinity (Eq. 6) at the three patch levels: row softmax of X_T X_S^T, bf16 MFMA."""
    import numpy as np
    import torch

    import paper_2503_11731_amd as gs
    from gen import patches as P
    dev = torch.device("cuda:0")
    res = {}
    for side, b, n in ((8.0, 32, 1024), (4.0, 128, 256), (2.0, 512, 64)):
        xt, xs = P.patch_pairs(seed=int(side), batch=b, p=n, q=n, side=side, d=64)
        t = torch.from_numpy(xt.view(np.int16).copy()).to(dev)
        s = torch.from_numpy(xs.view(np.int16).copy()).to(dev)
        out = torch.empty((b, n, n), dtype=torch.float32, device=dev)
        ms = _timed(lambda: gs.affinity(t, s, out=out), steps, warmup)
        nbytes = 4 * b * n * n + 2 * b * 2 * n * 64
        res[f"{int(side)}m"] = {"pairs": b, "anchors_per_patch": n, "d": 64, "ms": ms,
                               "algorithmic_bytes": nbytes, "gbs": nbytes / (ms / 1e3) / 1e9,
                               "hbm_frac": nbytes / (ms / 1e3) / (PEAK_HBM_GBS * 1e9)}
    return {"workload": "inpainting patch affinity, softmax over source anchors of X_T X_S^T (Eq. 6), "
                        "synthetic bf16 anchor rows (32 features + 16 positional-encoding terms, padded to 64)",
            "levels": res}


def bench_rig(steps, warmup):
    """Six cameras + LiDAR per step: batched graph path vs the plain per-sensor FP32 path."""
    import numpy as np
    import torch

    import paper_2503_11731_amd as gs
    from gen import scenes as S
    dev = torch.device("cuda:0")
    cam_sc, lid_sc, sensors = S.config5()
    n_s = len(sensors)
    rays = sum(s["width"] * s["height"] for s in sensors)
    k = cam_sc.k
    n = cam_sc.n_anchors * k
    offs = tuple(int(x) * k for x in cam_sc.group_offsets)
    sens = []
    for i, s in enumerate(sensors):
        s = dict(s)
        s["scene"] = i
        sens.append(s)
    shapes = [gs.SceneShape(n, -1, s["kind"] != "pinhole", offs) for s in sens]
    sp = gs.poses_tensor([s["pose"] for s in sens], dev)
    gp_c = gs.poses_tensor(cam_sc.group_poses, dev)
    gp_l = gs.poses_tensor(lid_sc.group_poses, dev)
    gp_all = torch.cat([gp_c] * (n_s - 1) + [gp_l]).contiguous()
    cap = 6 * n
    res = {"workload": "3 pinhole 1920x1080 (f=960) + 3 pinhole 1280x720 (f=640) + 128x1800 LiDAR; 300k corridor "
                       "anchors + 20 vehicle assets x 2k anchors, x 10 offsets = 3.4M surfels decoded per sensor",
           "rays_per_step": rays, "surfels_per_sensor": n}

    def build(batched, plain):
        dc = gs.Decoder.from_gen(cam_sc, dev, plain_fp32=plain)
        dl = gs.Decoder.from_gen(lid_sc, dev, plain_fp32=plain)
        ss = [dict(s) for s in sens]
        if plain:
            for s in ss:
                s["tile"] = (16, 16)
        r = gs.Renderer(shapes, ss, opts=gs.PRODUCTION, device=dev, batched=batched, pair_capacity=cap,
                        segment_pairs=-1 if plain else 0)
        ds = [(dc if s["kind"] == "pinhole" else dl).new_decoded() for s in sens]
        outs = r.new_outputs()

        def fwd():
            for i, s in enumerate(sens):
                if s["kind"] == "pinhole":
                    dc.forward(sp[i], gp_c, out=ds[i])
                else:
                    dl.forward(sp[i], gp_l, out=ds[i])
            r.forward(ds, sp, gp_all, outputs=outs)
        return dc, dl, r, ds, outs, fwd

    for label, batched, plain in (("plain_per_sensor_fp32", False, True), ("batched", True, False)):
        dc, dl, r, ds, outs, fwd = build(batched, plain)
        fwd()
        st = r.status()
        if st["overflow"]:
            raise RuntimeError(f"{label}: pair capacity overflow")
        entry = {"fwd_ms_eager": _timed(fwd, steps, warmup), "pairs": int(sum(st["pairs"])),
                 "segments": st["segments"]}
        if batched:
            stream = torch.cuda.Stream()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.stream(stream):
                fwd()
                stream.synchronize()
                with torch.cuda.graph(graph, stream=stream):
                    fwd()
            ref = [o.clone() for o in outs]
            entry["fwd_ms"] = _timed(graph.replay, steps, warmup)
            entry["graph_replay_matches_eager"] = bool(all(torch.equal(a, b) for a, b in zip(ref, outs)))
        else:
            entry["fwd_ms"] = entry["fwd_ms_eager"]
        targets = [torch.rand_like(o) for o in outs]
        gsurf = [{kk: torch.zeros_like(v) for kk, v in d.items()} for d in ds]
        g_outs = [torch.zeros_like(o) for o in outs]
        agc = [None]
        agl = [None]

        def step():
            if batched:
                graph.replay()
            else:
                fwd()
            for o, t, g in zip(outs, targets, g_outs):
                torch.sign(o - t, out=g)
            _zero(gsurf)
            r.backward(ds, sp, gp_all, outs, g_outs, grads=gsurf)
            for i, s in enumerate(sens):
                if s["kind"] == "pinhole":
                    agc[0] = dc.backward(sp[i], gp_c, gsurf[i], grads=agc[0])
                else:
                    agl[0] = dl.backward(sp[i], gp_l, gsurf[i], grads=agl[0])

        entry["fwd_bwd_ms"] = _timed(step, steps, warmup)
        entry["fwd_rays_per_s"] = rays / (entry["fwd_ms"] / 1e3)
        entry["fwd_bwd_rays_per_s"] = rays / (entry["fwd_bwd_ms"] / 1e3)
        res[label] = entry
        del r, ds, outs, gsurf, g_outs, targets
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    res["fwd_speedup_vs_plain"] = res["plain_per_sensor_fp32"]["fwd_ms"] / res["batched"]["fwd_ms"]
    res["fwd_bwd_speedup_vs_plain"] = res["plain_per_sensor_fp32"]["fwd_bwd_ms"] / res["batched"]["fwd_bwd_ms"]
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=8)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (HBM counter calibration under rocprofv3) and exit")
    ap.add_argument("--workloads", default="train720p,lidar,rig,affinity",
                    help="extra workloads to time (comma list of train720p, lidar, rig, affinity; empty for none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures a single MI355X: multi-GPU runs are not part of this build "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe > 0:
        # reads and writes exactly BYTES each: the reference for FETCH_SIZE / WRITE_SIZE scaling
        src = torch.ones(args.copy_probe, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "dispatches": 4}), flush=True)
        return

    import paper_2503_11731_amd as gs
    from gen import scenes as S

    dev = torch.device("cuda:0")
    log("generating the driving-scene workload (1M surfels, SH3)")
    sc, sensors = S.config2()
    cam = sensors[0]
    scene = dict(mean=sc.mean, quat=sc.quat, scale=sc.scale, opacity=sc.opacity, sh=sc.sh, sh_degree=3,
                 group_offsets=sc.group_offsets, group_poses=sc.group_poses)
    st = gs.scene_tensors(scene, dev)
    sp = gs.poses_tensor([cam["pose"]], dev)
    gp = gs.poses_tensor(sc.group_poses, dev)
    r = gs.Renderer([gs.SceneShape(sc.n, 3, False, (0, sc.n))], [cam], opts=gs.PRODUCTION, device=dev)
    rays = cam["width"] * cam["height"]
    outs = r.new_outputs()

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        r.forward([st], sp, gp, outputs=outs)
    status = r.status()
    if status["overflow"]:
        raise RuntimeError("pair capacity overflow")

    # The frame rate is timed without per-stage events (each event record
    # costs the frame a few microseconds); the same number of frames is then
    # run again with HIP events around every stage for the stage split and
    # the compositing kernel's average launch time.
    log(f"timed forward x{args.steps}")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        r.forward([st], sp, gp, outputs=outs)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1) / args.steps
    log(f"instrumented forward x{args.steps}")
    r.set_timing(8 * (args.steps + 2))
    e0.record()
    for _ in range(args.steps):
        r.forward([st], sp, gp, outputs=outs)
    e1.record()
    torch.cuda.synchronize()
    ms_instr = e0.elapsed_time(e1) / args.steps
    stages = r.stage_times(reset=True)
    r.set_timing(0)
    status = r.status()
    blend_ms, blend_n = stages["blend"]
    blend_s = blend_ms / max(blend_n, 1) / 1e3
    flop = status["evaluated"] * FLOP_EVAL + status["composited"] * FLOP_COMPOSITE
    achieved = flop / blend_s / 1e12
    value = rays / (ms / 1e3)

    line = {
        "metric": "rays/s fwd 2DGS raster (1920x1080 camera, 1M surfels, SH3)",
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "driving-scene camera forward: 1920x1080 pinhole f=960, 1M corridor surfels "
                               "(ground 60%, facades 30%, vehicles 10%), SH degree 3, production compositing",
                   "rays": rays, "surfels": sc.n, "frames_per_step": 1},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_ALU_TFLOPS, "traffic": measured_traffic(),
                     "kernel": "k_blend_queue<256, false, 1> (forward compositing, camera)", "avg_launch_ms": blend_s * 1e3},
    }
    extra = {"wall_s_timed": wall, "ms_per_step_with_stage_events": ms_instr,
             "stage_ms": {k: v[0] / max(v[1], 1) for k, v in stages.items() if v[1]},
             "pairs": status["pairs"][0], "evaluated_pairs": status["evaluated"],
             "composited_pairs": status["composited"], "fp64_pairs": status["fp64_pairs"],
             "visible": status["n_visible"][0]}
    n_touch = status["n_visible"][0]
    fb = forward_bytes(sc.n, n_touch, status["pairs"][0], rays, 48)
    extra["forward_algorithmic_bytes"] = fb
    extra["forward_hbm_frac"] = fb / (ms / 1e3) / (PEAK_HBM_GBS * 1e9)

    if not args.no_extras:
        log("timed forward+backward")
        target = torch.rand_like(outs[0])
        grads = [{k: torch.zeros_like(v) for k, v in st.items()}]
        for _ in range(2):
            o = r.forward([st], sp, gp, outputs=outs)
            g = torch.sign(o[0] - target) / o[0].numel()
            r.backward([st], sp, gp, o, [g], grads=grads)
        def fwd_bwd():
            o = r.forward([st], sp, gp, outputs=outs)
            g = torch.sign(o[0] - target) / o[0].numel()
            for d in grads:
                for v in d.values():
                    v.zero_()
            r.backward([st], sp, gp, o, [g], grads=grads)

        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            fwd_bwd()
        e1.record()
        torch.cuda.synchronize()
        fb_ms = e0.elapsed_time(e1) / args.steps
        r.set_timing(10 * (args.steps + 2))
        for _ in range(args.steps):
            fwd_bwd()
        torch.cuda.synchronize()
        st2 = r.stage_times(reset=True)
        r.set_timing(0)
        extra["fwd_bwd_rays_per_s"] = rays / (fb_ms / 1e3)
        extra["fwd_bwd_ms_per_step"] = fb_ms
        extra["fwd_bwd_stage_ms"] = {k: v[0] / max(v[1], 1) for k, v in st2.items() if v[1]}
        extra["grad_finite"] = bool(all(torch.isfinite(v).all() for v in grads[0].values()))

    if not args.no_extras:
        for w in [x for x in args.workloads.split(",") if x]:
            log(f"workload {w}")
            fn = {"train720p": bench_train720p, "lidar": bench_lidar, "rig": bench_rig, "affinity": bench_affinity}[w]
            extra[w] = fn(args.steps, args.warmup)

    if not args.no_cpu_baseline:
        log(f"cpu baseline (oracle, stride {args.cpu_stride})")
        line["cpu_baseline"] = cpu_baseline(scene, cam, args.cpu_stride)
    line["extra"] = extra
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
