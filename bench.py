#!/usr/bin/env python3
"""Throughput of one training step of the Student's t rasterizer hot path.

A step = sss_project -> sss_bin_sort -> sss_render_fwd -> sss_render_bwd
(L1 loss against a target image, gradient fused into the backward) ->
sss_sghmc_step (SGHMC on the means, Adam on the other parameters), over one
batch of seeded synthetic input resident in HBM.

Default workload (the throughput metric's configuration): 1M components, SH
degree 3, one 1920x1080 camera on a ring of radius 4.

    python bench.py [--steps K] [--warmup W] [--mode stored|recompute]
                    [--workload m1|train|small|large] [--no-cpu-baseline]

Prints ONE JSON line.  Only one GPU is used: --gpus N with N > 1 exits.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd Mpix/s & HBM GB/s @1M comps 1080p; serving p50/p99 ms vs plain"

# VALU issue slots per (pixel, component) evaluation that the definition
# needs (FP32 ops counted 1, transcendentals 4): forward 28, backward 70.
SLOTS_FWD, SLOTS_BWD = 28, 70
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz FP32 lane-ops per second
# (no packed FP32), and 8 TB/s HBM3E.
PEAK_VALU = 256 * 4 * 16 * 2.4e9
PEAK_HBM = 8.0e12
PARAMS = ("means", "scales", "quats", "nu", "opacity", "sh")

WORKLOADS = {
    "m1": "1M components, SH degree 3, one 1920x1080 camera, fwd+bwd+SGHMC",
    "train": "300k components, SH degree 3, one 1297x840 camera, fwd+bwd+SGHMC",
    "small": "10k components, SH degree 0, one 256x256 camera, fwd+bwd+SGHMC",
    "large": "3M clustered components, nu 1..150, 30% negative, one 1920x1080 camera, fwd+bwd+SGHMC",
    "multiview": "5M clustered components, SH degree 3, 8 cameras of 1600x1064 in one launch per kernel "
                 "(recompute mode: per tile the forward walk and the backward in one launch, L1 loss fused), "
                 "fwd+bwd+SGHMC",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(workload):
    from paper_2503_10148_amd import scenes
    scene, cams = scenes.workload(workload)
    target = np.concatenate([scenes.smooth_target(c["width"], c["height"], seed=scenes.SEED_TARGET + v).reshape(-1, 3)
                             for v, c in enumerate(cams)])
    return scene, cams, target


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_frame(scene, cam, w, h):
    """Seconds of the FP64 oracle for one full-frame fwd+bwd, from the
    projection (+ its backward) of every component and the raster fwd+bwd of
    a central w x h window, scaled by pixel count (w, h are clamped to the
    frame; the full frame needs no scaling)."""
    import oracle
    from paper_2503_10148_amd import scenes
    W, H = cam["width"], cam["height"]
    w, h = min(w, W), min(h, H)
    x0, y0 = (W - w) // 2 // 16 * 16, (H - h) // 2 // 16 * 16
    win = oracle.window_camera(cam, x0, y0, w, h)
    target = scenes.smooth_target(W, H)[y0:y0 + h, x0:x0 + w]
    t0 = time.perf_counter()
    proj = oracle.project(scene, win)
    t1 = time.perf_counter()
    fwd = oracle.render(scene, win, proj=proj)
    t2 = time.perf_counter()
    g = oracle.l1_grad(fwd["image"], target)
    oracle.render_backward(scene, win, g, fwd=fwd)
    t3 = time.perf_counter()
    # the backward call includes the per-component projection backward;
    # count it with the projection, estimated as the forward projection time
    t_proj = (t1 - t0) * 2.0
    t_raster = (t2 - t1) + (t3 - t2) - (t1 - t0)
    return t_proj + max(t_raster, 0.0) * (W * H) / float(w * h), t3 - t0, (x0, y0, w, h)


def cpu_baseline(scene, cam, side_one=512):
    """The FP64 oracle, on all host threads over the whole frame and on one
    thread over a central side_one x side_one window (scaled to the frame):
    projection (+ its backward) of every component and the raster fwd+bwd."""
    import oracle
    W, H = cam["width"], cam["height"]
    threads = oracle.max_threads()
    t_all, wall_all, win_all = _oracle_frame(scene, cam, W, H)
    oracle.set_threads(1)
    try:
        t_one, wall_one, win_one = _oracle_frame(scene, cam, side_one, side_one)
    finally:
        oracle.set_threads(threads)
    n = scene["means"].shape[0]
    return {"value": round(W * H / t_all / 1e6, 6), "unit": "Mpix/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle, {threads} OpenMP threads: projection and its backward of all {n} components, "
                       f"raster fwd+bwd of the whole {W}x{H} frame; measured {wall_all:.1f} s"),
            "single_thread": {"value": round(W * H / t_one / 1e6, 6), "unit": "Mpix/s", "cores": 1,
                              "sample": (f"same, one thread, raster over a {win_one[2]}x{win_one[3]} window at "
                                         f"({win_one[0]},{win_one[1]}) scaled to the frame; measured {wall_one:.1f} s")},
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def serving(scene_np, rates, seconds, closed_clients=16):
    """Batched server vs plain one-request-per-launch on the resident 1M
    scene (SH 3): Poisson arrivals, cameras on a sphere of radius 3..5,
    resolution uniform over {640x360, 1280x720, 1920x1080}, batch <= 16."""
    import torch
    from paper_2503_10148_amd import scenes, serve, sss
    scene = sss.scene_to_device(scene_np)
    rng = np.random.default_rng(scenes.SEED_ARRIVALS)
    sizes = [(640, 360), (1280, 720), (1920, 1080)]
    res = {"workload": "resident scene of the bench workload; requests: camera direction uniform on the sphere, "
                       "radius U[3,5], resolution uniform over 640x360/1280x720/1920x1080; batch <= 16, "
                       "memory budget 6 GiB", "runs": []}
    # warm both paths (allocator, code objects)
    warm = [scenes.sphere_camera(rng, *sizes[i % 3]) for i in range(6)]
    serve.run_load("plain", scene, warm, [0.0] * 6)
    serve.run_load("batched", scene, warm, [0.0] * 6)
    torch.cuda.synchronize()
    for rate in rates:
        arr = serve.poisson_arrivals(rate, seconds, rng)
        cams = [scenes.sphere_camera(rng, *sizes[int(rng.integers(0, 3))]) for _ in arr]
        px = sum(c["width"] * c["height"] for c in cams)
        row = {"rate_req_s": rate, "requests": len(arr)}
        # both start warm: buffers sized for a burst of four of the largest
        # requests
        big = [scenes.sphere_camera(rng, *sizes[-1]) for _ in range(4)]
        for kind in ("plain", "batched"):
            lat, wall, stats = serve.run_load(kind, scene, cams, arr, warm=big)
            row[kind] = {"p50_ms": round(serve.percentile(lat, 50) * 1e3, 3),
                         "p99_ms": round(serve.percentile(lat, 99) * 1e3, 3),
                         "mpix_s": round(px / wall / 1e6, 2), **stats}
            log(f"serve rate {rate} {kind}: {row[kind]}")
        res["runs"].append(row)
    if closed_clients > 0:
        # saturation: closed loop of clients, each sending its next request
        # when the previous one returns
        crng = np.random.default_rng(scenes.SEED_ARRIVALS + 1)
        ccams = [scenes.sphere_camera(crng, *sizes[int(crng.integers(0, 3))]) for _ in range(100000)]
        big = [scenes.sphere_camera(crng, *sizes[-1]) for _ in range(4)]
        row = {"closed_loop_clients": closed_clients}
        for kind in ("plain", "batched"):
            lat, nreq, px, wall, stats = serve.run_closed(kind, scene, lambda k: ccams[k % len(ccams)],
                                                          closed_clients, seconds, warm=big)
            row[kind] = {"req_s": round(nreq / wall, 1), "mpix_s": round(px / wall / 1e6, 2),
                         "p50_ms": round(serve.percentile(lat, 50) * 1e3, 3),
                         "p99_ms": round(serve.percentile(lat, 99) * 1e3, 3), **stats}
            log(f"serve closed loop {closed_clients} clients {kind}: {row[kind]}")
        res["closed_loop"] = row
    return res


def kernel_source_hash():
    """sha256 of the sources the backward raster kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("raster.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2503_10148_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(open(os.path.join(ROOT, "include", "sss.h"), "rb").read())
    return h.hexdigest()


def measured_counters(workload):
    """The committed rocprofv3 counter summary of the render_bwd launch
    (HBM bytes = FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel
    calibration; SQ_INSTS_VALU per launch where taken); {} if there is none
    or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"render_bwd_{workload}_traffic.json")
    if not os.path.exists(path):
        return {}
    d = json.load(open(path))
    if d.get("source_sha256") != kernel_source_hash():
        return {}
    return d


def roofline(achieved, bwd_ms, evals, step_bytes, ms_step, ctr):
    """The dominant kernel (render_bwd) against the VALU model peak, with
    the counter cross-checks: its measured HBM bytes per launch, and the VALU
    issue rate its SQ_INSTS_VALU count gives at the live launch time (wave
    instructions x 64 lanes per second over the same peak); plus the whole
    step's algorithmic bytes over its time as a fraction of HBM peak."""
    out = {"bound": "alu", "kernel": "render_bwd", "achieved": round(achieved / 1e12, 3),
           "peak": round(PEAK_VALU / 1e12, 3), "unit": "Tops/s", "frac": round(achieved / PEAK_VALU, 4),
           "traffic": ctr.get("hbm_bytes_per_launch"), "avg_ms": round(bwd_ms, 4), "units": evals,
           "ops_per_unit": SLOTS_BWD,
           "basis": "frac: model estimate of 70 lane-ops per evaluation; valu_issue_frac: measured SQ_INSTS_VALU x 64 "
                    "per launch (committed counters) over the live launch time; step_hbm_frac: the whole step's "
                    "algorithmic bytes over its time",
           "step_hbm_frac": round(step_bytes / (ms_step * 1e-3) / PEAK_HBM, 4)}
    vi = ctr.get("valu_insts_per_launch")
    out["valu_issue_frac"] = round(vi * 64 / (bwd_ms * 1e-3) / PEAK_VALU, 4) if vi else None
    return out


def copy_probe():
    """A plain device copy of known size, for scaling the FETCH_SIZE /
    WRITE_SIZE counters (run under rocprofv3 --pmc), then the HBM rate of
    the runtime's copy and of the library's streaming copy (the rate the
    memory-bound stages are read against), each timed over 20 launches."""
    import torch
    from paper_2503_10148_amd import sss
    n = 1 << 28                                            # 1 GiB of float32
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    out = {"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}
    for name, fn in (("runtime_copy", lambda: b.copy_(a)), ("stream_copy", lambda: sss.stream_copy(a, b))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            fn()
        e1.record()
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 20
        out[name] = {"us_per_launch": round(us, 1), "tb_s_read_plus_write": round(8 * n / (us * 1e-6) / 1e12, 3)}
    if not torch.equal(a, b):
        raise RuntimeError("stream_copy did not copy")
    print(json.dumps(out))


def measure(sss, torch, workload, mode_name, deterministic, steps, warmup, instrument=True, fused=True):
    """Run warmup + timed (uninstrumented) training steps of a workload; with
    `instrument`, a few more steps with per-kernel HIP-event timing and the
    algorithmic work of the last step.  fused: the backward pass and the
    SGHMC/Adam step as one call (sss_render_bwd_step), else the two calls."""
    scene_np, cams, target_np = make_inputs(workload)
    n = scene_np["means"].shape[0]
    P = sss.total_pixels(cams)
    log(f"workload {workload}: n={n} pixels={P}")
    scene = sss.scene_to_device(scene_np)
    target = torch.as_tensor(target_np.reshape(-1, 3), device="cuda")
    mom = torch.zeros_like(scene["means"])
    grads = {k: torch.zeros_like(scene[k]) for k in PARAMS}
    adam_state = {k: (torch.zeros_like(scene[k]), torch.zeros_like(scene[k])) for k in PARAMS if k != "means"}
    bounds = dict(scales=(1e-4, 3.0e38), quats=(-3.0e38, 3.0e38), nu=(1.0, 1e4), opacity=(-1.0, 1.0),
                  sh=(-3.0e38, 3.0e38))
    lrs = dict(scales=1e-4, quats=1e-3, nu=1e-2, opacity=1e-3, sh=2.5e-4)
    # the bin sort reads its counts on the device and never waits (after the
    # first call, which sizes the pair buffers); every step's counts land in
    # its own row of step_counts and are checked against the capacity after
    # the timed loop.  The deterministic backward needs the host counts.
    binner = sss.BinSorter(0, keep_offsets=deterministic, no_wait=not deterministic)
    n_all = warmup + steps + max(1, min(steps, 5)) + 1
    step_counts = torch.zeros((n_all, 2), dtype=torch.int64, device="cuda")
    image = torch.empty((P, 3), device="cuda")
    t_final = torch.empty(P, device="cuda")
    n_contrib = torch.empty(P, dtype=torch.int32, device="cuda")
    loss = torch.zeros(1, device="cuda")
    bwd_ws = torch.empty(int(sss.lib().sss_render_bwd_workspace(n * len(cams), sss.total_tiles(cams))) // 4,
                         device="cuda")
    mode = sss.BWD_STORED if mode_name == "stored" else sss.BWD_RECOMPUTE
    state = {"proj": None, "bins": None}
    T = sss.total_tiles(cams)

    cams = sss.CameraBatch(cams)          # marshalled once for every call of every step
    adam_fused = dict(beta1=0.9, beta2=0.999, eps=1e-15, m={k: adam_state[k][0] for k in adam_state},
                      v={k: adam_state[k][1] for k in adam_state}, lr=lrs,
                      lo={k: bounds[k][0] for k in adam_state}, hi={k: bounds[k][1] for k in adam_state})

    def step(it):
        nonlocal bwd_ws
        proj = sss.project(scene, cams, out=state["proj"])
        state["proj"] = proj
        bins = binner(proj, cams, n, out=state["bins"], counts=step_counts[it])
        state["bins"] = bins
        if deterministic:
            need = int(sss.lib().sss_render_bwd_workspace_det(n * len(cams), bins.n_pairs, T))
            if bwd_ws.numel() * 4 < need:
                bwd_ws = torch.empty(int(need * 1.1) // 4 + 64, device="cuda")
        stored = mode == sss.BWD_STORED
        if stored:
            sss.render_fwd(bins, cams, image=image, t_final=t_final, n_contrib=n_contrib)
        if fused:
            adam_fused["t"] = it + 1
            sss.render_bwd_step(scene, proj, bins, cams, target, mom, dict(lr=1e-3, friction=0.1, seed=4, step=it),
                                adam=adam_fused, mode=mode, loss=sss.LOSS_L1, image=image if stored else None,
                                n_contrib=n_contrib if stored else None, image_out=None if stored else image,
                                loss_out=loss, ws=bwd_ws, deterministic=deterministic)
            return
        if stored:
            sss.render_bwd(scene, proj, bins, cams, target, mode=mode, loss=sss.LOSS_L1, image=image,
                           n_contrib=n_contrib, loss_out=loss, grads=grads, ws=bwd_ws, overwrite=True,
                           deterministic=deterministic)
        else:
            sss.render_bwd(scene, proj, bins, cams, target, mode=mode, loss=sss.LOSS_L1, image_out=image,
                           loss_out=loss, grads=grads, ws=bwd_ws, overwrite=True, deterministic=deterministic)
        adam = dict(beta1=0.9, beta2=0.999, eps=1e-15, t=it + 1,
                    arrays=[dict(param=scene[k], grad=grads[k], m=adam_state[k][0], v=adam_state[k][1], lr=lrs[k],
                                 lo=bounds[k][0], hi=bounds[k][1]) for k in adam_state])
        sss.sghmc_step(scene["means"], mom, grads["means"], scene["opacity"], lr=1e-3, friction=0.1, seed=4,
                       step=it, scales=scene["scales"], quats=scene["quats"], adam=adam)

    def check_counts(upto):
        """Every step so far had the pair capacity it needed."""
        c = step_counts[:upto].cpu()
        cap = state["bins"].pair_rank.numel()
        if int(c[:, 1].max()) > cap:
            raise RuntimeError(f"a step needed {int(c[:, 1].max())} pairs, more than the capacity {cap}")
        return c

    for it in range(warmup):
        step(it)
    torch.cuda.synchronize()
    check_counts(warmup)
    log(f"warmup done: pairs={int(step_counts[warmup - 1, 1])} visible={int(step_counts[warmup - 1, 0])}")

    # the timed steps run uninstrumented; the per-kernel breakdown comes from
    # a few further steps with HIP events around every launch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(warmup, warmup + steps):
        step(it)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    check_counts(warmup + steps)
    ms_step = (t1 - t0) * 1e3 / steps
    value = P * steps / (t1 - t0) / 1e6
    log(f"timed {steps} steps: {ms_step:.3f} ms/step, {value:.1f} Mpix/s")
    n_inst = max(1, min(steps, 5))
    if not instrument:
        torch.cuda.synchronize()
        return dict(ms_step=ms_step, value=value, P=P, n=n, views=len(cams), bins=state["bins"].resolve())
    sss.timing_enable(True)
    sss.timing_reset()
    torch.cuda.synchronize()
    ti0 = time.perf_counter()
    for it in range(warmup + steps, warmup + steps + n_inst):
        step(it)
    torch.cuda.synchronize()
    ti1 = time.perf_counter()
    kt = sss.timing_read()
    sss.timing_enable(False)
    check_counts(warmup + steps + n_inst)

    # algorithmic work of the last step
    if mode == sss.BWD_RECOMPUTE:
        sss.render_fwd(state["bins"], cams, image=image, t_final=t_final, n_contrib=n_contrib)
    torch.cuda.synchronize()
    evals = float(n_contrib.to(torch.float64).sum().item())
    bins = state["bins"].resolve()
    avg = {k: v[1] / v[0] for k, v in kt.items()}          # ms per launch
    per_step = {k: v[1] / n_inst for k, v in kt.items()}
    bwd_ms = avg.get("render_bwd", float("nan"))
    achieved = SLOTS_BWD * evals / (bwd_ms * 1e-3)
    # compulsory HBM bytes of the HBM-bound kernels (per launch)
    K = (scene_np["sh_degree"] + 1) ** 2
    par_b = 4 * (3 + 3 + 4 + 1 + 1 + 3 * K)
    V = len(cams)
    bytes_ = {
        # params in; 128 B entry line (104 B written), key and count out, per entry
        "project": n * V * (par_b + 104 + 8),
        # means, scales, quats, nu + per view touched and 80 B of FP64 screen gradients in;
        # means (read-modify-write), scales, quats, opacity, nu out
        "project_bwd": n * (4 * (3 + 3 + 4 + 1) + V * 84 + 4 * (3 + 3 + 3 + 4 + 1 + 1)),
        # means, SH, per view touched and 24 B FP64 colour gradient in; d_sh and d_means out
        "sh_bwd": n * (4 * (3 + 3 * K) + V * 28 + 4 * (3 * K + 3)),
        "sghmc": n * 64,
        "adam": n * (3 + 4 + 1 + 1 + 3 * K) * 28,               # one launch over the 5 arrays
    }
    if fused:
        # the gradients stay in registers: SH kernel reads means, SH, per
        # view touched and 24 B of colour gradient, and the SH moments;
        # writes SH, moments and the 12 B means partial.  Geometry kernel
        # reads means, scales, quats, nu, opacity, momentum, their moments,
        # the partial and per view touched + 64 B of screen gradients;
        # writes means, momentum, scales, quats, nu, opacity and moments.
        bytes_["sh_bwd"] = n * (4 * (3 + 3 * K * 3) + V * 28 + 4 * (3 * K * 3) + 12)
        bytes_["project_bwd"] = n * (4 * (3 + 3 + 4 + 1 + 1 + 3 + 2 * 9 + 3) + V * 68 + 4 * (3 + 3 + 3 + 4 + 1 + 1 + 2 * 9))
        del bytes_["sghmc"], bytes_["adam"]
    stages = {k: {"ms_per_step": round(per_step[k], 4), "launches_per_step": kt[k][0] / n_inst}
              for k in sorted(kt)}
    for k, b in bytes_.items():
        if k in avg:
            stages[k]["alg_gbps"] = round(b / (avg[k] * 1e-3) / 1e9, 1)
            stages[k]["hbm_frac"] = round(b / (avg[k] * 1e-3) / PEAK_HBM, 4)
    if "render_fwd" in avg:
        stages["render_fwd"]["valu_frac"] = round(SLOTS_FWD * evals / (avg["render_fwd"] * 1e-3) / PEAK_VALU, 4)
    step_bytes = (sum(bytes_.values())
                  # bin sort: keys and counts per entry; per visible entry its 104 B
                  # of entry line read, the 64 B record written, order and offset;
                  # 8 B per pair; per pixel image, t_final, n_contrib, target, loss
                  + 16 * n + 176 * bins.n_visible + 8 * bins.n_pairs + P * (12 + 12 + 4 + 12))

    return dict(ms_step=ms_step, value=value, evals=evals, bins=bins, stages=stages, kt=kt, P=P, n=n,
                bwd_ms=bwd_ms, achieved=achieved, step_bytes=step_bytes, ti0=ti0, ti1=ti1, n_inst=n_inst, loss=loss,
                views=len(cams), scene_np=scene_np, cams=cams)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--copy-probe", action="store_true", help="only run the counter calibration copy")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="m1", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="stored", choices=["stored", "recompute"])
    ap.add_argument("--other-workloads", default="large:recompute,multiview:recompute",
                    help="further workloads (name:mode, comma separated) timed for 5 steps each; '' to skip")
    ap.add_argument("--deterministic", action="store_true",
                    help="backward without float atomics (bit-identical gradients run to run)")
    ap.add_argument("--unfused", action="store_true",
                    help="backward and SGHMC/Adam step as two calls (gradients through memory)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-window", type=int, default=512, help="side of the one-thread oracle window")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="arrival window of each serving run (0 disables the serving measurement)")
    ap.add_argument("--serve-rates", default="200,500,1000,2000",
                    help="Poisson request rates (req/s) for the serving comparison")
    ap.add_argument("--serve-clients", type=int, default=16,
                    help="clients of the closed-loop serving run (0 disables it)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py measures a single GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_10148_amd import sss

    torch.cuda.set_device(0)
    r = measure(sss, torch, args.workload, args.mode, args.deterministic, args.steps, args.warmup,
                fused=not args.unfused)
    ms_step, value, evals, bins, stages, kt = r["ms_step"], r["value"], r["evals"], r["bins"], r["stages"], r["kt"]
    P, n, bwd_ms, achieved, step_bytes = r["P"], r["n"], r["bwd_ms"], r["achieved"], r["step_bytes"]
    ti0, ti1, n_inst, loss = r["ti0"], r["ti1"], r["n_inst"], r["loss"]
    scene_np, cams = r["scene_np"], r["cams"]
    del r
    others = {}
    for spec in [x for x in args.other_workloads.split(",") if x]:
        name, mode = spec.split(":")
        if name == args.workload:
            continue
        torch.cuda.empty_cache()
        o = measure(sss, torch, name, mode, False, 5, 1, instrument=False)
        others[name] = {"bwd_mode": mode, "ms_per_step": round(o["ms_step"], 3), "mpix_s": round(o["value"], 1),
                        "pixels_per_step": o["P"], "components": o["n"], "views": o["views"], "pairs": o["bins"].n_pairs,
                        "workload": WORKLOADS[name]}
        del o
        torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "components": n,
                   "pixels_per_step": P, "bwd_mode": args.mode,
                   "deterministic": args.deterministic, "loss": "L1", "pairs": bins.n_pairs,
                   "visible": bins.n_visible, "evaluations": evals},
        "hbm_gbps": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
        "roofline": roofline(achieved, bwd_ms, evals, step_bytes, ms_step, measured_counters(args.workload)),
        "stages": stages,
        "instrumented_ms_per_step": round((ti1 - ti0) * 1e3 / n_inst, 4),
        "other_workloads": others,
        "loss": float(loss.item()) / (args.warmup + args.steps + n_inst),
    }
    if args.serve_seconds > 0:
        out["serving"] = serving(scene_np, [float(r) for r in args.serve_rates.split(",") if r],
                                 args.serve_seconds, args.serve_clients)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(scene_np, cams[0], side_one=args.cpu_window)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
