#!/usr/bin/env python3
"""Throughput of the fan-beam renderer on one MI355X.

Workload (one "step" = the whole hot path once): a batch of B probe poses
over the 256^3 (1 mm) brain-like impedance volume, each pose a 70 deg fan of
256 rays x 1024 samples (ds = 0.25 mm) with in-system attenuation, speckle
and depth-dependent blur; the step renders every pose, forms the MSE loss
against per-pose targets, and runs the hand-written adjoint to dL/dZ (full
volume, cleared every step) and dL/dpose -- one captured HIP graph per step
(the batched fused form).  Synthetic, seeded inputs.

Printed: one JSON line with ray-samples/s of that step, the same for the
plain per-pose form and the forward-only form, the uneven 64-pose batch
(128-512 rays x 256-2048 samples per pose) in its batched and plain forms,
a batch of very uneven ray lengths (63 fans of 256 x 256 samples and one of
64 x 16384) beside the same ray-samples spread evenly, the roofline of the dominant kernel (HIP events on the launch stream) and the
FP64 CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--poses B] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue roof: 256 CUs x 4 SIMDs, each issuing one wave64 instruction per
# 4 cycles (16 lanes per cycle), at the 2.4 GHz peak clock; FP64 and
# non-packed FP32 instructions issue at this rate alike
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "adjoint_hbm_traffic_64x256x1024.md")
VALU_FILE = os.path.join(ROOT, "profiles", "instruction_mix_64x256x1024.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2508_06768_amd", "csrc", "kernels.hip")
CALIB_BYTES = 512 << 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(fn, reps, stream_events):
    """Average ms of fn() over reps launches, HIP events on the current stream."""
    import torch
    start, stop = stream_events
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def profile_field(path, name):
    """A number recorded in a committed rocprofv3 counter summary, or None
    when the kernel source has changed since the counters were taken (each
    summary records the SHA-256 of the kernel source it measured)."""
    import hashlib
    try:
        text = open(path).read()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.lstrip().startswith("- `"):
            k, v = line.split(":", 1)
            fields[k.strip(" -`")] = v.strip(" `")
    if fields.get("kernel_source_sha256") != src:
        return None
    try:
        return float(fields[name])
    except (KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes per adjoint launch (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    return profile_field(TRAFFIC_FILE, "traffic_bytes_per_launch")


def cpu_baseline(case, budget_s: float):
    """FP64 oracle (forward + MSE + adjoint), pose after pose of the batch and
    round again, until budget_s seconds of work (whole poses only)."""
    from oracle import oracle as O
    from tests import helpers as H

    vol = H.oracle_volume(case)
    ph = H.oracle_physics(case.phys)
    gV = np.zeros_like(vol.Z)
    fans = [H.oracle_fan(f) for f in case.fans]
    t0 = time.perf_counter()
    done = 0
    samples = 0
    while True:
        p = done % len(fans)
        pose = case.poses[p].astype(np.float64)
        img = O.render(vol, pose, fans[p], ph)
        _, g = O.mse_loss_grad(img, np.zeros_like(img))     # the target does not change the cost
        O.backward(vol, pose, fans[p], ph, g, grad_volume=gV)   # dL/dZ added into gV in place
        done += 1
        samples += fans[p].n_rays * fans[p].n_samples
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    threads = O.num_threads()
    out = {"value": samples / dt, "unit": "ray-samples/s", "cores": threads, "kind": "oracle",
           "sample": f"{done} pose steps ({done / len(fans):.1f} passes over the {len(fans)} poses, 256x1024 "
                     f"each), FP64 forward + MSE + adjoint (dL/dZ and dL/dpose), {dt:.1f} s"}
    # the same oracle: forward only on all threads, forward + adjoint on one
    # thread (one pose each), and the literal O(S^2) progressive solve of
    # Sec. 2.4 on the 64^3 phantom's 64 x 256 fan, once
    t1 = time.perf_counter()
    nf = 0
    while nf < 4 or time.perf_counter() - t1 < 1.0:
        O.render(vol, case.poses[nf % len(fans)].astype(np.float64), fans[nf % len(fans)], ph)
        nf += 1
    out["forward_value"] = nf * fans[0].n_rays * fans[0].n_samples / (time.perf_counter() - t1)
    O.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        img = O.render(vol, case.poses[0].astype(np.float64), fans[0], ph)
        _, g = O.mse_loss_grad(img, np.zeros_like(img))
        O.backward(vol, case.poses[0].astype(np.float64), fans[0], ph, g)
        out["single_thread_value"] = fans[0].n_rays * fans[0].n_samples / (time.perf_counter() - t1)
    finally:
        O.set_num_threads(threads)
    from paper_2508_06768_amd import synth
    c1 = synth.case_small_forward()
    v1, f1, p1 = H.oracle_volume(c1), H.oracle_fan(c1.fans[0]), H.oracle_physics(c1.phys)
    for solver in ("transfer", "banded"):
        t1 = time.perf_counter()
        O.render(v1, c1.poses[0].astype(np.float64), f1, p1, solver=solver)
        out[f"phantom_64x256_forward_{solver}_s"] = time.perf_counter() - t1
    return out


def uneven_batch(Z, dev, reps: int, plain: bool, ev):
    """The uneven 64-pose batch (128-512 rays x 256-2048 samples, 40-90 deg,
    100-240 mm deep, speckle + blur) on the same volume: the fused step
    (forward + MSE + adjoint with dL/dZ and dL/dpose) and the forward alone,
    batched (one graph per step, one launch per kernel) and plain (one launch
    sequence per pose, no graph), with ray-samples/s and the algorithmic
    bytes as a share of the HBM peak."""
    import torch

    from paper_2508_06768_amd import synth
    from paper_2508_06768_amd.render import FusedStep, Geometry, footprint_voxels, render

    case = synth.case_batched()
    geom = Geometry(case.Z.shape, case.spacing, case.origin, case.fans, case.phys)
    poses = torch.from_numpy(case.poses).to(dev)
    target = render(Z, torch.from_numpy(case.extra["target_poses"]).to(dev), geom).clone()
    N = geom.total
    vfp = footprint_voxels(poses, geom)
    # forward: 4 B per pixel written + 4 B per footprint voxel read; step:
    # 4 B per pixel of target read + 4 B (volume) + 8 B (dL/dZ read-modify-
    # write) per footprint voxel
    fwd_bytes, step_bytes = 4.0 * N + 4.0 * vfp, 4.0 * N + 12.0 * vfp
    step = FusedStep(geom, zero_grad_z=True)
    gZ = torch.zeros_like(Z)
    gp = torch.empty((geom.n_poses, 6), device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    out = torch.empty(N, device=dev)
    ws_f = geom.workspace(False, dev)

    def rec(ms, nbytes):
        return {"ms": ms, "value": N / (ms * 1e-3), "pct_hbm": 100.0 * nbytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}

    fused = lambda: step.step(Z, poses, target, loss=loss, grad_Z=gZ, grad_pose=gp)  # noqa: E731
    fused()
    res = {"poses": geom.n_poses, "ray_samples_per_step": N, "footprint_voxels": vfp,
           "fused_batched": rec(timed(fused, reps, ev), step_bytes)}
    render(Z, poses, geom, out=out, ws=ws_f)
    res["forward_batched"] = rec(timed(lambda: render(Z, poses, geom, out=out, ws=ws_f), reps, ev), fwd_bytes)
    if plain:
        singles = []
        for p in range(geom.n_poses):
            g1 = Geometry(case.Z.shape, case.spacing, case.origin, [case.fans[p]], case.phys)
            o0, o1 = int(geom.offsets[p]), int(geom.offsets[p + 1])
            singles.append((FusedStep(g1, zero_grad_z=False, graph=False), poses[p:p + 1].contiguous(),
                            target[o0:o1], g1, out[o0:o1], g1.workspace(False, dev)))
        gp1 = torch.empty((1, 6), device=dev)

        def plain_step():
            gZ.zero_()
            for s1, p1, t1, *_ in singles:
                s1.step(Z, p1, t1, loss=loss, grad_Z=gZ, grad_pose=gp1)

        def plain_fwd():
            for _, p1, _, g1, o1, w1 in singles:
                render(Z, p1, g1, out=o1, ws=w1)

        plain_step()
        res["fused_plain"] = rec(timed(plain_step, max(2, reps // 4), ev), step_bytes)
        plain_fwd()
        res["forward_plain"] = rec(timed(plain_fwd, max(2, reps // 4), ev), fwd_bytes)
        for s1, *_ in singles:
            s1.close()
    step.close()
    return res


def skewed_batch(Z, dev, reps: int, ev):
    """A batch whose ray lengths are very uneven (63 fans of 256 x 256
    samples and one of 64 x 16384, speckle + blur) and the same ray-samples
    spread over 64 fans of 256 x 316: the fused step (graph), with the long
    rays walked by several wavefronts each (the default) and by one."""
    import torch

    from paper_2508_06768_amd import synth
    from paper_2508_06768_amd.render import FusedStep, Geometry, render

    res = {}
    for name, case, span in (("skewed", synth.case_skewed(), 0), ("skewed_one_wave_per_ray", synth.case_skewed(), -1),
                             ("even", synth.case_skewed(even=True), 0)):
        geom = Geometry(case.Z.shape, case.spacing, case.origin, case.fans, case.phys)
        poses = torch.from_numpy(case.poses).to(dev)
        target = render(Z, torch.from_numpy(case.extra["target_poses"]).to(dev), geom).clone()
        step = FusedStep(geom, zero_grad_z=True, schedule={"span_samples": span})
        gZ = torch.zeros_like(Z)
        gp = torch.empty((geom.n_poses, 6), device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        fused = lambda: step.step(Z, poses, target, loss=loss, grad_Z=gZ, grad_pose=gp)  # noqa: E731
        fused()
        ms = timed(fused, reps, ev)
        res[name] = {"ms": ms, "value": geom.total / (ms * 1e-3), "ray_samples_per_step": geom.total}
        step.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    # the GPU's clock climbs over the first tens of milliseconds of steady
    # work: about 100 steps (60 ms) of warm-up before the timed steps
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--poses", type=int, default=64)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--one-stream", action="store_true",
                    help="profiling runs: the timed step too on one stream (one launch per kernel and step)")
    ap.add_argument("--step-only", action="store_true",
                    help="skip the uneven and skewed batches (profiling runs: every launch at the step's "
                         "grid then belongs to the step)")
    ap.add_argument("--tune-cache", default="", help="reuse / store the tuned schedule in this JSON file")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also launch a plain device copy of 512 MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the renderer has no multi-GPU path "
              "(poses would shard across GPUs with no communication). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2508_06768_amd import synth
    from paper_2508_06768_amd.render import FusedStep, Geometry, footprint_voxels, render

    dev = torch.device("cuda:0")
    B = args.poses
    log(f"bench: building workload, {B} poses x 256 rays x 1024 samples on 256^3")
    case = synth.case_batched_c2(B=B)
    geom = Geometry(case.Z.shape, case.spacing, case.origin, case.fans, case.phys)
    Z = torch.from_numpy(case.Z).to(dev)
    poses = torch.from_numpy(case.poses).to(dev)
    tposes = torch.from_numpy(case.extra["target_poses"]).to(dev)
    target = render(Z, tposes, geom).clone()
    N = geom.total
    log("bench: targets rendered")

    step = FusedStep(geom, zero_grad_z=True, one_stream=args.one_stream)
    gZ = torch.zeros_like(Z)
    gp = torch.empty((B, 6), device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def fused():
        step.step(Z, poses, target, loss=loss, grad_Z=gZ, grad_pose=gp)

    tune = None
    if not args.no_tune:
        from paper_2508_06768_amd.autotune import autotune
        if args.tune_cache:
            os.environ["DUS_AUTOTUNE_CACHE"] = args.tune_cache
        tune = autotune(step, fused, reps=10, use_cache=bool(args.tune_cache))
        log(f"bench: autotuned schedule {tune['schedule']} ({tune['ms']:.3f} ms)")
    for _ in range(args.warmup):
        fused()
    torch.cuda.synchronize()
    log("bench: warmup done")
    t0 = time.perf_counter()
    ms = timed(fused, args.steps, ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = N / (ms * 1e-3)
    log(f"bench: fused batched step {ms:.3f} ms ({value:.3e} ray-samples/s)")

    # forward only, batched (render + blur)
    out = torch.empty(N, device=dev)
    ws_f = geom.workspace(False, dev)
    ms_fwd = timed(lambda: render(Z, poses, geom, out=out, ws=ws_f), max(5, args.steps), ev)
    log(f"bench: forward batched {ms_fwd:.3f} ms")

    # plain form: one launch sequence per pose, no graph
    plain_ms = plain_fwd_ms = None
    if not args.no_plain:
        singles = []
        for p in range(B):
            g1 = Geometry(case.Z.shape, case.spacing, case.origin, [case.fans[p]], case.phys)
            s1 = FusedStep(g1, zero_grad_z=False, graph=False)
            singles.append((s1, poses[p:p + 1].contiguous(), target[geom.offsets[p]:geom.offsets[p + 1]], g1,
                            out[geom.offsets[p]:geom.offsets[p + 1]], g1.workspace(False, dev)))
        gp1 = torch.empty((1, 6), device=dev)

        def plain_fwd():
            for _, p1, _, g1, o1, w1 in singles:
                render(Z, p1, g1, out=o1, ws=w1)

        plain_fwd()
        plain_fwd_ms = timed(plain_fwd, max(2, args.steps // 4), ev)
        log(f"bench: plain per-pose forward {plain_fwd_ms:.3f} ms")

        def plain():
            gZ.zero_()
            for s1, p1, t1, *_ in singles:
                s1.step(Z, p1, t1, loss=loss, grad_Z=gZ, grad_pose=gp1)

        plain()
        plain_ms = timed(plain, max(2, args.steps // 4), ev)
        log(f"bench: plain per-pose step {plain_ms:.3f} ms")

    # per-kernel durations: the step splits the fans into two chains of
    # launches on two streams, whose kernels overlap, so the kernels are
    # timed on the same workload in a plan held to one stream (one launch
    # per kernel over all 16384 rays), launched eagerly with HIP events at
    # the phase boundaries (on the launch stream).  Each timed step is queued
    # right behind a graph replay of that plan, so the GPU is busy when it
    # starts, as in the timed region, rather than idle after a host wait.
    step1 = FusedStep(geom, zero_grad_z=True, one_stream=True)
    step1.set_schedule(**step.get_schedule())
    fused1 = lambda: step1.step(Z, poses, target, loss=loss, grad_Z=gZ, grad_pose=gp)  # noqa: E731
    for _ in range(args.warmup):
        fused1()
    ms_one = timed(fused1, args.steps, ev)
    log(f"bench: fused batched step on one stream {ms_one:.3f} ms")
    reps = max(5, args.steps // 2)
    phases = None
    for _ in range(reps):
        fused1()
        ph_ms = step1.step_timed(Z, poses, target, loss=loss, grad_Z=gZ, grad_pose=gp)
        phases = ph_ms if phases is None else {k: phases[k] + v for k, v in ph_ms.items()}
    phases = {k: v / reps for k, v in phases.items()}
    log(f"bench: phases (ms) {json.dumps(phases)}")
    # the eager step pays a launch gap at every phase boundary that the graph
    # replay does not: each phase's kernel time is its eager time scaled by
    # (graph-replayed one-stream step / sum of the eager phases)
    gap_scale = ms_one / sum(phases.values())
    vfp = footprint_voxels(poses, geom)
    n_vox = int(np.prod(case.Z.shape))
    # algorithmic bytes per launch (per ray-sample figures times N, per
    # footprint voxel figures times V_fp): forward 4 N (pixels) + 4 V_fp
    # (volume); adjoint scan 4 N (dL/dI) + 4 V_fp (volume); scatter
    # 8 V_fp (gradient read-modify-write)
    alg = {"forward": 4.0 * N + 4.0 * vfp, "adjoint": 4.0 * N + 4.0 * vfp, "scatter": 8.0 * vfp}
    kern = {k: {"ms": phases[k] * gap_scale, "ms_eager": phases[k], "alg_bytes": alg[k],
                "GBs": alg[k] / (phases[k] * gap_scale * 1e-3) / 1e9}
            for k in ("forward", "adjoint", "scatter")}
    dom = max(kern, key=lambda k: kern[k]["ms"])
    log(f"bench: kernels {json.dumps(kern)} footprint voxels {vfp}")

    # display and ablation modes: sampling-only render of the whole batch,
    # scan conversion of one fan onto 512 x 512 pixels
    from paper_2508_06768_amd.render import sample_volume, scan_convert
    samp = torch.empty(N, device=dev)
    ms_samp = timed(lambda: sample_volume(Z, poses, geom, out=samp), 10, ev)
    render(Z, poses, geom, out=out, ws=ws_f)
    depth = case.fans[0].r0 + case.fans[0].n_samples * case.fans[0].ds
    half = depth * np.sin(case.fans[0].aperture / 2)
    ms_scan = timed(lambda: scan_convert(out, geom, 0, 512, 512, -half, 0.0, 2 * half / 511, depth / 511), 10, ev)
    modes = {"sampling_only": {"ms": ms_samp, "value": N / (ms_samp * 1e-3)},
             "scan_convert_512x512": {"ms": ms_scan}}
    log(f"bench: modes {json.dumps(modes)}")

    uneven = skewed = None
    if not args.step_only:
        log("bench: uneven 64-pose batch")
        uneven = uneven_batch(Z, dev, max(5, args.steps // 2), not args.no_plain, ev)
        log(f"bench: uneven batch {json.dumps(uneven)}")
        log("bench: skewed batch")
        skewed = skewed_batch(Z, dev, max(5, args.steps // 2), ev)
        log(f"bench: skewed batch {json.dumps(skewed)}")

    if args.calib_copy:
        src = torch.empty(CALIB_BYTES // 4, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {CALIB_BYTES} bytes done")

    cpu = None
    if not args.no_cpu:
        log("bench: timing the FP64 CPU oracle")
        cpu = cpu_baseline(case, args.cpu_budget)

    # roofline of the dominant kernel: algorithmic HBM bytes over its
    # event-timed duration (frac is on HBM), and the VALU issue roof from
    # the committed instruction counters (lane-operations = SQ_INSTS_VALU x
    # 64 per launch), which decide the bound while they match the source
    hbm_frac = kern[dom]["GBs"] / HBM_PEAK_GBS
    lane_ops = profile_field(VALU_FILE, f"valu_lane_ops_per_launch_{dom}")
    alu = None
    if lane_ops is not None:
        ach = lane_ops / (kern[dom]["ms"] * 1e-3)
        alu = {"achieved": ach, "peak": VALU_PEAK_LANE_OPS, "unit": "lane-op/s", "frac": ach / VALU_PEAK_LANE_OPS,
               "lane_ops_per_launch": lane_ops, "lane_ops_per_ray_sample": lane_ops / N}
    bound = "alu" if alu is None or alu["frac"] > hbm_frac else "hbm"
    # whole step: 4 B per pixel of target + 4 B (volume) + 8 B (dL/dZ
    # read-modify-write) per footprint voxel; the full clear of dL/dZ
    # (4 B per voxel) is reported beside it
    step_bytes = 4.0 * N + 12.0 * vfp

    res = {
        "metric": "ray-samples/s, batched fused forward+MSE+adjoint (256^3 vol, 256 rays x 1024 samples/pose)",
        "value": value,
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 volume, images and gradients; fp64 positions, samples and recurrence",
        "data": "synthetic",
        "config": {
            "workload": f"{B} poses x 256 rays x 1024 samples, 70 deg fans over a 256^3 1 mm brain-like "
                        "impedance volume, in-system attenuation, speckle + depth blur, fwd + MSE + adjoint "
                        "(dL/dZ full volume, dL/dpose), one HIP graph per step",
            "poses": B, "ray_samples_per_step": N, "footprint_voxels": vfp, "volume_voxels": n_vox,
        },
        "step_alg_bytes": step_bytes,
        "step_pct_hbm": 100.0 * step_bytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "step_pct_hbm_with_grad_clear": 100.0 * (step_bytes + 4.0 * n_vox) / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "forward_batched": {"ms": ms_fwd, "value": N / (ms_fwd * 1e-3)},
        "plain_per_pose": None if plain_ms is None else {"ms": plain_ms, "value": N / (plain_ms * 1e-3)},
        "plain_forward_per_pose": (None if plain_fwd_ms is None
                                   else {"ms": plain_fwd_ms, "value": N / (plain_fwd_ms * 1e-3)}),
        "modes": modes,
        "phases_ms": phases,
        "phase_gap_scale": gap_scale,
        "ms_per_step_one_stream": ms_one,
        "kernels": kern,
        "roofline": {
            "bound": bound,
            "kernel": dom,
            "achieved": kern[dom]["GBs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": hbm_frac,
            "frac_of": "hbm",
            "traffic": measured_traffic() if dom == "adjoint" else None,
            "alg_bytes": kern[dom]["alg_bytes"],
            "ms": kern[dom]["ms"],
            "alu": alu,
        },
        "uneven_batch": uneven,
        "skewed_batch": skewed,
        "schedule": step.get_schedule(),
        "autotune_trials": None if tune is None else tune.get("trials"),
        "cpu_baseline": cpu,
        "wall_s_timed": wall,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
