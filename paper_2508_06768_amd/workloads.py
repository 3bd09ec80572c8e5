"""Timings of the renderer on its named workloads.

    python -m paper_2508_06768_amd.workloads

* ``fwd_64cube_64x256``: forward on the 64^3 phantom, one 64 x 256 fan;
* ``fwd_256cube_256x1024_effects``: forward with speckle and blur on the
  256^3 volume, one 256 x 1024 fan;
* ``fwdbwd_256cube_512x1024``: forward + MSE + adjoint (dL/dZ, dL/dpose) at
  512 x 1024;
* ``batched_256cube_64poses``: the uneven 64-pose batch, forward + MSE +
  adjoint, one launch sequence per pose against one graph-replayed step;
* ``skewed`` / ``skewed_even``: a batched step whose ray lengths are very
  uneven (63 fans of 256 x 256 and one of 64 x 16384 samples) against the
  same ray-samples spread evenly (64 fans of 256 x 316): the cost of rays
  that are each walked by one wavefront from end to end;
* ``table_R_rays_S_samples``: single renders at the shapes of the paper's
  timing tables (Sec. 3.4, Tables 2-3: 64-256 rays, 32-200 samples, one
  voxel per sample) on the 256^3 volume with speckle and blur;
* ``map_impedance_256cube``: the intensity -> impedance table over a 256^3
  volume (12 knots) and its adjoint; bytes = 4 B read + 4 B written per
  voxel forward, 8 B read + 4 B written adjoint.

Prints one JSON line per workload: ms per call, ray-samples/s, and the
algorithmic bytes as a share of the 8 TB/s HBM peak (forward: 4 B per
ray-sample written + 4 B per footprint voxel read; forward + MSE + adjoint:
4 B per ray-sample of target + 12 B per footprint voxel, the volume read and
the dL/dZ read-modify-write).  Inputs are the seeded synthetic volumes of
``synth``.
"""
from __future__ import annotations

import json
import sys

import numpy as np
import torch

from . import synth
from .render import FusedStep, Geometry, footprint_voxels, map_impedance, map_impedance_backward, render

HBM_PEAK = 8.0e12


def _timed(fn, reps: int) -> float:
    """Average ms of fn() over reps calls, HIP events on the current stream."""
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def _upload(case, dev):
    geom = Geometry(case.Z.shape, case.spacing, case.origin, case.fans, case.phys)
    Z = torch.from_numpy(case.Z).to(dev)
    P = torch.from_numpy(np.ascontiguousarray(case.poses, dtype=np.float32)).to(dev)
    return geom, Z, P


def _line(name, ms, n, alg_bytes, **extra):
    out = {"workload": name, "ms": ms, "ray_samples": int(n), "ray_samples_per_s": n / (ms * 1e-3),
           "alg_bytes": int(alg_bytes), "hbm_frac": alg_bytes / (ms * 1e-3) / HBM_PEAK}
    out.update(extra)
    print(json.dumps(out), flush=True)


def forward_only(case, dev, reps=50):
    geom, Z, P = _upload(case, dev)
    out = torch.empty(geom.total, device=dev)
    ws = geom.workspace(False, dev)
    ms = _timed(lambda: render(Z, P, geom, out=out, ws=ws), reps)
    vfp = footprint_voxels(P, geom)
    _line(case.name, ms, geom.total, 4 * geom.total + 4 * vfp, form="plain forward", footprint_voxels=vfp)


def fused(case, dev, per_pose: bool, reps=20):
    geom, Z, P = _upload(case, dev)
    T = render(Z, torch.from_numpy(np.ascontiguousarray(case.extra["target_poses"], dtype=np.float32)).to(dev),
               geom).clone()
    gZ = torch.zeros_like(Z)
    gp = torch.empty((geom.n_poses, 6), device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    vfp = footprint_voxels(P, geom)
    alg = 4 * geom.total + 12 * vfp
    if per_pose:
        singles = []
        for p in range(geom.n_poses):
            g1 = Geometry(case.Z.shape, case.spacing, case.origin, [case.fans[p]], case.phys)
            o0, o1 = int(geom.offsets[p]), int(geom.offsets[p + 1])
            singles.append((FusedStep(g1, zero_grad_z=False, graph=False), P[p:p + 1].contiguous(), T[o0:o1],
                            gp[p:p + 1]))

        def run():
            gZ.zero_()
            for s1, p1, t1, g1 in singles:
                s1.step(Z, p1, t1, loss=loss, grad_Z=gZ, grad_pose=g1)

        ms = _timed(run, max(2, reps // 4))
        _line(case.name, ms, geom.total, alg, form="plain: one launch sequence per pose", footprint_voxels=vfp)
    else:
        step = FusedStep(geom, zero_grad_z=True)
        ms = _timed(lambda: step.step(Z, P, T, loss=loss, grad_Z=gZ, grad_pose=gp), reps)
        _line(case.name, ms, geom.total, alg, form="batched: one graph-replayed step", footprint_voxels=vfp)
        step.close()


def table_shapes(dev, reps=50):
    Z = synth.brain256(1002)
    for S in (32, 70, 100, 200):
        for R in (64, 128, 256):
            fan = synth.FanSpec(R, S, 70 * synth.DEG, 1.0, 0.0, 0)
            case = synth.Case(f"table_{R}_rays_{S}_samples", Z, (1.0,) * 3, (0.0,) * 3,
                              synth.top_pose(256)[None, :], [fan], synth.effects_physics(1002))
            forward_only(case, dev, reps)


def mapping(dev, reps=50):
    n = 256 ** 3
    rng = np.random.default_rng(1008)
    xk = np.cumsum(rng.uniform(20.0, 200.0, 12)).astype(np.float32) - 500.0
    zk = rng.uniform(1.3, 7.8, 12).astype(np.float32)
    inten = torch.from_numpy(rng.uniform(float(xk[0]) - 50.0, float(xk[-1]) + 50.0, n).astype(np.float32)).to(dev)
    Z = torch.empty_like(inten)
    gZ = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(dev)
    for name, fn, nbytes in (("forward", lambda: map_impedance(inten, xk, zk, out=Z), 8 * n),
                             ("adjoint", lambda: map_impedance_backward(inten, xk, zk, gZ), 12 * n)):
        ms = _timed(fn, reps)
        print(json.dumps({"workload": "map_impedance_256cube", "form": name, "ms": ms, "voxels": n,
                          "voxels_per_s": n / (ms * 1e-3), "alg_bytes": nbytes,
                          "hbm_frac": nbytes / (ms * 1e-3) / HBM_PEAK}), flush=True)


def main(argv=None) -> None:
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--skip-table", action="store_true", help="leave out the paper-table shapes")
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    print("workloads: building inputs", file=sys.stderr, flush=True)
    forward_only(synth.case_small_forward(), dev)
    forward_only(synth.case_forward_effects(), dev)
    fused(synth.case_adjoint(), dev, per_pose=True)
    case = synth.case_batched()
    fused(case, dev, per_pose=True)
    fused(case, dev, per_pose=False)
    fused(synth.case_skewed(), dev, per_pose=False)
    fused(synth.case_skewed(even=True), dev, per_pose=False)
    mapping(dev)
    if not args.skip_table:
        table_shapes(dev)


if __name__ == "__main__":
    main()
