"""Volume reconstruction with the differentiable renderer.

The paper names recovering the impedance volume from B-modes as a use of the
gradient (Sec. 1, Sec. 4).  Here the volume is the parameter: each step runs
the batched fused step over all poses (forward, MSE to the pose's target,
adjoint to dL/dZ, replayed from a HIP graph), adds a smoothness prior
(``dus_smoothness``) and applies one Adam update on the device
(``dus_adam_step``), with the impedance kept in [lo, hi] (Eq. 1 needs Z > 0).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from .render import FusedStep, Geometry, adam_step, smoothness


@dataclass
class ReconstructionResult:
    Z: torch.Tensor               # reconstructed volume
    loss_history: np.ndarray      # [steps] data loss + prior
    steps_per_s: float
    ms_per_step: float


def reconstruct(Z0: torch.Tensor, geom: Geometry, poses: torch.Tensor, targets: torch.Tensor, steps: int = 100,
                lr: float = 1e-3, weight: float = 1e-4, lo: float = 0.5, hi: float = 12.0, betas=(0.9, 0.999),
                eps: float = 1e-8, graph: bool = True) -> ReconstructionResult:
    """Adam on the voxels of Z0 (a copy is optimised)."""
    dev = Z0.device
    Z = Z0.detach().clone().contiguous()
    step = FusedStep(geom, zero_grad_z=True, graph=graph)
    g = torch.zeros_like(Z)
    m = torch.zeros_like(Z)
    v = torch.zeros_like(Z)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    hist = torch.zeros(steps, dtype=torch.float64, device=dev)
    b1, b2 = betas
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        if it == 1:
            # the first step captured the graph: time the replays
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        step.step(Z, poses, targets, loss=loss, grad_Z=g)
        smoothness(Z, geom, weight, g, loss)
        hist[it] = loss[0]
        adam_step(Z, g, m, v, it + 1, lr, b1, b2, eps, lo, hi)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timed = max(1, steps - 1)
    step.close()
    return ReconstructionResult(Z, hist.cpu().numpy(), timed / dt, dt / timed * 1e3)


def main(argv=None) -> None:
    """Reconstruction benchmark: ``python -m paper_2508_06768_amd.reconstruction``
    renders targets from a synthetic brain-like volume at many poses, starts
    from that volume blurred (or with a smooth bump added), and prints one
    JSON line with the loss, the volume error on the footprint (or the bump)
    before and after, and steps/s."""
    import argparse
    import json
    import sys

    from scipy.ndimage import gaussian_filter

    from . import synth
    from .render import footprint_mask, render

    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128, help="voxels per axis (256 mm across)")
    ap.add_argument("--poses", type=int, default=64)
    ap.add_argument("--rays", type=int, default=256)
    ap.add_argument("--samples", type=int, default=512)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--weight", type=float, default=1e-5)
    ap.add_argument("--init", choices=["blur", "bump", "cube"], default="blur",
                    help="start from the volume blurred, with a Gaussian bump added inside the footprint, "
                         "or with a cube of the footprint scaled (sharp faces)")
    ap.add_argument("--init-sigma", type=float, default=2.0, help="blur of the starting volume (voxels)")
    ap.add_argument("--bump", type=float, default=0.05, help="bump amplitude (MRayl); radius 3 voxels")
    ap.add_argument("--cube", type=int, default=8, help="cube side (voxels) for --init cube")
    ap.add_argument("--cube-scale", type=float, default=1.05, help="impedance factor inside the cube")
    ap.add_argument("--refl", choices=["abs", "signed"], default="signed")
    ap.add_argument("--effects", action="store_true", help="speckle and blur in the renders")
    ap.add_argument("--seed", type=int, default=1007)
    args = ap.parse_args(argv)

    dev = torch.device("cuda:0")
    h = 256.0 / args.n
    print(f"reconstruction: building the {args.n}^3 volume", file=sys.stderr, flush=True)
    gt = synth.brain_volume(args.seed, args.n, h)
    rng = np.random.default_rng(args.seed)
    poses_np = synth.random_poses(rng, args.poses, (args.n - 1) * h)
    fans = [synth.FanSpec(args.rays, args.samples, 70 * synth.DEG, 200.0 / args.samples, 0.0, p)
            for p in range(args.poses)]
    phys = synth.PhysicsSpec(refl_mode=1 if args.refl == "signed" else 0, speckle_on=args.effects,
                             blur_on=args.effects, seed=args.seed)
    geom = Geometry(gt.shape, (h,) * 3, (0.0,) * 3, fans, phys)
    Zgt = torch.from_numpy(gt).to(dev)
    poses = torch.from_numpy(np.ascontiguousarray(poses_np, dtype=np.float32)).to(dev)
    targets = render(Zgt, poses, geom).clone()
    mask = footprint_mask(poses, geom).bool()
    if args.init == "blur":
        Z0 = torch.from_numpy(gaussian_filter(gt, args.init_sigma, mode="nearest").astype(np.float32)).to(dev)
        region = mask
    else:
        # the perturbation sits at the footprint voxel seen by the most poses
        cover = torch.zeros(gt.shape, dtype=torch.int32, device=dev)
        for p in range(args.poses):
            g1 = Geometry(gt.shape, (h,) * 3, (0.0,) * 3, [fans[p]], phys)
            cover += footprint_mask(poses[p:p + 1].contiguous(), g1).int()
        c = np.unravel_index(int(torch.argmax(cover).item()), gt.shape)
        iz, iy, ix = np.meshgrid(*[np.arange(k) for k in gt.shape], indexing="ij")
        if args.init == "bump":
            r2 = (iz - c[0]) ** 2 + (iy - c[1]) ** 2 + (ix - c[2]) ** 2
            bump = (args.bump * np.exp(-r2 / (2 * 3.0 ** 2))).astype(np.float32)
            Z0 = torch.from_numpy(gt + bump).to(dev)
            region = torch.from_numpy(bump > 0.1 * args.bump).to(dev)
        else:
            lo = [int(ci) - args.cube // 2 for ci in c]
            inside = ((iz >= lo[0]) & (iz < lo[0] + args.cube) & (iy >= lo[1]) & (iy < lo[1] + args.cube) &
                      (ix >= lo[2]) & (ix < lo[2] + args.cube))
            Z0 = torch.from_numpy(np.where(inside, gt * np.float32(args.cube_scale), gt).astype(np.float32)).to(dev)
            region = torch.from_numpy(inside).to(dev)

    def err(Z):
        # l2 error on the footprint (blurred start) or on the bump
        return float(torch.linalg.vector_norm((Z - Zgt)[region].double()))

    print("reconstruction: targets rendered, optimising", file=sys.stderr, flush=True)
    e0 = err(Z0)
    res = reconstruct(Z0, geom, poses, targets, steps=args.steps, lr=args.lr, weight=args.weight)
    e1 = err(res.Z)
    out = {
        "workload": f"{args.poses} poses x {args.rays} rays x {args.samples} samples, {args.n}^3 volume at "
                    f"{h:g} mm, {args.refl} reflection{', speckle + blur' if args.effects else ''}, start: "
                    + {"blur": f"the volume blurred by {args.init_sigma:g} voxels",
                       "bump": f"the volume plus a {args.bump:g} MRayl Gaussian bump (3 voxels) in the footprint",
                       "cube": f"the volume with a {args.cube}-voxel cube in the footprint scaled by "
                               f"{args.cube_scale:g}"}[args.init]
                    + f"; fused step + smoothness "
                    f"(weight {args.weight:g}) + Adam (lr {args.lr:g}), {args.steps} steps",
        "ray_samples_per_step": int(geom.total),
        "voxels": int(np.prod(gt.shape)),
        "footprint_voxels": int(mask.sum().item()),
        "steps_per_s": res.steps_per_s,
        "ms_per_step": res.ms_per_step,
        "loss_first": float(res.loss_history[0]),
        "loss_last": float(res.loss_history[-1]),
        "error_region": {"blur": "footprint", "bump": "bump", "cube": "cube"}[args.init],
        "error_region_voxels": int(region.sum().item()),
        "error_l2_first": e0,
        "error_l2_last": e1,
        "error_ratio": e1 / e0 if e0 > 0 else None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
