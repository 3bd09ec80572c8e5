"""Slice-to-volume registration with the differentiable renderer.

The paper names registration of ultrasound to preoperative volumes as the
purpose of differentiability (abstract, Sec. 1, Sec. 4).  Here every pose of
a batch is optimised independently: one fused step (batched forward, MSE to
the pose's target image, pose-only adjoint, replayed from a HIP graph)
followed by an Adam update of the poses in place on the device.

Translation and rotation are updated with separate learning rates (mm and
rad per step).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from .render import FusedStep, Geometry


@dataclass
class RegistrationResult:
    poses: torch.Tensor           # [P, 6] final poses
    loss_history: np.ndarray      # [steps] summed loss
    steps_per_s: float
    ms_per_step: float


def rotation_matrix(w: np.ndarray) -> np.ndarray:
    """exp([w]x) for a batch of rotation vectors [P, 3] (evaluation only)."""
    w = np.asarray(w, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((w.shape[0], 3, 3))
    for i, v in enumerate(w):
        th = np.linalg.norm(v)
        K = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])
        if th < 1e-12:
            out[i] = np.eye(3) + K
        else:
            out[i] = np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K
    return out


def pose_errors(est: np.ndarray, gt: np.ndarray):
    """(translation error mm [P], geodesic rotation error deg [P])."""
    est = np.asarray(est, dtype=np.float64)
    gt = np.asarray(gt, dtype=np.float64)
    dt = np.linalg.norm(est[:, :3] - gt[:, :3], axis=1)
    Re, Rg = rotation_matrix(est[:, 3:]), rotation_matrix(gt[:, 3:])
    cos = (np.einsum("pij,pij->p", Re, Rg) - 1.0) / 2.0
    dr = np.degrees(np.arccos(np.clip(cos, -1.0, 1.0)))
    return dt, dr


def register(Z: torch.Tensor, geom: Geometry, targets: torch.Tensor, init_poses: torch.Tensor,
             steps: int = 200, lr_t: float = 0.5, lr_w: float = math.radians(0.5),
             betas=(0.9, 0.999), eps: float = 1e-8, graph: bool = True) -> RegistrationResult:
    """Adam on the 6-DOF poses; returns the final poses and the loss curve."""
    dev = Z.device
    poses = init_poses.detach().clone().contiguous().to(dev)
    step = FusedStep(geom, pose_only=True, zero_grad_z=False, graph=graph)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros_like(poses)
    m = torch.zeros_like(poses)
    v = torch.zeros_like(poses)
    lr = torch.tensor([lr_t] * 3 + [lr_w] * 3, dtype=torch.float32, device=dev)
    hist = torch.zeros(steps, dtype=torch.float64, device=dev)
    b1, b2 = betas
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        step.step(Z, poses, targets, loss=loss, grad_pose=g)
        hist[it] = loss[0]
        # Adam per pose component
        m.mul_(b1).add_(g, alpha=1 - b1)
        v.mul_(b2).addcmul_(g, g, value=1 - b2)
        mh = m / (1 - b1 ** (it + 1))
        vh = v / (1 - b2 ** (it + 1))
        poses.sub_(lr * mh / (vh.sqrt() + eps))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step.close()
    return RegistrationResult(poses, hist.cpu().numpy(), steps / dt, dt / steps * 1e3)
