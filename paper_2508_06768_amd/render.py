"""PyTorch front end of the fan-beam renderer.

PyTorch provides device memory and streams; the renderer itself is the HIP
library behind the C ABI (``_lib``).  ``Geometry`` packs the volume shape,
the fans and the physics into the ABI's records once; ``render`` and
``RenderBmode`` (a ``torch.autograd.Function`` with the hand-written adjoint)
call the library on the current HIP stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import DusFan, DusPhysics, DusSchedule, DusVolume, check


def _stream() -> int:
    return int(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


@dataclass
class Geometry:
    """Volume shape + fans + physics as ABI records.

    fans: sequence of objects with n_rays, n_samples, aperture, ds, r0 and
    speckle_id attributes (``synth.FanSpec``).  Images of consecutive poses
    are packed back to back: pose p starts at ``offsets[p]``.
    """
    shape: tuple                      # (nz, ny, nx)
    spacing: tuple                    # (hx, hy, hz) mm
    origin: tuple                     # (ox, oy, oz) mm
    fans: list
    phys: object                      # synth.PhysicsSpec-like
    vol_c: DusVolume = field(init=False)
    fans_c: ctypes.Array = field(init=False)
    phys_c: DusPhysics = field(init=False)
    offsets: np.ndarray = field(init=False)
    total: int = field(init=False)

    def __post_init__(self):
        nz, ny, nx = self.shape
        v = DusVolume()
        v.nx, v.ny, v.nz = nx, ny, nz
        v.spacing_mm = (ctypes.c_float * 3)(*[float(x) for x in self.spacing])
        v.origin_mm = (ctypes.c_float * 3)(*[float(x) for x in self.origin])
        self.vol_c = v
        n = len(self.fans)
        arr = (DusFan * max(n, 1))()
        offs = np.zeros(n + 1, dtype=np.int64)
        for i, f in enumerate(self.fans):
            arr[i].n_rays = int(f.n_rays)
            arr[i].n_samples = int(f.n_samples)
            arr[i].aperture_rad = float(f.aperture)
            arr[i].ds_mm = float(f.ds)
            arr[i].r0_mm = float(f.r0)
            arr[i].speckle_id = int(f.speckle_id)
            arr[i].out_offset = int(offs[i])
            offs[i + 1] = offs[i] + int(f.n_rays) * int(f.n_samples)
        self.fans_c = arr
        self.offsets = offs
        self.total = int(offs[-1])
        self.phys_c = physics_record(self.phys)

    @property
    def n_poses(self) -> int:
        return len(self.fans)

    @property
    def total_rays(self) -> int:
        return int(sum(int(f.n_rays) for f in self.fans))

    def image(self, flat: torch.Tensor, p: int) -> torch.Tensor:
        f = self.fans[p]
        o = int(self.offsets[p])
        return flat[o:o + int(f.n_rays) * int(f.n_samples)].view(int(f.n_rays), int(f.n_samples))

    def workspace(self, with_backward: bool, device) -> torch.Tensor:
        nb = check(_lib.lib().dus_workspace_bytes(ctypes.byref(self.vol_c), self.fans_c, self.n_poses,
                                                 ctypes.byref(self.phys_c), int(with_backward)),
                   "dus_workspace_bytes")
        return torch.empty(max(int(nb), 1), dtype=torch.uint8, device=device)


def physics_record(ph) -> DusPhysics:
    p = DusPhysics()
    p.alpha_db_cm_mhz = float(ph.alpha)
    p.f_mhz = float(ph.freq)
    p.refl_mode = int(ph.refl_mode)
    p.atten_mode = int(ph.atten_mode)
    p.speckle_on = int(bool(ph.speckle_on))
    p.spk_cell = int(ph.spk_cell)
    p.spk_Ar, p.spk_gamma = float(ph.Ar), float(ph.gamma)
    p.spk_Ag0, p.spk_Ag1 = float(ph.Ag0), float(ph.Ag1)
    p.blur_on = int(bool(ph.blur_on))
    p.blur_sigma0, p.blur_sigma1 = float(ph.sigma0), float(ph.sigma1)
    p.reserved = 0
    p.seed = int(ph.seed) & 0xFFFFFFFFFFFFFFFF
    return p


def _check_inputs(Z: torch.Tensor, poses: torch.Tensor, geom: Geometry):
    if not Z.is_cuda or Z.dtype != torch.float32 or not Z.is_contiguous():
        raise ValueError("Z must be a contiguous float32 CUDA tensor")
    if tuple(Z.shape) != tuple(geom.shape):
        raise ValueError(f"Z shape {tuple(Z.shape)} != geometry {tuple(geom.shape)}")
    if (not poses.is_cuda or poses.dtype != torch.float32 or not poses.is_contiguous()
            or tuple(poses.shape) != (geom.n_poses, 6)):
        raise ValueError("poses must be a contiguous float32 CUDA tensor [n_poses, 6]")


def _check_buffer(t, name: str, numel: int, dtype=torch.float32, device=None):
    """A buffer the library writes or reads through a raw pointer: it must be
    a contiguous CUDA tensor of `dtype` with at least `numel` elements (the
    C ABI cannot see sizes)."""
    if t is None:
        return
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")


def render(Z: torch.Tensor, poses: torch.Tensor, geom: Geometry, want_pivot: bool = False,
           out: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """Forward render; returns the packed image (and per-ray min pivots)."""
    _check_inputs(Z, poses, geom)
    dev = Z.device
    if out is None:
        out = torch.empty(max(geom.total, 1), dtype=torch.float32, device=dev)
    _check_buffer(out, "out", geom.total, device=dev)
    piv = torch.empty(max(geom.total_rays, 1), dtype=torch.float32, device=dev) if want_pivot else None
    if ws is None:
        ws = geom.workspace(False, dev)
    _check_buffer(ws, "ws", 0, torch.uint8, dev)
    check(_lib.lib().dus_render_bmode(_ptr(Z), ctypes.byref(geom.vol_c), _ptr(poses), geom.fans_c,
                                      geom.n_poses, ctypes.byref(geom.phys_c), _ptr(out), _ptr(piv),
                                      _ptr(ws), ws.numel(), _stream()),
          "dus_render_bmode")
    out = out[:geom.total]
    return (out, piv[:geom.total_rays]) if want_pivot else out


def render_backward(Z: torch.Tensor, poses: torch.Tensor, geom: Geometry, grad_bmode: torch.Tensor,
                    want_Z: bool = True, want_pose: bool = True, grad_Z: torch.Tensor | None = None,
                    ws: torch.Tensor | None = None):
    """Hand-written adjoint: (dL/dZ, dL/dpose) for dL/dbmode."""
    _check_inputs(Z, poses, geom)
    dev = Z.device
    g = grad_bmode.contiguous().to(torch.float32)
    _check_buffer(g, "grad_bmode", geom.total, device=dev)
    gZ = None
    if want_Z:
        gZ = grad_Z if grad_Z is not None else torch.zeros_like(Z)
        _check_buffer(gZ, "grad_Z", Z.numel(), device=dev)
    gp = torch.empty((geom.n_poses, 6), dtype=torch.float32, device=dev) if want_pose else None
    if ws is None:
        ws = geom.workspace(True, dev)
    _check_buffer(ws, "ws", 0, torch.uint8, dev)
    check(_lib.lib().dus_render_bmode_backward(_ptr(Z), ctypes.byref(geom.vol_c), _ptr(poses),
                                               geom.fans_c, geom.n_poses, ctypes.byref(geom.phys_c),
                                               _ptr(g), _ptr(gZ), _ptr(gp), _ptr(ws), ws.numel(),
                                               _stream()),
          "dus_render_bmode_backward")
    return gZ, gp


def render_backward_static(Z: torch.Tensor, poses: torch.Tensor, geom: Geometry, grad_bmode: torch.Tensor,
                           grad_Z: torch.Tensor | None = None, grad_pose: torch.Tensor | None = None) -> None:
    """The adjoint with the library's static device scratch instead of a
    workspace (``dus_render_bmode_backward_static``): the library allocates
    nothing.  The caller passes the outputs: grad_Z (FP32, +=) and/or
    grad_pose (FP32 [n_poses, 6], overwritten); either may be None."""
    _check_inputs(Z, poses, geom)
    dev = Z.device
    _check_buffer(grad_bmode, "grad_bmode", geom.total, device=dev)
    _check_buffer(grad_Z, "grad_Z", Z.numel(), device=dev)
    _check_buffer(grad_pose, "grad_pose", 6 * geom.n_poses, device=dev)
    check(_lib.lib().dus_render_bmode_backward_static(_ptr(Z), ctypes.byref(geom.vol_c), _ptr(poses), geom.fans_c,
                                                      geom.n_poses, ctypes.byref(geom.phys_c), _ptr(grad_bmode),
                                                      _ptr(grad_Z), _ptr(grad_pose), _stream()),
          "dus_render_bmode_backward_static")


class RenderBmode(torch.autograd.Function):
    """bmode = render(Z, poses); gradients from the hand-written adjoint."""

    @staticmethod
    def forward(ctx, Z, poses, geom):
        ctx.geom = geom
        ctx.save_for_backward(Z, poses)
        return render(Z, poses, geom)

    @staticmethod
    def backward(ctx, grad):
        Z, poses = ctx.saved_tensors
        gZ, gp = render_backward(Z, poses, ctx.geom, grad, want_Z=ctx.needs_input_grad[0],
                                 want_pose=ctx.needs_input_grad[1])
        return gZ, gp, None


def render_ad(Z, poses, geom):
    return RenderBmode.apply(Z, poses, geom)


def philox(counters: torch.Tensor, seed: int) -> torch.Tensor:
    """Philox4x32-10 words (int32 view of uint32) for int32 counters [n, 4]."""
    c = counters.contiguous()
    out = torch.empty_like(c)
    check(_lib.lib().dus_philox4x32_10(_ptr(c), c.shape[0], int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(out),
                                       _stream()), "dus_philox4x32_10")
    return out


def pixel_gain(fan, phys, device) -> torch.Tensor:
    f = DusFan()
    f.n_rays, f.n_samples = int(fan.n_rays), int(fan.n_samples)
    f.aperture_rad, f.ds_mm, f.r0_mm = float(fan.aperture), float(fan.ds), float(fan.r0)
    f.speckle_id, f.out_offset = int(fan.speckle_id), 0
    out = torch.empty((max(f.n_rays, 1), max(f.n_samples, 1)), dtype=torch.float32, device=device)
    pr = physics_record(phys)
    check(_lib.lib().dus_pixel_gain(ctypes.byref(f), ctypes.byref(pr), _ptr(out), _stream()), "dus_pixel_gain")
    return out[:f.n_rays, :f.n_samples]


def set_schedule(fwd_chunk=0, bwd_chunk=0, xcd_group=0, scatter_rays=0, span_samples=0):
    """Schedule of the direct render / adjoint calls (0 = library default)."""
    s = DusSchedule(int(fwd_chunk), int(bwd_chunk), int(xcd_group), int(scatter_rays), int(span_samples))
    check(_lib.lib().dus_set_schedule(ctypes.byref(s)), "dus_set_schedule")


def get_schedule() -> dict:
    s = DusSchedule()
    check(_lib.lib().dus_get_schedule(ctypes.byref(s)), "dus_get_schedule")
    return {"fwd_chunk": s.fwd_chunk, "bwd_chunk": s.bwd_chunk, "xcd_group": s.xcd_group,
            "scatter_rays": s.scatter_rays, "span_samples": s.span_samples}


def sample_volume(Z: torch.Tensor, poses: torch.Tensor, geom: Geometry, out: torch.Tensor | None = None):
    """Sampling-only render: the impedance at every ray sample (packed image)."""
    _check_inputs(Z, poses, geom)
    if out is None:
        out = torch.empty(max(geom.total, 1), dtype=torch.float32, device=Z.device)
    _check_buffer(out, "out", geom.total, device=Z.device)
    check(_lib.lib().dus_sample_volume(_ptr(Z), ctypes.byref(geom.vol_c), _ptr(poses), geom.fans_c, geom.n_poses,
                                       _ptr(out), _stream()), "dus_sample_volume")
    return out[:geom.total]


def scan_convert(bmode: torch.Tensor, geom: Geometry, pose: int, nx: int, nz: int, x0_mm: float, z0_mm: float,
                 dx_mm: float, dz_mm: float, fill: float = 0.0) -> torch.Tensor:
    """Pose `pose`'s polar image (inside the packed `bmode`) on an nz x nx
    Cartesian grid of the probe's x-z plane."""
    if not 0 <= pose < geom.n_poses:
        raise ValueError(f"pose {pose} out of range")
    _check_buffer(bmode, "bmode", int(geom.offsets[pose + 1]))
    out = torch.empty((max(nz, 0), max(nx, 0)), dtype=torch.float32, device=bmode.device)
    grid = _lib.DusGrid2d(int(nx), int(nz), float(x0_mm), float(z0_mm), float(dx_mm), float(dz_mm), float(fill))
    check(_lib.lib().dus_scan_convert(_ptr(bmode), ctypes.byref(geom.fans_c[pose]), ctypes.byref(grid), _ptr(out),
                                      _stream()), "dus_scan_convert")
    return out


def smoothness(Z: torch.Tensor, geom: Geometry, weight: float, grad_Z: torch.Tensor,
               loss: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> None:
    """Smoothness prior: grad_Z += dR/dZ and loss += R (FP64 device scalar)."""
    if not (Z.is_cuda and Z.dtype == torch.float32 and Z.is_contiguous() and tuple(Z.shape) == tuple(geom.shape)):
        raise ValueError("Z must be a contiguous CUDA float32 tensor of the geometry's shape")
    _check_buffer(grad_Z, "grad_Z", Z.numel(), device=Z.device)
    _check_buffer(loss, "loss", 1, torch.float64, Z.device)
    L = _lib.lib()
    if ws is None:
        nbytes = int(check(L.dus_smoothness_workspace_bytes(ctypes.byref(geom.vol_c)),
                           "dus_smoothness_workspace_bytes"))
        ws = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=Z.device)
    check(L.dus_smoothness(_ptr(Z), ctypes.byref(geom.vol_c), float(weight), _ptr(grad_Z), _ptr(loss), _ptr(ws),
                           ws.numel() * ws.element_size(), _stream()), "dus_smoothness")


def adam_step(x: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, t: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, lo: float = -3.4e38,
              hi: float = 3.4e38) -> None:
    """One Adam step on x in place (m, v updated), x clamped to [lo, hi]."""
    for a in (x, grad, m, v):
        if not (a.is_cuda and a.dtype == torch.float32 and a.is_contiguous() and a.numel() == x.numel()):
            raise ValueError("x, grad, m, v must be contiguous CUDA float32 tensors of one size")
    check(_lib.lib().dus_adam_step(_ptr(x), _ptr(grad), _ptr(m), _ptr(v), x.numel(), float(lr), float(beta1),
                                   float(beta2), float(eps), int(t), float(lo), float(hi), _stream()),
          "dus_adam_step")


def lut_record(x, z) -> _lib.DusLut:
    """Piecewise-linear intensity -> impedance table as the ABI's record."""
    x = np.asarray(x, dtype=np.float32).reshape(-1)
    z = np.asarray(z, dtype=np.float32).reshape(-1)
    if x.shape != z.shape or not 2 <= x.size <= _lib.MAX_KNOTS:
        raise ValueError(f"the table needs 2..{_lib.MAX_KNOTS} (x, z) pairs of equal length")
    r = _lib.DusLut()
    r.n = int(x.size)
    for j in range(x.size):
        r.x[j], r.z[j] = float(x[j]), float(z[j])
    return r


def map_impedance(intensity: torch.Tensor, lut_x, lut_z, out: torch.Tensor | None = None) -> torch.Tensor:
    """Impedance volume from an intensity volume through the piecewise-linear
    table (lut_x, lut_z), constant beyond its ends."""
    _check_buffer(intensity, "intensity", 0)
    if out is None:
        out = torch.empty_like(intensity)
    _check_buffer(out, "out", intensity.numel(), device=intensity.device)
    lut = lut_record(lut_x, lut_z)
    check(_lib.lib().dus_map_impedance(_ptr(intensity), intensity.numel(), ctypes.byref(lut), _ptr(out), _stream()),
          "dus_map_impedance")
    return out


def map_impedance_backward(intensity: torch.Tensor, lut_x, lut_z, grad_Z: torch.Tensor, want_intensity: bool = True,
                           want_table: bool = True):
    """(dL/dintensity, dL/dz_j) of map_impedance for dL/dZ."""
    _check_buffer(intensity, "intensity", 0)
    _check_buffer(grad_Z, "grad_Z", intensity.numel(), device=intensity.device)
    lut = lut_record(lut_x, lut_z)
    gi = torch.empty_like(intensity) if want_intensity else None
    gz = torch.zeros(lut.n, dtype=torch.float64, device=intensity.device) if want_table else None
    check(_lib.lib().dus_map_impedance_backward(_ptr(intensity), intensity.numel(), ctypes.byref(lut), _ptr(grad_Z),
                                                _ptr(gi), _ptr(gz), _stream()), "dus_map_impedance_backward")
    return gi, gz


def footprint_mask(poses: torch.Tensor, geom: Geometry) -> torch.Tensor:
    """uint8 [nz][ny][nx]: 1 on every voxel of some trilinear stencil."""
    nz, ny, nx = geom.shape
    mask = torch.zeros((nz, ny, nx), dtype=torch.uint8, device=poses.device)
    check(_lib.lib().dus_footprint_mask(ctypes.byref(geom.vol_c), _ptr(poses), geom.fans_c, geom.n_poses,
                                        _ptr(mask), _stream()), "dus_footprint_mask")
    return mask


def footprint_voxels(poses: torch.Tensor, geom: Geometry) -> int:
    """Number of distinct voxels in the union of all trilinear stencils."""
    return int(footprint_mask(poses, geom).sum(dtype=torch.int64).item())


class FusedStep:
    """Batched fused forward + MSE + adjoint over all poses of ``geom``,
    replayed from a captured HIP graph (``dus_plan``).  ``deterministic``:
    dL/dZ bit-identical from step to step; ``one_stream``: every launch on
    the caller's stream (by default the fans run as two chains of launches
    on two streams)."""

    def __init__(self, geom: Geometry, pose_only: bool = False, zero_grad_z: bool = True,
                 graph: bool = True, schedule: dict | None = None, deterministic: bool = False,
                 one_stream: bool = False):
        L = _lib.lib()
        self.geom = geom
        flags = (_lib.PLAN_POSE_ONLY if pose_only else 0) | (_lib.PLAN_ZERO_GRAD_Z if zero_grad_z else 0)
        flags |= 0 if graph else _lib.PLAN_NO_GRAPH
        flags |= _lib.PLAN_DETERMINISTIC if deterministic else 0
        flags |= _lib.PLAN_ONE_STREAM if one_stream else 0
        h = ctypes.c_void_p()
        check(L.dus_plan_create(ctypes.byref(h), ctypes.byref(geom.vol_c), geom.fans_c, geom.n_poses,
                                ctypes.byref(geom.phys_c), flags), "dus_plan_create")
        self._h = h
        self._ws = None
        if schedule:
            self.set_schedule(**schedule)

    def set_schedule(self, fwd_chunk=0, bwd_chunk=0, xcd_group=0, scatter_rays=0, span_samples=0):
        s = DusSchedule(int(fwd_chunk), int(bwd_chunk), int(xcd_group), int(scatter_rays), int(span_samples))
        check(_lib.lib().dus_plan_set_schedule(self._h, ctypes.byref(s)), "dus_plan_set_schedule")

    def get_schedule(self) -> dict:
        s = DusSchedule()
        check(_lib.lib().dus_plan_get_schedule(self._h, ctypes.byref(s)), "dus_plan_get_schedule")
        return {"fwd_chunk": s.fwd_chunk, "bwd_chunk": s.bwd_chunk, "xcd_group": s.xcd_group,
                "scatter_rays": s.scatter_rays, "span_samples": s.span_samples}

    def workspace(self, device) -> torch.Tensor:
        if self._ws is None or self._ws.device != torch.device(device):
            nb = check(_lib.lib().dus_plan_workspace_bytes(self._h), "dus_plan_workspace_bytes")
            self._ws = torch.empty(max(int(nb), 1), dtype=torch.uint8, device=device)
        return self._ws

    def _check_step(self, Z, poses, target, bmode, loss, grad_Z, grad_pose):
        _check_inputs(Z, poses, self.geom)
        dev = Z.device
        if target is None:
            raise ValueError("target is required")
        _check_buffer(target, "target", self.geom.total, device=dev)
        _check_buffer(bmode, "bmode", self.geom.total, device=dev)
        _check_buffer(loss, "loss", 1, torch.float64, dev)
        _check_buffer(grad_Z, "grad_Z", Z.numel(), device=dev)
        _check_buffer(grad_pose, "grad_pose", 6 * self.geom.n_poses, device=dev)

    def step(self, Z, poses, target, bmode=None, loss=None, grad_Z=None, grad_pose=None):
        self._check_step(Z, poses, target, bmode, loss, grad_Z, grad_pose)
        ws = self.workspace(Z.device)
        check(_lib.lib().dus_plan_step(self._h, _ptr(Z), _ptr(poses), _ptr(target), _ptr(bmode), _ptr(loss),
                                       _ptr(grad_Z), _ptr(grad_pose), _ptr(ws), ws.numel(), _stream()),
              "dus_plan_step")

    def step_timed(self, Z, poses, target, bmode=None, loss=None, grad_Z=None, grad_pose=None) -> dict:
        """One step launched eagerly with HIP events at the phase boundaries;
        returns {phase: ms} (blocks until the step has finished)."""
        self._check_step(Z, poses, target, bmode, loss, grad_Z, grad_pose)
        ws = self.workspace(Z.device)
        ms = (ctypes.c_float * len(_lib.PHASES))()
        check(_lib.lib().dus_plan_step_timed(self._h, _ptr(Z), _ptr(poses), _ptr(target), _ptr(bmode), _ptr(loss),
                                             _ptr(grad_Z), _ptr(grad_pose), _ptr(ws), ws.numel(), _stream(), ms),
              "dus_plan_step_timed")
        return {name: float(ms[i]) for i, name in enumerate(_lib.PHASES)}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().dus_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
