"""Seeded synthetic inputs for the fan-beam renderer.

This module holds no rendering arithmetic: it only draws impedance volumes,
probe poses and fan geometries from ``numpy.random.default_rng(seed)``.  Both
the GPU path (tests, bench) and the FP64 oracle consume what it returns.

The volumes stand in for the MRI-derived brain impedance maps the paper
renders (Sec. 3.1): a soft-tissue background around 1.5 MRayl, ellipsoidal
regions of other soft-tissue impedances, Gaussian-smoothed impedance noise
and a skull-like shell of 7.8 MRayl.  Nothing from any dataset is used.

Coordinates: the volume is Z[nz][ny][nx] (x fastest), voxel (i, j, k) has
its centre at origin + (i hx, j hy, k hz) mm.  A pose is (t_x, t_y, t_z,
w_x, w_y, w_z): apex position in mm and rotation vector in rad, mapping probe
coordinates q to world t + R(w) q.  In probe coordinates the beam points
along +z and the fan opens in the x-z plane.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

DEG = np.pi / 180.0


@dataclass
class FanSpec:
    n_rays: int
    n_samples: int
    aperture: float          # rad, full fan angle
    ds: float                # mm per depth sample
    r0: float = 0.0          # mm from apex to first sample
    speckle_id: int = 0


@dataclass
class PhysicsSpec:
    alpha: float = 0.5       # dB/cm/MHz
    freq: float = 5.0        # MHz
    refl_mode: int = 0       # 0 = |R| as printed in Eq. 1, 1 = signed
    atten_mode: int = 0      # 0 = in system, 1 = post hoc, 2 = off
    speckle_on: bool = False
    spk_cell: int = 8
    Ar: float = 0.3
    gamma: float = 1.5
    Ag0: float = 0.2
    Ag1: float = 0.3
    blur_on: bool = False
    sigma0: float = 0.5
    sigma1: float = 2.5
    seed: int = 0


@dataclass
class Case:
    """One workload: a volume, P poses with their fans, and the physics."""
    name: str
    Z: np.ndarray                      # float32 [nz][ny][nx]
    spacing: tuple
    origin: tuple
    poses: np.ndarray                  # float32 [P][6]
    fans: list                         # FanSpec per pose
    phys: PhysicsSpec
    extra: dict = field(default_factory=dict)

    @property
    def ray_samples(self) -> int:
        return int(sum(f.n_rays * f.n_samples for f in self.fans))


# --------------------------------------------------------------------------
# volumes
# --------------------------------------------------------------------------
def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _paint_ellipsoid(Z, spacing, origin, centre, semi, Q, value):
    """Z[p] = value where |Q^T (p - centre) / semi| <= 1 (painted in place)."""
    nz, ny, nx = Z.shape
    r = float(np.max(semi))
    lo = [int(np.floor((centre[a] - r - origin[a]) / spacing[a])) for a in range(3)]
    hi = [int(np.ceil((centre[a] + r - origin[a]) / spacing[a])) for a in range(3)]
    n = (nx, ny, nz)
    lo = [max(0, v) for v in lo]
    hi = [min(n[a] - 1, hi[a]) for a in range(3)]
    if any(hi[a] < lo[a] for a in range(3)):
        return
    xs = origin[0] + spacing[0] * np.arange(lo[0], hi[0] + 1) - centre[0]
    ys = origin[1] + spacing[1] * np.arange(lo[1], hi[1] + 1) - centre[1]
    zs = origin[2] + spacing[2] * np.arange(lo[2], hi[2] + 1) - centre[2]
    zz, yy, xx = np.meshgrid(zs, ys, xs, indexing="ij")
    # body coordinates b = Q^T d
    b0 = Q[0, 0] * xx + Q[1, 0] * yy + Q[2, 0] * zz
    b1 = Q[0, 1] * xx + Q[1, 1] * yy + Q[2, 1] * zz
    b2 = Q[0, 2] * xx + Q[1, 2] * yy + Q[2, 2] * zz
    inside = (b0 / semi[0]) ** 2 + (b1 / semi[1]) ** 2 + (b2 / semi[2]) ** 2 <= 1.0
    sub = Z[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
    sub[inside] = value


def _paint_shell(Z, spacing, origin, centre, outer, thickness, value):
    inner = np.asarray(outer, dtype=np.float64) - thickness
    eye = np.eye(3)
    # outer ellipsoid mask minus inner ellipsoid mask, axis aligned
    tmp_out = np.zeros(Z.shape, dtype=np.uint8)
    _paint_ellipsoid(tmp_out, spacing, origin, centre, np.asarray(outer, float), eye, 1)
    tmp_in = np.zeros(Z.shape, dtype=np.uint8)
    _paint_ellipsoid(tmp_in, spacing, origin, centre, inner, eye, 1)
    shell = (tmp_out > 0) & ~(tmp_in > 0)
    Z[shell] = value


def brain_volume(seed: int, n: int = 256, spacing: float = 1.0, n_ell_range=(8, 16),
                 centre_frac=(0.25, 0.75), semi_range=(6.0, 40.0), z_range=(1.3, 1.8),
                 noise_sigma_vox: float = 2.0, noise_std: float = 0.02,
                 shell_centre=None, shell_outer=None, shell_thick: float = 7.0,
                 shell_Z: float = 7.8) -> np.ndarray:
    """Piecewise-smooth impedance volume (MRayl, float32 [n][n][n])."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    ext = (n - 1) * spacing
    origin = (0.0, 0.0, 0.0)
    sp = (spacing, spacing, spacing)
    Z = np.full((n, n, n), rng.uniform(1.45, 1.65), dtype=np.float32)
    n_ell = int(rng.integers(n_ell_range[0], n_ell_range[1] + 1))
    scale = ext / 255.0
    for _ in range(n_ell):
        c = rng.uniform(centre_frac[0] * ext, centre_frac[1] * ext, size=3)
        a = rng.uniform(semi_range[0], semi_range[1], size=3) * scale
        Q = _random_rotation(rng)
        _paint_ellipsoid(Z, sp, origin, c, a, Q, np.float32(rng.uniform(*z_range)))
    if noise_std > 0:
        w = rng.standard_normal(size=Z.shape).astype(np.float32)
        w = gaussian_filter(w, sigma=noise_sigma_vox, mode="reflect")
        w *= noise_std / float(np.std(w))
        Z += w
    if shell_centre is None:
        shell_centre = (ext / 2.0, ext / 2.0, ext / 2.0 + 8.0 * scale)
    if shell_outer is None:
        shell_outer = (100.0 * scale, 118.0 * scale, 110.0 * scale)
    _paint_shell(Z, sp, origin, shell_centre, shell_outer, shell_thick * scale, np.float32(shell_Z))
    return np.ascontiguousarray(Z, dtype=np.float32)


def simple_volume(seed: int, n: int = 64) -> np.ndarray:
    """Piecewise-constant 64^3 phantom: one background value, 4 ellipsoids,
    one shell crossed twice by a vertical ray."""
    rng = np.random.default_rng(seed)
    sp = (1.0, 1.0, 1.0)
    o = (0.0, 0.0, 0.0)
    Z = np.full((n, n, n), rng.uniform(1.45, 1.65), dtype=np.float32)
    f = n / 64.0
    for _ in range(4):
        c = rng.uniform(16 * f, 48 * f, size=3)
        a = rng.uniform(4 * f, 12 * f, size=3)
        Q = _random_rotation(rng)
        _paint_ellipsoid(Z, sp, o, c, a, Q, np.float32(rng.uniform(1.3, 1.8)))
    ctr = ((n - 1) / 2.0, (n - 1) / 2.0, 36.0 * f)
    _paint_shell(Z, sp, o, ctr, (28.0 * f, 28.0 * f, 26.0 * f), 3.0 * f, np.float32(7.8))
    return Z


# --------------------------------------------------------------------------
# poses and fans
# --------------------------------------------------------------------------
def top_pose(n: int, spacing: float = 1.0) -> np.ndarray:
    """Apex centred on the top face (z = 0), beam straight down +z."""
    c = (n - 1) * spacing / 2.0
    return np.array([c, c, 0.0, 0.0, 0.0, 0.0], dtype=np.float32)


def random_poses(rng, P: int, ext: float):
    """c4-style poses: apex (U(96,160), U(96,160), U(0,8)) mm scaled to the
    volume extent, rotation vector U(-15 deg, 15 deg)^3."""
    s = ext / 255.0
    t = np.stack([rng.uniform(96 * s, 160 * s, P), rng.uniform(96 * s, 160 * s, P),
                  rng.uniform(0, 8 * s, P)], axis=1)
    w = rng.uniform(-15 * DEG, 15 * DEG, size=(P, 3))
    return np.concatenate([t, w], axis=1).astype(np.float32)


def offset_poses(rng, poses: np.ndarray, dt_mm: float, dw_deg: float) -> np.ndarray:
    P = poses.shape[0]
    d = np.concatenate([rng.uniform(-dt_mm, dt_mm, (P, 3)),
                        rng.uniform(-dw_deg * DEG, dw_deg * DEG, (P, 3))], axis=1)
    return (poses.astype(np.float64) + d).astype(np.float32)


def effects_physics(seed: int) -> PhysicsSpec:
    return PhysicsSpec(speckle_on=True, blur_on=True, seed=seed)


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------
def case_small_forward(seed: int = 1001) -> Case:
    """64^3 phantom (1 mm), one 60 deg fan of 64 rays x 256 samples from the
    top face, ds = 0.25 mm, 0.5 dB/cm/MHz at 5 MHz, no speckle or blur."""
    Z = simple_volume(seed, 64)
    fan = FanSpec(64, 256, 60 * DEG, 0.25)
    return Case("fwd_64cube_64x256", Z, (1.0,) * 3, (0.0,) * 3, top_pose(64)[None, :], [fan],
                PhysicsSpec(seed=seed))


_VOL_CACHE: dict = {}


def brain256(seed: int = 1002) -> np.ndarray:
    key = ("brain", seed, 256)
    if key not in _VOL_CACHE:
        _VOL_CACHE[key] = brain_volume(seed, 256, 1.0)
    return _VOL_CACHE[key]


def case_forward_effects(seed: int = 1002) -> Case:
    """256^3 brain-like volume, one 70 deg fan of 256 rays x 1024 samples,
    ds = 0.25 mm, speckle and depth-dependent blur on."""
    Z = brain256(seed)
    fan = FanSpec(256, 1024, 70 * DEG, 0.25)
    return Case("fwd_256cube_256x1024_effects", Z, (1.0,) * 3, (0.0,) * 3,
                top_pose(256)[None, :], [fan], effects_physics(seed))


def case_adjoint(seed: int = 1003, vol_seed: int = 1002) -> Case:
    """Volume of the 256^3 case, 512 rays x 1024 samples, effects on; the
    target is rendered at a pose offset by U(-5,5) mm and U(-5,5) deg."""
    Z = brain256(vol_seed)
    rng = np.random.default_rng(seed)
    base = top_pose(256)[None, :]
    tgt = offset_poses(rng, base, 5.0, 5.0)
    fan = FanSpec(512, 1024, 70 * DEG, 0.25)
    return Case("fwdbwd_256cube_512x1024", Z, (1.0,) * 3, (0.0,) * 3, base, [fan],
                effects_physics(seed), extra={"target_poses": tgt})


def uneven_fans(rng, P: int, ext: float, rays=(128, 512), samples=(256, 2048),
                aperture_deg=(40, 90), depth=(100, 240)):
    s = ext / 255.0
    fans = []
    for p in range(P):
        n_r = int(rng.integers(rays[0], rays[1] + 1))
        S = int(rng.integers(samples[0], samples[1] + 1))
        A = rng.uniform(*aperture_deg) * DEG
        d = rng.uniform(depth[0], depth[1]) * s
        fans.append(FanSpec(n_r, S, A, d / S, 0.0, p))
    return fans


def case_batched(seed: int = 1004, vol_seed: int = 1002, P: int = 64) -> Case:
    """64 poses with uneven fans (128-512 rays, 256-2048 samples, 40-90 deg,
    100-240 mm deep) over the 256^3 volume; targets at +-5 mm / +-5 deg."""
    Z = brain256(vol_seed)
    rng = np.random.default_rng(seed)
    ext = 255.0
    poses = random_poses(rng, P, ext)
    fans = uneven_fans(rng, P, ext)
    tgt = offset_poses(rng, poses, 5.0, 5.0)
    return Case("batched_256cube_64poses", Z, (1.0,) * 3, (0.0,) * 3, poses, fans,
                effects_physics(seed), extra={"target_poses": tgt})


def case_batched_c2(B: int = 64, seed: int = 1006, vol_seed: int = 1002) -> Case:
    """B poses, each the 256 x 1024, 70 deg fan of the 256^3 case, apexes
    spread over the top face and tilted by up to 15 deg."""
    Z = brain256(vol_seed)
    rng = np.random.default_rng(seed)
    poses = random_poses(rng, B, 255.0)
    fans = [FanSpec(256, 1024, 70 * DEG, 0.25, 0.0, p) for p in range(B)]
    tgt = offset_poses(rng, poses, 5.0, 5.0)
    return Case(f"batched_256cube_{B}x256x1024", Z, (1.0,) * 3, (0.0,) * 3, poses, fans,
                effects_physics(seed), extra={"target_poses": tgt})


def case_skewed(even: bool = False, seed: int = 1007, vol_seed: int = 1002, P: int = 64) -> Case:
    """A batch whose ray lengths are very uneven: P - 1 poses of 256 rays x
    256 samples and one pose of 64 rays x 16384 samples (the longest rays the
    renderer takes), all 70 deg fans 200 mm deep, speckle and blur.  With
    even=True the same number of ray-samples is spread over P fans of 256 rays
    x 316 samples instead (the reference for the skewed batch's time)."""
    Z = brain256(vol_seed)
    rng = np.random.default_rng(seed)
    poses = random_poses(rng, P, 255.0)
    if even:
        fans = [FanSpec(256, 316, 70 * DEG, 200.0 / 316, 0.0, p) for p in range(P)]
    else:
        fans = [FanSpec(256, 256, 70 * DEG, 200.0 / 256, 0.0, p) for p in range(P - 1)]
        fans.append(FanSpec(64, 16384, 70 * DEG, 200.0 / 16384, 0.0, P - 1))
    tgt = offset_poses(rng, poses, 5.0, 5.0)
    return Case("skewed_even" if even else "skewed", Z, (1.0,) * 3, (0.0,) * 3, poses, fans,
                effects_physics(seed), extra={"target_poses": tgt})


def case_registration(seed: int = 1005, n: int = 512, P: int = 32, offset: float = 10.0) -> Case:
    """512^3 volume at 0.5 mm (noise sigma 4 voxels), 32 ground-truth poses,
    initial poses +-offset mm / +-offset deg (10 by default), 384 rays x 1536
    samples, 70 deg, 192 mm."""
    h = 255.5 / (n - 1)
    Z = brain_volume(seed, n, h, noise_sigma_vox=4.0)
    rng = np.random.default_rng(seed)
    gt = random_poses(rng, P, (n - 1) * h)
    init = offset_poses(rng, gt, offset, offset)
    fans = [FanSpec(384, 1536, 70 * DEG, 192.0 / 1536, 0.0, p) for p in range(P)]
    return Case(f"registration_{n}cube_{P}poses", Z, (h,) * 3, (0.0,) * 3, init, fans,
                effects_physics(seed), extra={"gt_poses": gt})
