"""Plain FP64 CPU oracle of the DiffUS fan-beam renderer (arXiv 2508.06768).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It never imports
the GPU package and the GPU package never imports it; the two share nothing
but the seeded input generator, which holds none of the method's arithmetic.

The numerical work lives in ``diffus_oracle.c`` (FP64, OpenMP over rays),
loaded here with ctypes.  This module adds the pieces that are plainest in
NumPy:

* ``dense_system`` / ``echo_dense`` -- the paper's sparse system (Sec. 2.3,
  Eq. 3 and Eq. 4) built entry by entry as a dense matrix and solved with
  LAPACK for every truncation depth k (Sec. 2.4).  Used as a pin on tiny rays.
* ``echo_paths`` -- the same echo as a sum over scattering paths (Neumann
  series of Eq. 4), a pin for the multiple-reflection claim of Sec. 2.3.
* finite differences of the rendered loss (``fd_*``), the pin of the adjoint.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "diffus_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

REFL_ABS, REFL_SIGNED = 0, 1
ATTEN_IN_SYSTEM, ATTEN_POST_HOC, ATTEN_OFF = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Vol(ctypes.Structure):
    _fields_ = [("V", ctypes.POINTER(ctypes.c_double)),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("pad_", ctypes.c_int32),
                ("h", ctypes.c_double * 3), ("o", ctypes.c_double * 3)]


class _Fan(ctypes.Structure):
    _fields_ = [("n_rays", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("aperture", ctypes.c_double), ("ds", ctypes.c_double), ("r0", ctypes.c_double),
                ("speckle_id", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class _Phys(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("freq", ctypes.c_double),
                ("refl_mode", ctypes.c_int32), ("atten_mode", ctypes.c_int32),
                ("speckle_on", ctypes.c_int32), ("spk_cell", ctypes.c_int32),
                ("Ar", ctypes.c_double), ("gam", ctypes.c_double),
                ("Ag0", ctypes.c_double), ("Ag1", ctypes.c_double),
                ("blur_on", ctypes.c_int32), ("sigma0", ctypes.c_float), ("sigma1", ctypes.c_float),
                ("pad_", ctypes.c_int32), ("seed", ctypes.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d = ctypes.POINTER(ctypes.c_double)
        _lib.orc_sample.restype = ctypes.c_double
        _lib.orc_step_amplitude.restype = ctypes.c_double
        _lib.orc_render.restype = ctypes.c_int
        _lib.orc_backward.restype = ctypes.c_int
        _lib.orc_blur_radius.restype = ctypes.c_int
        _lib.orc_num_threads.restype = ctypes.c_int
        _lib.orc_rayleigh.restype = ctypes.c_double
        _lib.orc_rayleigh.argtypes = [ctypes.c_uint32]
        _lib.orc_set_num_threads.restype = None
        del d
    return _lib


def num_threads() -> int:
    """Threads of the oracle's OpenMP loops."""
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's OpenMP loops from now on (timing only)."""
    lib().orc_set_num_threads(ctypes.c_int(int(n)))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Volume:
    """Impedance volume Z[nz][ny][nx] (MRayl) with spacing and origin in mm."""
    Z: np.ndarray
    spacing: tuple = (1.0, 1.0, 1.0)
    origin: tuple = (0.0, 0.0, 0.0)

    def __post_init__(self):
        self.Z = np.ascontiguousarray(self.Z, dtype=np.float64)

    def c(self) -> _Vol:
        nz, ny, nx = self.Z.shape
        v = _Vol()
        v.V = _dp(self.Z)
        v.nx, v.ny, v.nz = nx, ny, nz
        v.h = (ctypes.c_double * 3)(*[float(x) for x in self.spacing])
        v.o = (ctypes.c_double * 3)(*[float(x) for x in self.origin])
        return v


@dataclass
class Fan:
    n_rays: int
    n_samples: int
    aperture: float     # rad
    ds: float           # mm
    r0: float = 0.0     # mm
    speckle_id: int = 0

    def c(self) -> _Fan:
        f = _Fan()
        f.n_rays, f.n_samples = int(self.n_rays), int(self.n_samples)
        f.aperture, f.ds, f.r0 = float(self.aperture), float(self.ds), float(self.r0)
        f.speckle_id = int(self.speckle_id)
        return f


@dataclass
class Physics:
    alpha: float = 0.5          # dB/cm/MHz
    freq: float = 5.0           # MHz
    refl_mode: int = REFL_ABS
    atten_mode: int = ATTEN_IN_SYSTEM
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

    def c(self) -> _Phys:
        p = _Phys()
        p.alpha, p.freq = float(self.alpha), float(self.freq)
        p.refl_mode, p.atten_mode = int(self.refl_mode), int(self.atten_mode)
        p.speckle_on, p.spk_cell = int(bool(self.speckle_on)), int(self.spk_cell)
        p.Ar, p.gam, p.Ag0, p.Ag1 = float(self.Ar), float(self.gamma), float(self.Ag0), float(self.Ag1)
        p.blur_on = int(bool(self.blur_on))
        p.sigma0, p.sigma1 = float(self.sigma0), float(self.sigma1)
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        return p


def _pose(pose) -> np.ndarray:
    p = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(6))
    return p


# --------------------------------------------------------------------------
# Whole-fan rendering and its derivative
# --------------------------------------------------------------------------
def render(vol: Volume, pose, fan: Fan, phys: Physics, solver: str = "transfer",
           want_raw: bool = False, want_pivot: bool = False):
    """B-mode image [n_rays][n_samples] of one fan (Sec. 2.4), FP64.

    solver="transfer": O(S) composition of the per-interface Moebius maps;
    solver="banded": the literal progressive solve, O(S^2) per ray.
    """
    L = lib()
    p = _pose(pose)
    img = np.zeros((fan.n_rays, fan.n_samples), dtype=np.float64)
    raw = np.zeros_like(img) if want_raw else None
    piv = np.zeros(fan.n_rays, dtype=np.float64) if want_pivot else None
    cv, cf, cp = vol.c(), fan.c(), phys.c()
    rc = L.orc_render(ctypes.byref(cv), _dp(p), ctypes.byref(cf), ctypes.byref(cp),
                      1 if solver == "banded" else 0, _dp(img),
                      _dp(raw) if raw is not None else None,
                      _dp(piv) if piv is not None else None)
    if rc != 0:
        raise RuntimeError("oracle render failed")
    out = [img]
    if want_raw:
        out.append(raw)
    if want_pivot:
        out.append(piv)
    return out[0] if len(out) == 1 else tuple(out)


def backward(vol: Volume, pose, fan: Fan, phys: Physics, grad_img: np.ndarray,
             want_volume: bool = True, grad_volume: np.ndarray | None = None):
    """dL/dZ (volume, FP64) and dL/dpose (t_xyz mm, w_xyz rad) for dL/dimg.

    grad_volume: optional C-contiguous FP64 array of the volume's shape that
    receives dL/dZ added in place (the C routine accumulates); it is then
    the returned volume gradient.  Without it a zeroed one is allocated."""
    L = lib()
    p = _pose(pose)
    g = np.ascontiguousarray(grad_img, dtype=np.float64).reshape(fan.n_rays, fan.n_samples)
    gV = None
    if grad_volume is not None:
        if (grad_volume.dtype != np.float64 or grad_volume.shape != vol.Z.shape
                or not grad_volume.flags["C_CONTIGUOUS"]):
            raise ValueError("grad_volume must be a C-contiguous float64 array of the volume's shape")
        gV = grad_volume
    elif want_volume:
        gV = np.zeros_like(vol.Z)
    gp = np.zeros(6, dtype=np.float64)
    cv, cf, cp = vol.c(), fan.c(), phys.c()
    rc = L.orc_backward(ctypes.byref(cv), _dp(p), ctypes.byref(cf), ctypes.byref(cp), _dp(g),
                        _dp(gV) if gV is not None else None, _dp(gp))
    if rc != 0:
        raise RuntimeError("oracle backward failed")
    return gV, gp


def mse_loss_grad(img: np.ndarray, target: np.ndarray):
    """L = mean((img - target)^2) and dL/dimg."""
    d = img - target
    return float(np.mean(d * d)), 2.0 * d / d.size


# --------------------------------------------------------------------------
# Per-ray pieces (pins)
# --------------------------------------------------------------------------
def ray_samples(vol: Volume, pose, fan: Fan, j: int, want_grad: bool = False):
    L = lib()
    p = _pose(pose)
    Zs = np.zeros(fan.n_samples)
    gp = np.zeros(3 * fan.n_samples) if want_grad else None
    q = np.zeros(3 * fan.n_samples)
    cv, cf = vol.c(), fan.c()
    L.orc_ray_samples(ctypes.byref(cv), _dp(p), ctypes.byref(cf), ctypes.c_int(j), _dp(Zs),
                      _dp(gp) if gp is not None else None, _dp(q))
    if want_grad:
        return Zs, gp.reshape(-1, 3), q.reshape(-1, 3)
    return Zs


def sample_image(vol: Volume, pose, fan: Fan) -> np.ndarray:
    """Sampling-only image [n_rays][n_samples]: the impedance at every ray
    sample (the ablation row of Table 1)."""
    return np.stack([ray_samples(vol, pose, fan, j) for j in range(fan.n_rays)]) if fan.n_rays else \
        np.zeros((0, fan.n_samples))


def scan_convert(img, fan: Fan, nx: int, nz: int, x0: float, z0: float, dx: float, dz: float,
                 fill: float = 0.0) -> np.ndarray:
    """One fan's polar image [n_rays][n_samples] on an nz x nx Cartesian grid
    of the probe's x-z plane (bilinear; `fill` outside the fan)."""
    im = np.ascontiguousarray(np.asarray(img, dtype=np.float64).reshape(fan.n_rays, fan.n_samples))
    out = np.zeros((nz, nx))
    lib().orc_scan_convert(_dp(im), ctypes.c_int(fan.n_rays), ctypes.c_int(fan.n_samples),
                           ctypes.c_double(fan.aperture), ctypes.c_double(fan.r0), ctypes.c_double(fan.ds),
                           ctypes.c_int(nx), ctypes.c_int(nz), ctypes.c_double(x0), ctypes.c_double(z0),
                           ctypes.c_double(dx), ctypes.c_double(dz), ctypes.c_double(fill), _dp(out))
    return out


def smoothness(Z, spacing, weight: float):
    """Smoothness prior of the reconstruction, written from its definition:
    R = weight * sum over axes a of sum over neighbour pairs (v, v + e_a) of
    ((Z[v + e_a] - Z[v]) / h_a)^2, with its gradient.  Z is [nz][ny][nx];
    spacing = (h_x, h_y, h_z).  Returns (R, dR/dZ)."""
    Z = np.asarray(Z, dtype=np.float64)
    g = np.zeros_like(Z)
    R = 0.0
    for axis, h in ((2, spacing[0]), (1, spacing[1]), (0, spacing[2])):
        w = weight / (h * h)
        n = Z.shape[axis]
        for i in range(n - 1):
            a = [slice(None)] * 3
            b = [slice(None)] * 3
            a[axis] = i
            b[axis] = i + 1
            d = Z[tuple(b)] - Z[tuple(a)]
            R += w * float(np.sum(d * d))
            g[tuple(a)] -= 2.0 * w * d
            g[tuple(b)] += 2.0 * w * d
    return R, g


def map_impedance(v, xk, zk):
    """Impedance mapping (Sec. 2.2: intensities to impedance, voxel by voxel)
    as a piecewise-linear table, written from its definition: z_0 at or
    below x_0, z_{n-1} at or above x_{n-1}, and for x_j <= v < x_{j+1}
    Z = z_j + t (z_{j+1} - z_j) with t = (v - x_j) / (x_{j+1} - x_j).
    Also returns dZ/dv (the slope of the segment to the right at a knot, 0
    beyond the ends).  NaN stays NaN.  FP64."""
    v = np.asarray(v, dtype=np.float64)
    xk = np.asarray(xk, dtype=np.float64)
    zk = np.asarray(zk, dtype=np.float64)
    Z = np.full(v.shape, np.nan)
    dv = np.zeros(v.shape)
    Z[v <= xk[0]] = zk[0]
    Z[v >= xk[-1]] = zk[-1]
    for j in range(len(xk) - 1):
        sel = (v >= xk[j]) & (v < xk[j + 1]) & (v > xk[0])
        t = (v[sel] - xk[j]) / (xk[j + 1] - xk[j])
        Z[sel] = zk[j] + t * (zk[j + 1] - zk[j])
        dv[sel] = (zk[j + 1] - zk[j]) / (xk[j + 1] - xk[j])
    return Z, dv


def map_impedance_grad(v, xk, zk, gZ):
    """Adjoint of map_impedance for dL/dZ = gZ: (dL/dv, dL/dz_j).  Each voxel
    hands (1 - t) gZ to z_j and t gZ to z_{j+1} inside segment j, all of gZ
    to the end knot beyond an end."""
    v = np.asarray(v, dtype=np.float64)
    gZ = np.asarray(gZ, dtype=np.float64)
    xk = np.asarray(xk, dtype=np.float64)
    _, dv = map_impedance(v, xk, zk)
    gz = np.zeros(len(xk))
    gz[0] += gZ[v <= xk[0]].sum()
    gz[-1] += gZ[v >= xk[-1]].sum()
    for j in range(len(xk) - 1):
        sel = (v >= xk[j]) & (v < xk[j + 1]) & (v > xk[0])
        t = (v[sel] - xk[j]) / (xk[j + 1] - xk[j])
        gz[j] += ((1.0 - t) * gZ[sel]).sum()
        gz[j + 1] += (t * gZ[sel]).sum()
    return gZ * dv, gz


def adam(x, g, m, v, t: int, lr: float, beta1: float, beta2: float, eps: float, lo: float, hi: float):
    """One Adam step (Kingma and Ba, 2015) with the result clamped to
    [lo, hi]; returns (x, m, v) as new arrays (FP64)."""
    x, g, m, v = (np.asarray(a, dtype=np.float64) for a in (x, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    x = np.clip(x - lr * mh / (np.sqrt(vh) + eps), lo, hi)
    return x, m, v


def sample(vol: Volume, u):
    L = lib()
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(3))
    g = np.zeros(3)
    cv = vol.c()
    z = L.orc_sample(ctypes.byref(cv), _dp(uu), _dp(g), None, None)
    return z, g


def coeffs(Z1: float, Z2: float, refl_mode: int = REFL_ABS):
    """(R_{1->2}, R_{2->1}, T_{1->2}, T_{2->1}) of Eq. 1."""
    out = np.zeros(4)
    lib().orc_coeffs(ctypes.c_double(Z1), ctypes.c_double(Z2), ctypes.c_int(refl_mode), _dp(out))
    return tuple(out)


def step_amplitude(phys: Physics, ds: float) -> float:
    cp = phys.c()
    return float(lib().orc_step_amplitude(ctypes.byref(cp), ctypes.c_double(ds)))


def echo_banded(Zs, a: float = 1.0, refl_mode: int = REFL_ABS):
    """d_0^(k), k = 0..S-1, by the literal O(S^2) progressive solve; and min pivot."""
    Zs = np.ascontiguousarray(Zs, dtype=np.float64)
    d0 = np.zeros(len(Zs))
    mp = ctypes.c_double()
    lib().orc_echo_banded(_dp(Zs), ctypes.c_int(len(Zs)), ctypes.c_double(a), ctypes.c_int(refl_mode),
                          _dp(d0), ctypes.byref(mp))
    return d0, mp.value


def echo_transfer(Zs, a: float = 1.0, refl_mode: int = REFL_ABS):
    """(e, d0, min forward pivot) by the O(S) transfer-matrix composition."""
    Zs = np.ascontiguousarray(Zs, dtype=np.float64)
    e = np.zeros(len(Zs))
    d0 = np.zeros(len(Zs))
    mp = ctypes.c_double()
    lib().orc_echo_transfer(_dp(Zs), ctypes.c_int(len(Zs)), ctypes.c_double(a), ctypes.c_int(refl_mode),
                            _dp(e), _dp(d0), ctypes.byref(mp))
    return e, d0, mp.value


def rotation(w) -> np.ndarray:
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(3))
    R = np.zeros(9)
    lib().orc_rotation(_dp(w), _dp(R))
    return R.reshape(3, 3)


def rotation_grad(w) -> np.ndarray:
    """dR/dw_c as an array [3 (c)][3][3]."""
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(3))
    dR = np.zeros(27)
    lib().orc_rotation_grad(_dp(w), _dp(dR))
    return dR.reshape(3, 3, 3)


def philox(counters: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 words for an array of 4-word counters (uint32 [n][4])."""
    c = np.ascontiguousarray(counters, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.zeros_like(c)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib().orc_philox_batch(c.ctypes.data_as(u32p), ctypes.c_int64(c.shape[0]), k.ctypes.data_as(u32p),
                           out.ctypes.data_as(u32p))
    return out


def rayleigh(word: int) -> float:
    """Unit-mean Rayleigh variate of one 32-bit generator word (the map the
    speckle multipliers use)."""
    return float(lib().orc_rayleigh(ctypes.c_uint32(int(word) & 0xFFFFFFFF)))


def speckle_ray(fan: Fan, phys: Physics, j: int) -> np.ndarray:
    m = np.zeros(fan.n_samples)
    cf, cp = fan.c(), phys.c()
    lib().orc_speckle_ray(ctypes.byref(cf), ctypes.byref(cp), ctypes.c_int(j), _dp(m))
    return m


def blur(fan: Fan, phys: Physics, img: np.ndarray, transpose: bool = False) -> np.ndarray:
    x = np.ascontiguousarray(img, dtype=np.float64).reshape(fan.n_rays, fan.n_samples)
    out = np.zeros_like(x)
    cf, cp = fan.c(), phys.c()
    fn = lib().orc_blur_T if transpose else lib().orc_blur
    fn(ctypes.byref(cf), ctypes.byref(cp), _dp(x), _dp(out))
    return out


def blur_radius(phys: Physics, S: int, k: int) -> int:
    cp = phys.c()
    return int(lib().orc_blur_radius(ctypes.byref(cp), ctypes.c_int(S), ctypes.c_int(k)))


# --------------------------------------------------------------------------
# Dense form of the paper's system (Sec. 2.3, Eq. 3-4), pins on tiny rays
# --------------------------------------------------------------------------
def dense_system(Zs, a: float = 1.0, refl_mode: int = REFL_ABS):
    """A (2N+2 x 2N+2) and b for N = len(Zs)-1 interfaces, unknowns
    x = [g_0, d_0, ..., g_N, d_N] (Eq. 3).  Entries as in Eq. 4; with an
    in-system attenuation a != 1 the cross-step couplings carry a (one step)
    or a^2 (a round trip over one step)."""
    Zs = np.asarray(Zs, dtype=np.float64)
    N = len(Zs) - 1
    n = 2 * N + 2
    A = np.zeros((n, n))
    A[0, 0] = 1.0
    A[n - 1, n - 1] = 1.0
    for i in range(N):
        R, Rb, T, Tb = coeffs(Zs[i], Zs[i + 1], refl_mode)
        A[2 * i + 1, 2 * i] = -R
        A[2 * i + 1, 2 * i + 1] = 1.0
        A[2 * i + 1, 2 * i + 3] = -a * Tb
        A[2 * i + 2, 2 * i] = -a * T
        A[2 * i + 2, 2 * i + 2] = 1.0
        A[2 * i + 2, 2 * i + 3] = -a * a * Rb
    b = np.zeros(n)
    b[0] = 1.0
    return A, b


def echo_dense(Zs, a: float = 1.0, refl_mode: int = REFL_ABS):
    """d_0^(k) for k = 0..S-1 from a dense LAPACK solve of the depth-k system."""
    Zs = np.asarray(Zs, dtype=np.float64)
    out = np.zeros(len(Zs))
    for k in range(1, len(Zs)):
        A, b = dense_system(Zs[: k + 1], a, refl_mode)
        x = np.linalg.solve(A, b)
        out[k] = x[1]
    return out


def echo_paths(Zs, a: float = 1.0, refl_mode: int = REFL_ABS, n_terms: int = 200):
    """d_0 of the full ray as the Neumann series x = sum_n (I - A)^n b, i.e. the
    sum over all scattering paths of up to n_terms interface events."""
    A, b = dense_system(Zs, a, refl_mode)
    Sm = np.eye(A.shape[0]) - A
    x = np.zeros_like(b)
    term = b.copy()
    for _ in range(n_terms):
        x += term
        term = Sm @ term
    return x[1], float(np.max(np.abs(np.linalg.eigvals(Sm))))


# --------------------------------------------------------------------------
# Finite differences of the rendered MSE loss (pins of the adjoint)
# --------------------------------------------------------------------------
def loss(vol: Volume, pose, fan: Fan, phys: Physics, target: np.ndarray) -> float:
    img = render(vol, pose, fan, phys)
    d = img - target
    return float(np.mean(d * d))


def _central(f, h: float, richardson: bool) -> float:
    """Central difference of f at 0 with step h; with richardson, the
    extrapolation (4 D(h/2) - D(h)) / 3, exact to O(h^4)."""
    d1 = (f(h) - f(-h)) / (2 * h)
    if not richardson:
        return d1
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3


def fd_pose(vol: Volume, pose, fan: Fan, phys: Physics, target: np.ndarray,
            h_t: float = 1e-4, h_w: float = 1e-6, richardson: bool = False) -> np.ndarray:
    p = _pose(pose)
    target = np.asarray(target, dtype=np.float64).reshape(fan.n_rays, fan.n_samples)
    g = np.zeros(6)
    for i in range(6):
        def f(d, i=i):
            q = p.copy()
            q[i] += d
            return loss(vol, q, fan, phys, target)
        g[i] = _central(f, h_t if i < 3 else h_w, richardson)
    return g


def fd_voxels(vol: Volume, pose, fan: Fan, phys: Physics, target: np.ndarray, flat_idx,
              h: float = 1e-6, richardson: bool = False) -> np.ndarray:
    out = np.zeros(len(flat_idx))
    flat = vol.Z.reshape(-1)
    target = np.asarray(target, dtype=np.float64).reshape(fan.n_rays, fan.n_samples)
    for n, i in enumerate(flat_idx):
        z0 = flat[i]

        def f(d):
            flat[i] = z0 + d
            try:
                return loss(vol, pose, fan, phys, target)
            finally:
                flat[i] = z0
        out[n] = _central(f, h, richardson)
    return out
