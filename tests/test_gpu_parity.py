"""GPU parity: the HIP renderer (through the C ABI) against the FP64 oracle.

Bars:
  forward images      per-image relative l2 <= 1e-5, and every pixel within
                      1e-5 of the image's max |value|
  adjoint             dL/dZ relative l2 <= 1e-5 over the volume, and every
                      voxel within 1e-5 of max |dL/dZ|; dL/dpose per
                      component within 1e-5 * ||dL/dpose||
  speckle generator   Philox words bit-exact
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_06768_amd import synth
from tests import helpers as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
RTOL_IMG = 1e-5
RTOL_GRAD = 1e-5


def _gpu(case, geom=None):
    from paper_2508_06768_amd.render import Geometry
    geom = geom or Geometry(case.Z.shape, case.spacing, case.origin, case.fans, case.phys)
    Z = torch.from_numpy(case.Z).to(DEV)
    poses = torch.from_numpy(np.ascontiguousarray(case.poses, dtype=np.float32)).to(DEV)
    return geom, Z, poses


def ragged_case(refl=0, atten=0, effects=False, seed=7) -> synth.Case:
    """48^3 brain-like volume; three tilted poses whose fans span several
    tiles with ragged tails, a single-ray fan and a short fan."""
    Z = synth.brain_volume(seed, 48, 1.0, semi_range=(3.0, 10.0))
    rng = np.random.default_rng(seed)
    poses = np.array([[23.5, 24.0, 0.0, 0.05, -0.04, 0.1],
                      [20.0, 26.0, 1.5, -0.12, 0.08, -0.3],
                      [25.0, 22.0, 0.5, 0.2, 0.1, 0.7]], dtype=np.float32)
    fans = [synth.FanSpec(37, 1000, 1.1, 0.047, 0.3, 0),
            synth.FanSpec(1, 777, 0.0, 0.061, 0.0, 1),
            synth.FanSpec(65, 129, 1.4, 0.33, 1.0, 2)]
    ph = synth.PhysicsSpec(refl_mode=refl, atten_mode=atten, speckle_on=effects, blur_on=effects,
                           seed=int(rng.integers(1 << 40)), alpha=0.8, freq=4.0)
    return synth.Case("ragged48", Z, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), poses, fans, ph)


def coarse_case(seed=5, ds=3.0) -> synth.Case:
    """Coarse depth steps.  The scatter takes 4, 2 or 1 depths per lane as
    the step grows (0.35 and 0.7 voxel the thresholds); at 3 voxels per
    sample even its groups of 8 depths do not fit the LDS box and take the
    per-sample atomic path; at 0.5 and 1 voxel (the paper's one sample per
    voxel) the box takes groups of 16 and 8 depths."""
    Z = synth.brain_volume(seed, 40, 1.0, semi_range=(3.0, 9.0))
    poses = np.array([[19.5, 18.0, 0.0, 0.3, -0.2, 0.1]], dtype=np.float32)
    fans = [synth.FanSpec(9, max(int(100 * 1.2 / ds), 20), 0.6, ds, 0.0, 0)]
    ph = synth.PhysicsSpec(seed=seed, speckle_on=True)
    return synth.Case("coarse40", Z, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), poses, fans, ph)


def _check_images(gpu, ref, tag, fans=None):
    rep = H.parity_report(gpu, ref, fans)
    print(tag, rep, flush=True)
    assert rep["rel_l2"] <= RTOL_IMG, rep
    assert rep["max_abs_over_max"] <= RTOL_IMG, rep


def check_grad_volume(gZ, rV, tag):
    """dL/dZ against the oracle: relative l2 over the volume and the largest
    voxel error over the largest |dL/dZ| (the elementwise bar)."""
    rep = H.grad_report(gZ, rV)
    print(tag, "dZ", rep, flush=True)
    assert rep["rel_l2"] <= RTOL_GRAD, rep
    assert rep["max_abs_over_max"] <= RTOL_GRAD, rep


def check_grad_pose(gp, rp, tag):
    """Every pose's gradient: each component within 1e-5 of the norm of the
    oracle's gradient of that pose."""
    worst = 0.0
    for p in range(len(rp)):
        nrm = np.linalg.norm(rp[p])
        err = float(np.abs(gp[p] - rp[p]).max())
        worst = max(worst, err / nrm if nrm > 0 else err)
        assert np.all(np.abs(gp[p] - rp[p]) <= RTOL_GRAD * nrm + 1e-30), (tag, p, gp[p], rp[p])
    print(tag, "pose worst |error| / |gradient|", worst, flush=True)


# --------------------------------------------------------------------------
def test_philox_bitexact():
    from oracle import oracle as O
    from paper_2508_06768_amd.render import philox
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x0123456789ABCDEF
    out = philox(torch.from_numpy(ctr.view(np.int32)).to(DEV), seed).cpu().numpy().view(np.uint32)
    ref = O.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32])
    np.testing.assert_array_equal(out, ref)
    # and the generator's published known-answer vectors
    from tests.test_oracle_pins import philox_kat
    kc, kk, kr = philox_kat()
    for c, k, r in zip(kc, kk, kr):
        got = philox(torch.from_numpy(c[None].copy().view(np.int32)).to(DEV), int(k[0]) | (int(k[1]) << 32))
        np.testing.assert_array_equal(got.cpu().numpy().view(np.uint32).reshape(-1), r)


@pytest.mark.parametrize("atten", [0, 1])
def test_pixel_gain_matches_oracle(atten):
    from oracle import oracle as O
    from paper_2508_06768_amd.render import pixel_gain
    fan = synth.FanSpec(5, 1037, 1.0, 0.21, 0.0, 9)
    ph = synth.PhysicsSpec(speckle_on=True, atten_mode=atten, seed=12345, spk_cell=8)
    g = pixel_gain(fan, ph, DEV).cpu().numpy()
    of = H.oracle_fan(fan)
    op = H.oracle_physics(ph)
    ref = np.stack([O.speckle_ray(of, op, j) for j in range(5)])
    if atten == 1:
        k = np.arange(1037)
        ref = ref * 10 ** (-2 * op.alpha * op.freq * (k * of.ds / 10) / 20)
    np.testing.assert_allclose(g, ref, rtol=2e-6, atol=0)


@pytest.mark.parametrize("refl,atten,effects", [(0, 0, False), (1, 0, False), (0, 1, True), (1, 2, True),
                                                (0, 0, True)])
def test_forward_parity_ragged(refl, atten, effects):
    from paper_2508_06768_amd.render import render
    case = ragged_case(refl, atten, effects)
    geom, Z, poses = _gpu(case)
    img, piv = render(Z, poses, geom, want_pivot=True)
    ref, rpiv = H.oracle_render(case, want_pivot=True)
    _check_images(img.cpu().numpy(), ref, f"ragged refl={refl} atten={atten} fx={effects}", case.fans)
    np.testing.assert_allclose(piv.cpu().numpy(), rpiv, rtol=1e-5)


def test_forward_parity_phantom():
    """64^3 phantom, 64 rays x 256 samples (near-pole rays included)."""
    from paper_2508_06768_amd.render import render
    case = synth.case_small_forward()
    geom, Z, poses = _gpu(case)
    img, piv = render(Z, poses, geom, want_pivot=True)
    ref, rpiv = H.oracle_render(case, want_pivot=True)
    _check_images(img.cpu().numpy(), ref, "phantom64", case.fans)
    np.testing.assert_allclose(piv.cpu().numpy(), rpiv, rtol=1e-5)


def test_homogeneous_volume_is_exactly_silent():
    from paper_2508_06768_amd.render import render
    case = ragged_case(0, 0, True)
    case.Z = np.full_like(case.Z, 1.61)
    geom, Z, poses = _gpu(case)
    img = render(Z, poses, geom).cpu().numpy()
    assert np.all(img == 0.0)


@pytest.mark.parametrize("refl,effects", [(0, False), (1, True), (0, True), ("coarse", 3.0), ("coarse", 1.0),
                                          ("coarse", 0.5)])
def test_backward_parity_ragged(refl, effects):
    from paper_2508_06768_amd.render import render_backward
    case = coarse_case(ds=effects) if refl == "coarse" else ragged_case(refl, 0, effects, seed=11)
    geom, Z, poses = _gpu(case)
    rng = np.random.default_rng(3)
    w = rng.standard_normal(geom.total).astype(np.float32)
    gZ, gp = render_backward(Z, poses, geom, torch.from_numpy(w).to(DEV))
    rV, rp = H.oracle_backward(case, w.astype(np.float64))
    check_grad_volume(gZ.cpu().numpy(), rV, f"backward {refl} fx={effects}")
    check_grad_pose(gp.cpu().numpy(), rp, f"backward {refl} fx={effects}")


def _plan_reference(case, target, want_volume=True):
    """Oracle image, MSE loss (mean per fan, summed over fans), dL/dZ (None
    without want_volume) and dL/dpose of the fused step."""
    img = H.oracle_render(case)
    tf = target.astype(np.float32).astype(np.float64)
    ref_loss = 0.0
    grad = np.zeros_like(img)
    off = 0
    for f in case.fans:
        n = f.n_rays * f.n_samples
        if n == 0:
            continue                            # an empty fan adds nothing
        d = img[off:off + n] - tf[off:off + n]
        ref_loss += np.mean(d * d)
        grad[off:off + n] = 2 * d / n
        off += n
    rV, rp = H.oracle_backward(case, grad, want_volume=want_volume)
    return img, ref_loss, rV, rp


def _run_plan(case, target, schedule=None, replays=3, image=True, pose_only=False):
    from paper_2508_06768_amd.render import FusedStep
    geom, Z, poses = _gpu(case)
    T = torch.from_numpy(target.astype(np.float32)).to(DEV)
    step = FusedStep(geom, zero_grad_z=not pose_only, pose_only=pose_only, schedule=schedule)
    bm = torch.empty(geom.total, device=DEV) if image else None
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    gZ = None if pose_only else torch.full_like(Z, 123.0)
    gp = torch.empty((geom.n_poses, 6), device=DEV)
    for _ in range(replays):                    # replays of the same graph
        step.step(Z, poses, T, bmode=bm, loss=loss, grad_Z=gZ, grad_pose=gp)
    torch.cuda.synchronize()
    out = (bm.cpu().numpy() if image else None, loss.item(), None if gZ is None else gZ.cpu().numpy(),
           gp.cpu().numpy())
    step.close()
    return out


def _check_plan(case, got, ref, tag):
    bm, loss, gZ, gp = got
    img, ref_loss, rV, rp = ref
    if bm is not None:
        _check_images(bm, img, f"{tag} image", case.fans)
    print(tag, "loss", loss, ref_loss, flush=True)
    assert loss == pytest.approx(ref_loss, rel=1e-5)
    if rV is not None:
        check_grad_volume(gZ, rV, tag)
    check_grad_pose(gp, rp, tag)


def test_fused_plan_matches_oracle():
    """dus_plan step (forward + MSE + adjoint in one captured graph)."""
    for effects in (False, True):
        case = ragged_case(0, 0, effects, seed=21)
        tgt_poses = case.poses + np.float32([[0.6, -0.3, 0.2, 0.02, -0.03, 0.05]])
        target = H.oracle_render(case, poses=tgt_poses)
        _check_plan(case, _run_plan(case, target), _plan_reference(case, target), f"plan fx={effects}")


def test_fused_plan_without_image():
    """No blur and no image requested: the forward kernel does not run, and
    the fused adjoint forms the residual and the loss itself, starting from
    its own forward sweep (no carries or chunk states)."""
    case = ragged_case(1, 0, False, seed=23)
    target = H.oracle_render(case, poses=case.poses + np.float32([[0.5, 0.2, -0.3, 0.0, 0.03, 0.0]]))
    _check_plan(case, _run_plan(case, target, image=False), _plan_reference(case, target), "plan, no image")


def test_plan_with_two_fan_tables():
    """70 fans: more than one launch table (64 fans each), so the tables'
    carry records, loss partials and per-ray pose partials sit at offsets.
    The fused step (with blur) and render + adjoint against the oracle."""
    from paper_2508_06768_amd.render import render, render_backward
    Z = synth.brain_volume(17, 40, 1.0, semi_range=(3.0, 9.0))
    rng = np.random.default_rng(17)
    P = 70
    poses = np.concatenate([rng.uniform(14.0, 25.0, (P, 2)), rng.uniform(0.0, 2.0, (P, 1)),
                            rng.uniform(-0.2, 0.2, (P, 3))], axis=1).astype(np.float32)
    fans = [synth.FanSpec(int(rng.integers(1, 9)), int(rng.integers(20, 300)), 0.8, 0.13, 0.0, p) for p in range(P)]
    for effects in (False, True):
        case = synth.Case("tables70", Z, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), poses, fans,
                          synth.PhysicsSpec(speckle_on=effects, blur_on=effects, seed=17))
        target = H.oracle_render(case, poses=case.poses + np.float32([[0.4, -0.3, 0.2, 0.01, 0.0, -0.02]]))
        _check_plan(case, _run_plan(case, target, replays=2), _plan_reference(case, target), f"70 fans fx={effects}")
        geom, Zt, Pt = _gpu(case)
        _check_images(render(Zt, Pt, geom).cpu().numpy(), H.oracle_render(case), "70 fans render", case.fans)
        w = rng.standard_normal(geom.total).astype(np.float32)
        gZ, gp = render_backward(Zt, Pt, geom, torch.from_numpy(w).to(DEV))
        rV, rp = H.oracle_backward(case, w.astype(np.float64))
        check_grad_volume(gZ.cpu().numpy(), rV, f"70 fans backward fx={effects}")
        check_grad_pose(gp.cpu().numpy(), rp, f"70 fans backward fx={effects}")


def rough_column_case(refl, effects, seed=13) -> synth.Case:
    """A 1100 x 8 x 8 column of independent uniform voxels crossed one voxel
    per sample (U(1.4, 1.8) in the |R| convention, U(1, 3) signed): every
    interface reflects, and with the attenuation the largest entry of the
    carried row vector drops through several powers of two along a ray, so
    the forward's carry records and chunk states hold exponents that the
    adjoint must undo.  All pivots stay above 0.9.  Fans of 1000 and 777
    samples."""
    rng = np.random.default_rng(seed)
    lo, hi = (1.4, 1.8) if refl == 0 else (1.0, 3.0)
    Z = rng.uniform(lo, hi, size=(1100, 8, 8)).astype(np.float32)
    poses = np.array([[3.5, 3.5, 0.0, 0.0, 0.0, 0.0],
                      [3.2, 3.9, 1.0, 0.002, -0.003, 0.1]], dtype=np.float32)
    fans = [synth.FanSpec(3, 1000, 0.02, 1.0, 0.5, 0), synth.FanSpec(2, 777, 0.01, 1.0, 0.2, 1)]
    ph = synth.PhysicsSpec(refl_mode=refl, speckle_on=effects, blur_on=effects, seed=seed)
    return synth.Case("column", Z, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), poses, fans, ph)


@pytest.mark.parametrize("refl,effects", [(0, False), (1, True)])
def test_plan_schedules_with_renormalised_carries(refl, effects):
    """The forward hands the adjoint its tile carries and chunk states in
    the frames of its own tiles.  Every pairing of forward tile (4, 8, 16
    samples per lane) and adjoint tile (4, 8) must give the oracle's image,
    loss and gradients on rays whose carried vector is renormalised."""
    case = rough_column_case(refl, effects)
    # premise: the power of two of the carried vector changes from one
    # 256-sample block to the next (products of the Eq. 2-4 transfer maps
    # over the oracle's samples of the first ray)
    Zs = O.ray_samples(H.oracle_volume(case), case.poses[0].astype(np.float64), H.oracle_fan(case.fans[0]), 1)
    a2 = O.step_amplitude(H.oracle_physics(case.phys), case.fans[0].ds) ** 2
    sgn = 1.0 if refl == 0 else -1.0
    v = np.array([0.0, 1.0])
    ex = []
    for i in range(1, len(Zs)):
        r = O.coeffs(Zs[i - 1], Zs[i], refl)[0]
        v = v @ np.array([[a2 * (1.0 - r * r - sgn * r * r), r], [-a2 * sgn * r, 1.0]])
        if (i + 1) % 256 == 0:
            ex.append(int(np.floor(np.log2(np.abs(v).max()))))
    assert len(set(ex)) >= 2 and min(ex) < 0, ex
    tgt_poses = case.poses + np.float32([[0.1, -0.1, 0.0, 0.0, 0.0, 0.0]])
    target = H.oracle_render(case, poses=tgt_poses)
    ref = _plan_reference(case, target)
    for fc in (4, 8, 16):
        for bc in (4, 8):
            sched = {"fwd_chunk": fc, "bwd_chunk": bc, "xcd_group": 1, "scatter_rays": 2}
            _check_plan(case, _run_plan(case, target, sched, replays=2), ref, f"column fwd {fc} bwd {bc}")


# --------------------------------------------------------------------------
# display and ablation modes
# --------------------------------------------------------------------------
def test_sample_volume_matches_oracle():
    """Sampling-only render (impedance at every ray sample) on the ragged
    fans, including a single-ray fan and samples outside the volume."""
    from oracle import oracle as O
    from paper_2508_06768_amd.render import sample_volume
    case = ragged_case(0, 0, False, seed=51)
    geom, Z, poses = _gpu(case)
    out = sample_volume(Z, poses, geom).cpu().numpy().astype(np.float64)
    vol = H.oracle_volume(case)
    off = 0
    for p, f in enumerate(case.fans):
        n = f.n_rays * f.n_samples
        ref = O.sample_image(vol, case.poses[p].astype(np.float64), H.oracle_fan(f)).reshape(-1)
        np.testing.assert_allclose(out[off:off + n], ref, rtol=2e-7, atol=0)
        off += n


def test_scan_convert_matches_oracle():
    """Scan conversion of a rendered fan onto a grid that covers the fan, its
    apex region and pixels outside it."""
    from oracle import oracle as O
    from paper_2508_06768_amd.render import scan_convert
    case = ragged_case(0, 0, True, seed=52)
    geom, _, _ = _gpu(case)
    # the oracle's render, rounded to FP32, is the input of both sides
    img32 = H.oracle_render(case).astype(np.float32)
    img = torch.from_numpy(img32).to(DEV)
    for p, (nx, nz, x0, z0, dx, dz) in [(0, (97, 83, -31.7, -2.3, 0.61, 0.67)), (2, (64, 64, -40.1, -1.9, 1.43, 0.77))]:
        f = case.fans[p]
        out = scan_convert(img, geom, p, nx, nz, x0, z0, dx, dz, fill=-1.0).cpu().numpy()
        src = img32[geom.offsets[p]:geom.offsets[p + 1]].astype(np.float64)
        # the grid travels as FP32: the oracle takes the same values
        g32 = [float(np.float32(a)) for a in (x0, z0, dx, dz)]
        ref = O.scan_convert(src, H.oracle_fan(f), nx, nz, *g32, fill=-1.0)
        assert (ref != -1.0).sum() > 100 and (ref == -1.0).sum() > 100
        np.testing.assert_array_equal(out == -1.0, ref == -1.0)
        scale = np.abs(ref[ref != -1.0]).max()
        np.testing.assert_allclose(out, ref, rtol=0, atol=1e-6 * scale)


# --------------------------------------------------------------------------
# volume reconstruction helpers
# --------------------------------------------------------------------------
def test_smoothness_matches_oracle():
    """Smoothness prior on a 37 x 23 x 19 volume (partial blocks), anisotropic
    spacing: gradient added to an existing grad_Z, energy added to a loss."""
    from oracle import oracle as O
    from paper_2508_06768_amd.render import Geometry, smoothness
    rng = np.random.default_rng(61)
    Zn = (1.5 + 0.1 * rng.standard_normal((19, 23, 37))).astype(np.float32)
    h = (0.8, 1.1, 1.3)
    geom = Geometry(Zn.shape, h, (0.0, 0.0, 0.0), [], synth.PhysicsSpec())
    Z = torch.from_numpy(Zn).to(DEV)
    g0 = rng.standard_normal(Zn.shape).astype(np.float32)
    gZ = torch.from_numpy(g0).to(DEV)
    loss = torch.full((1,), 0.5, dtype=torch.float64, device=DEV)
    smoothness(Z, geom, 0.37, gZ, loss)
    R, g = O.smoothness(Zn.astype(np.float64), tuple(float(np.float32(x)) for x in h), float(np.float32(0.37)))
    assert loss.item() - 0.5 == pytest.approx(R, rel=1e-6)
    np.testing.assert_allclose(gZ.cpu().numpy() - g0, g, rtol=0, atol=1e-5 * np.abs(g).max())


def test_adam_matches_oracle():
    from oracle import oracle as O
    from paper_2508_06768_amd.render import adam_step
    rng = np.random.default_rng(62)
    n = 100003
    x0, g, m0 = (rng.standard_normal(n).astype(np.float32) for _ in range(3))
    v0 = np.abs(rng.standard_normal(n)).astype(np.float32)
    x, gg, m, v = (torch.from_numpy(a.copy()).to(DEV) for a in (x0, g, m0, v0))
    hyper = (0.01, 0.9, 0.999, 1e-8, -1.5, 2.5)
    adam_step(x, gg, m, v, 7, *hyper)
    # the hyperparameters travel as FP32: the oracle takes the same values
    rx, rm, rv = O.adam(x0, g, m0, v0, 7, *(float(np.float32(a)) for a in hyper))
    np.testing.assert_allclose(m.cpu().numpy(), rm, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(v.cpu().numpy(), rv, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(x.cpu().numpy(), rx, rtol=1e-6, atol=1e-6)


# --------------------------------------------------------------------------
# impedance mapping (Sec. 2.2)
# --------------------------------------------------------------------------
def test_map_impedance_matches_oracle():
    """Piecewise-linear intensity -> impedance table: values, dL/dintensity
    and dL/dz_j against the oracle on intensities below, inside and above
    the table and exactly at its knots (FP32 arithmetic on the GPU)."""
    from oracle import oracle as O
    from paper_2508_06768_amd.render import map_impedance, map_impedance_backward
    rng = np.random.default_rng(31)
    xk = np.cumsum(rng.uniform(20.0, 200.0, 12)).astype(np.float32) - 500.0   # CT-like numbers
    zk = rng.uniform(1.3, 7.8, 12).astype(np.float32)
    v = rng.uniform(float(xk[0]) - 100.0, float(xk[-1]) + 100.0, 300_001).astype(np.float32)
    v[:12] = xk
    gZ = rng.standard_normal(v.size).astype(np.float32)
    I = torch.from_numpy(v).to(DEV)
    Zg = map_impedance(I, xk, zk).cpu().numpy().astype(np.float64)
    gi, gz = map_impedance_backward(I, xk, zk, torch.from_numpy(gZ).to(DEV))
    Zr, _ = O.map_impedance(v.astype(np.float64), xk.astype(np.float64), zk.astype(np.float64))
    gir, gzr = O.map_impedance_grad(v.astype(np.float64), xk.astype(np.float64), zk.astype(np.float64),
                                    gZ.astype(np.float64))
    tol = 8 * np.finfo(np.float32).eps
    assert np.all(np.abs(Zg - Zr) <= tol * np.abs(zk).max())
    gin = gi.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(gin - gir) <= tol * np.abs(gir).max())
    np.testing.assert_allclose(gz.cpu().numpy(), gzr, rtol=1e-5, atol=1e-6 * np.abs(gzr).max())

