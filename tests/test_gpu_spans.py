"""Several wavefronts per long ray (the schedule's ``span_samples``).

Rays of at least ``span_samples`` samples are walked by several wavefronts
that take consecutive tiles of the ray together (the forward, and the fused
step's adjoint, which has the forward's carry records).  The state carried
into each tile, and the adjoint carried out of it, are pushed through the
other tiles' scan totals with the operations a single wavefront uses, so:

* images, per-sample dL/dZ and (in the deterministic plan) dL/dZ are the
  same bit for bit with and without spans; pose gradients differ only in
  the order of their FP64 sums;
* a batch of long rays (16384 and 5000 samples, whose carried vector falls
  through several powers of two) and short ones matches the oracle at every
  pairing of forward and adjoint tiles.
"""
import numpy as np
import pytest

from paper_2508_06768_amd import synth
from tests import helpers as H
from tests.test_gpu_parity import _check_images, _check_plan, _plan_reference, _run_plan, ragged_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def long_column_case(refl, effects, seed=31) -> synth.Case:
    """A 2100 x 8 x 8 column of independent uniform voxels (U(1.4, 1.8)
    |R| convention, U(1, 3) signed) crossed lengthwise: 3 rays of 16384
    samples at 0.125 voxel, 5 of 5000 at 0.4, 7 of 300 at 1 voxel."""
    rng = np.random.default_rng(seed)
    lo, hi = (1.4, 1.8) if refl == 0 else (1.0, 3.0)
    Z = rng.uniform(lo, hi, size=(2100, 8, 8)).astype(np.float32)
    poses = np.array([[3.5, 3.5, 0.0, 0.0, 0.0, 0.0],
                      [3.2, 3.9, 1.0, 0.002, -0.003, 0.1],
                      [3.7, 3.3, 2.0, -0.001, 0.002, -0.2]], dtype=np.float32)
    fans = [synth.FanSpec(3, 16384, 0.01, 0.125, 0.5, 0), synth.FanSpec(5, 5000, 0.02, 0.4, 0.2, 1),
            synth.FanSpec(7, 300, 0.03, 1.0, 0.0, 2)]
    ph = synth.PhysicsSpec(refl_mode=refl, speckle_on=effects, blur_on=effects, seed=seed)
    return synth.Case("long_column", Z, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), poses, fans, ph)


def _gpu(case):
    from paper_2508_06768_amd.render import Geometry
    geom = Geometry(case.Z.shape, case.spacing, case.origin, case.fans, case.phys)
    return (geom, torch.from_numpy(case.Z).to(DEV),
            torch.from_numpy(np.ascontiguousarray(case.poses, dtype=np.float32)).to(DEV))


@pytest.mark.parametrize("refl,effects", [(0, False), (1, True)])
def test_long_rays_match_oracle(refl, effects):
    case = long_column_case(refl, effects)
    print("case", case.name, "refl", refl, "effects", effects, flush=True)
    target = H.oracle_render(case, poses=case.poses + np.float32([[0.1, -0.1, 0.3, 0.0, 0.0, 0.0]]))
    ref = _plan_reference(case, target)
    for fc, bc in ((8, 4), (16, 8), (4, 4)):
        sched = {"fwd_chunk": fc, "bwd_chunk": bc, "xcd_group": 1}
        _check_plan(case, _run_plan(case, target, sched, replays=2), ref, f"long rays fwd {fc} bwd {bc}")


def _det_step(case, target, span, fc=8, bc=4, one_stream=False):
    from paper_2508_06768_amd.render import FusedStep
    geom, Z, P = _gpu(case)
    T = torch.from_numpy(target.astype(np.float32)).to(DEV)
    step = FusedStep(geom, zero_grad_z=True, deterministic=True, one_stream=one_stream,
                     schedule={"fwd_chunk": fc, "bwd_chunk": bc, "span_samples": span})
    bm = torch.empty(geom.total, device=DEV)
    gZ = torch.empty_like(Z)
    gp = torch.empty((geom.n_poses, 6), device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    for _ in range(2):
        step.step(Z, P, T, bmode=bm, loss=loss, grad_Z=gZ, grad_pose=gp)
    torch.cuda.synchronize()
    step.close()
    return bm.cpu().numpy(), loss.item(), gZ.cpu().numpy(), gp.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("which", ["ragged", "long"])
@pytest.mark.parametrize("fc,bc", [(8, 4), (16, 8)])
def test_spans_bit_identical(which, fc, bc):
    """Every ray walked by several wavefronts (span_samples = 1, idle
    wavefronts on short rays) against none (-1)."""
    case = ragged_case(0, 0, True, seed=33) if which == "ragged" else long_column_case(0, True, seed=35)
    print("case", case.name, "fwd", fc, "bwd", bc, flush=True)
    target = H.oracle_render(case, poses=case.poses + np.float32([[0.2, 0.1, -0.1, 0.01, 0.0, 0.0]]))
    a = _det_step(case, target, 1, fc, bc)
    b = _det_step(case, target, -1, fc, bc)
    np.testing.assert_array_equal(a[0], b[0])
    assert a[1] == b[1]                       # the loss comes from the blur kernel
    np.testing.assert_array_equal(a[2], b[2])
    np.testing.assert_allclose(a[3], b[3], rtol=1e-10, atol=1e-12 * np.abs(b[3]).max())
    img, ref_loss, rV, rp = _plan_reference(case, target)
    _check_plan(case, (a[0], a[1], a[2], a[3]), (img, ref_loss, rV, rp), f"spans {which}")


def test_spans_on_one_stream():
    """A plan held to one stream launches the long rays' wavefronts on the
    step's stream, after the others: the same images and dL/dZ bit for bit
    as the default plan, whose second stream takes them."""
    case = long_column_case(1, True, seed=39)
    target = H.oracle_render(case, poses=case.poses + np.float32([[-0.2, 0.1, 0.2, 0.0, 0.01, 0.0]]))
    a = _det_step(case, target, 0)
    b = _det_step(case, target, 0, one_stream=True)
    np.testing.assert_array_equal(a[0], b[0])
    assert a[1] == b[1]
    np.testing.assert_array_equal(a[2], b[2])
    np.testing.assert_array_equal(a[3], b[3])


def test_spans_forward_render_bit_identical():
    """The direct render takes the process-wide schedule: the same images
    with spans everywhere, at the default length, and never."""
    from paper_2508_06768_amd.render import get_schedule, render, set_schedule
    case = long_column_case(1, True, seed=37)
    geom, Z, P = _gpu(case)
    old = get_schedule()
    try:
        imgs = []
        for span in (1, 0, -1):
            set_schedule(**dict(old, span_samples=span))
            imgs.append(render(Z, P, geom).cpu().numpy())
    finally:
        set_schedule(**old)
    np.testing.assert_array_equal(imgs[0], imgs[2])
    np.testing.assert_array_equal(imgs[1], imgs[2])
    _check_images(imgs[1], H.oracle_render(case), "render with spans", case.fans)


def test_schedule_change_regroups_the_plan():
    """A plan with long rays runs one chain (their launches take the second
    stream); with span_samples = -1 it has no long rays and regroups its
    fans into two chains, in the same workspace.  Images stay the same bit
    for bit, the loss and the gradients within their rounding."""
    from paper_2508_06768_amd import _lib
    from paper_2508_06768_amd.render import FusedStep
    case = long_column_case(0, True, seed=41)
    geom, Z, P = _gpu(case)
    target = H.oracle_render(case, poses=case.poses + np.float32([[0.1, 0.1, 0.1, 0.0, 0.0, 0.01]]))
    T = torch.from_numpy(target.astype(np.float32)).to(DEV)
    step = FusedStep(geom, zero_grad_z=True)
    ws_bytes = _lib.lib().dus_plan_workspace_bytes(step._h)
    out = []
    for span in (0, -1, 0):
        step.set_schedule(span_samples=span)
        assert _lib.lib().dus_plan_workspace_bytes(step._h) == ws_bytes
        bm = torch.empty(geom.total, device=DEV)
        gZ = torch.empty_like(Z)
        gp = torch.empty((geom.n_poses, 6), device=DEV)
        loss = torch.zeros(1, dtype=torch.float64, device=DEV)
        for _ in range(2):
            step.step(Z, P, T, bmode=bm, loss=loss, grad_Z=gZ, grad_pose=gp)
        torch.cuda.synchronize()
        out.append((bm.cpu().numpy(), loss.item(), gZ.cpu().numpy().astype(np.float64), gp.cpu().numpy().astype(np.float64)))
    step.close()
    for o in out[1:]:
        np.testing.assert_array_equal(o[0], out[0][0])
        assert o[1] == pytest.approx(out[0][1], rel=1e-12)
        assert H.rel_l2(o[2], out[0][2]) <= 1e-6
        np.testing.assert_allclose(o[3], out[0][3], rtol=1e-9, atol=1e-12 * np.abs(out[0][3]).max())
    img, ref_loss, rV, rp = _plan_reference(case, target)
    _check_plan(case, out[1], (img, ref_loss, rV, rp), "regrouped plan")
