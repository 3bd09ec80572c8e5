"""GPU checks at the benchmark's full sizes and on the edge cases.

* the 512 x 1024 adjoint workload: GPU gradients against the FP64 oracle's
  adjoint (rel. 1e-5) and against FP64 central finite differences of the
  oracle's forward (64 footprint voxels, 8 voxels outside it, all 6 pose
  parameters) within 1e-3;
* the uneven 64-pose batch: batched launch == one pose per launch, and
  sampled poses against the oracle;
* the benchmark's own fused step (64 x 256 x 1024, effects on, graph
  replay, default and tuned schedules): all images, the loss, dL/dZ and all
  pose gradients against the oracle;
* every schedule gives the same result; graph replays agree;
* maximum sample count, single ray, single sample, empty fans, 2-voxel axes.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_06768_amd import synth
from tests import helpers as H
from tests.test_gpu_parity import _check_plan, _plan_reference, _run_plan, check_grad_pose, check_grad_volume

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _gpu(case, fans=None, poses=None):
    from paper_2508_06768_amd.render import Geometry
    fans = case.fans if fans is None else fans
    poses = case.poses if poses is None else poses
    geom = Geometry(case.Z.shape, case.spacing, case.origin, fans, case.phys)
    return (geom, torch.from_numpy(case.Z).to(DEV),
            torch.from_numpy(np.ascontiguousarray(poses, dtype=np.float32)).to(DEV))


def test_adjoint_full_size_vs_oracle_and_finite_differences():
    from paper_2508_06768_amd.render import render, render_backward
    case = synth.case_adjoint()
    geom, Z, P = _gpu(case)
    print("case", case.name, "rays", case.fans[0].n_rays, "samples", case.fans[0].n_samples, flush=True)
    target = H.oracle_render(case, poses=case.extra["target_poses"])
    tf = target.astype(np.float32).astype(np.float64)
    img = render(Z, P, geom)
    ref = H.oracle_render(case)
    rep = H.parity_report(img.cpu().numpy(), ref, case.fans)
    print("forward", rep, flush=True)
    assert rep["rel_l2"] <= 1e-5 and rep["max_abs_over_max"] <= 1e-5
    # MSE gradient of the GPU image, adjoint on the GPU
    n = ref.size
    gimg = 2.0 * (img.double() - torch.from_numpy(tf).to(DEV)) / n
    gZ, gp = render_backward(Z, P, geom, gimg.float())
    gZ = gZ.cpu().numpy().astype(np.float64)
    gp = gp.cpu().numpy()[0].astype(np.float64)
    # FP64 oracle adjoint with its own image
    _, g_or = O.mse_loss_grad(ref, tf)
    rV, rp = H.oracle_backward(case, g_or)
    print("pose", gp, rp[0], flush=True)
    check_grad_volume(gZ, rV, "adjoint 512 x 1024")
    check_grad_pose(gp[None], rp, "adjoint 512 x 1024")
    # finite differences of the oracle's forward
    vol = H.oracle_volume(case)
    fan = H.oracle_fan(case.fans[0])
    ph = H.oracle_physics(case.phys)
    pose = case.poses[0].astype(np.float64)
    rng = np.random.default_rng(1003)
    flat = np.abs(rV.reshape(-1))
    hot = np.flatnonzero(flat > 1e-2 * flat.max())
    idx = list(rng.choice(hot, size=64, replace=False))
    cold = np.flatnonzero(flat == 0.0)
    idx_cold = list(rng.choice(cold, size=8, replace=False))
    tf2 = tf.reshape(fan.n_rays, fan.n_samples)
    # the |R| convention puts rays of this workload close to poles of the
    # echo (min pivot 0.02, peak pixel 3e3): the loss is sharply curved, so
    # the differences use small steps with Richardson extrapolation
    fd = O.fd_voxels(vol, pose, fan, ph, tf2, idx + idx_cold, h=2e-7, richardson=True)
    g_sel = gZ.reshape(-1)[idx + idx_cold]
    err = np.abs(g_sel[:64] - fd[:64]) / np.abs(fd[:64])
    print("voxel FD rel err max", err.max(), "median", np.median(err), flush=True)
    assert np.all(g_sel[64:] == 0.0)
    assert np.all(fd[64:] == 0.0)
    assert np.linalg.norm(g_sel[:64] - fd[:64]) <= 1e-3 * np.linalg.norm(fd[:64])
    assert np.all(err <= 1e-3)
    fdp = O.fd_pose(vol, pose, fan, ph, tf2, h_t=2e-7, h_w=2e-9, richardson=True)
    print("pose FD", fdp, "gpu", gp, flush=True)
    assert np.all(np.abs(gp - fdp) <= 1e-3 * np.abs(fdp))


def test_batched_equals_plain_and_oracle():
    """The uneven 64-pose batch in one launch equals one pose per launch, and
    sampled poses (the longest, the widest, two others) match the oracle."""
    from paper_2508_06768_amd.render import Geometry, render, render_backward
    case = synth.case_batched()
    geom, Z, P = _gpu(case)
    print("case", case.name, "ray-samples", case.ray_samples, flush=True)
    img = render(Z, P, geom).cpu().numpy()
    w = np.random.default_rng(4).standard_normal(geom.total).astype(np.float32) * 1e-3
    gZb, gpb = render_backward(Z, P, geom, torch.from_numpy(w).to(DEV))
    gZb = gZb.cpu().numpy()
    gpb = gpb.cpu().numpy()
    gZp = torch.zeros_like(Z)
    for p in range(len(case.fans)):
        g1 = Geometry(case.Z.shape, case.spacing, case.origin, [case.fans[p]], case.phys)
        one = render(Z, P[p:p + 1].contiguous(), g1).cpu().numpy()
        o = geom.offsets
        np.testing.assert_array_equal(one, img[o[p]:o[p + 1]])
        _, gp1 = render_backward(Z, P[p:p + 1].contiguous(), g1, torch.from_numpy(w[o[p]:o[p + 1]]).to(DEV),
                                 grad_Z=gZp)
        np.testing.assert_allclose(gp1.cpu().numpy()[0], gpb[p], rtol=1e-5,
                                   atol=1e-6 * np.abs(gpb[p]).max())
    assert H.rel_l2(gZp.cpu().numpy(), gZb) <= 1e-6
    S = [f.n_samples for f in case.fans]
    R = [f.n_rays * (f.aperture) for f in case.fans]
    picks = sorted({int(np.argmax(S)), int(np.argmax(R)), 7, 33})
    for p in picks:
        sub = synth.Case(case.name, case.Z, case.spacing, case.origin, case.poses[p:p + 1],
                         [case.fans[p]], case.phys)
        ref = H.oracle_render(sub)
        o = geom.offsets
        rep = H.parity_report(img[o[p]:o[p + 1]], ref)
        print("pose", p, case.fans[p], rep, flush=True)
        assert rep["rel_l2"] <= 1e-5 and rep["max_abs_over_max"] <= 1e-5


def test_uneven_batch_fused_step_vs_oracle():
    """The uneven 64-pose batch (128-512 rays x 256-2048 samples, 40-90 deg,
    100-240 mm deep, speckle and blur) as one fused forward + MSE + adjoint
    step replayed from its graph: all 64 images, the loss, dL/dZ over the
    volume and all 64 pose gradients against the FP64 oracle, whose target
    is its own render at the +-5 mm / +-5 deg offset poses."""
    case = synth.case_batched()
    print("case", case.name, "ray-samples", case.ray_samples, flush=True)
    target = H.oracle_render(case, poses=case.extra["target_poses"])
    got = _run_plan(case, target, replays=2)
    print("GPU step done", flush=True)
    _check_plan(case, got, _plan_reference(case, target), "uneven batch")


def registration_shape_case(n_poses=4, n=320):
    """Fans of the registration workload (384 rays x 1536 samples, 70 deg,
    192 mm deep, ds = 0.125 mm) on a volume of 0.5 mm voxels, noise smoothed
    over 4 voxels, speckle and blur: a 320^3 crop of the 512^3 volume's
    extent (160 mm), so part of every ray runs past the volume; apexes and
    tilts drawn as for the registration poses; targets +-1 mm / +-1 deg
    away."""
    h = 0.5
    Z = synth.brain_volume(1005, n, h, noise_sigma_vox=4.0)
    rng = np.random.default_rng(1005)
    gt = synth.random_poses(rng, n_poses, (n - 1) * h)
    init = synth.offset_poses(rng, gt, 1.0, 1.0)
    fans = [synth.FanSpec(384, 1536, 70 * synth.DEG, 192.0 / 1536, 0.0, p) for p in range(n_poses)]
    return synth.Case(f"registration_shape_{n}cube", Z, (h,) * 3, (0.0,) * 3, init, fans,
                      synth.effects_physics(1005), extra={"gt_poses": gt})


def test_pose_only_step_vs_oracle_registration_shape():
    """The pose-only fused step (no dL/dZ, as registration runs it) at the
    registration fans' shape: images, loss and every pose gradient against
    the FP64 oracle."""
    case = registration_shape_case()
    print("case", case.name, "ray-samples", case.ray_samples, flush=True)
    target = H.oracle_render(case, poses=case.extra["gt_poses"])
    got = _run_plan(case, target, replays=2, pose_only=True)
    assert got[2] is None
    _check_plan(case, got, _plan_reference(case, target, want_volume=False), "pose-only 384 x 1536")


@pytest.mark.parametrize("schedule", [None, {"fwd_chunk": 16, "bwd_chunk": 4, "xcd_group": 16, "scatter_rays": 8}])
def test_bench_workload_full_size(schedule):
    """The benchmark's own step at its full size: 64 poses x 256 rays x 1024
    samples with speckle and blur, fused forward + MSE + adjoint replayed from
    the captured graph (library default schedule, and the one the tuner
    picks).  Every pose's image, the loss, dL/dZ and every pose gradient
    against the FP64 oracle; the target is the oracle's render at the offset
    poses."""
    from paper_2508_06768_amd.render import FusedStep
    case = synth.case_batched_c2(B=64)
    geom, Z, P = _gpu(case)
    print("case", case.name, "schedule", schedule, flush=True)
    target = H.oracle_render(case, poses=case.extra["target_poses"])
    tf = target.astype(np.float32).astype(np.float64)
    T = torch.from_numpy(tf.astype(np.float32)).to(DEV)
    step = FusedStep(geom, zero_grad_z=True, schedule=schedule)
    bm = torch.empty(geom.total, device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    gZ = torch.empty_like(Z)
    gp = torch.empty((geom.n_poses, 6), device=DEV)
    for _ in range(2):
        step.step(Z, P, T, bmode=bm, loss=loss, grad_Z=gZ, grad_pose=gp)
    torch.cuda.synchronize()
    img = H.oracle_render(case)
    print("oracle forward done", flush=True)
    ref_loss = 0.0
    grad = np.zeros_like(img)
    for p, f in enumerate(case.fans):
        o0, o1 = int(geom.offsets[p]), int(geom.offsets[p + 1])
        d = img[o0:o1] - tf[o0:o1]
        ref_loss += np.mean(d * d)
        grad[o0:o1] = 2.0 * d / (o1 - o0)
    rep = H.parity_report(bm.cpu().numpy(), img, case.fans)
    print("image", rep, flush=True)
    assert rep["rel_l2"] <= 1e-5 and rep["max_abs_over_max"] <= 1e-5
    print("loss", loss.item(), ref_loss, flush=True)
    assert loss.item() == pytest.approx(ref_loss, rel=1e-5)
    rV, rp = H.oracle_backward(case, grad)
    check_grad_volume(gZ.cpu().numpy(), rV, "bench step")
    check_grad_pose(gp.cpu().numpy(), rp, "bench step")
    step.close()


def _det_run(case, target, graph=True, zero=True, init=None, replays=3):
    from paper_2508_06768_amd.render import FusedStep
    geom, Z, P = _gpu(case)
    T = torch.from_numpy(target.astype(np.float32)).to(DEV)
    step = FusedStep(geom, zero_grad_z=zero, graph=graph, deterministic=True)
    out = []
    for _ in range(replays):
        gZ = torch.full_like(Z, init if init is not None else 0.0)
        gp = torch.empty((geom.n_poses, 6), device=DEV)
        loss = torch.zeros(1, dtype=torch.float64, device=DEV)
        step.step(Z, P, T, loss=loss, grad_Z=gZ, grad_pose=gp)
        torch.cuda.synchronize()
        out.append((gZ.cpu().numpy(), gp.cpu().numpy(), loss.item()))
        _ = (Z * 2).sum().item()            # unrelated eager work between replays
    step.close()
    return out


@pytest.mark.parametrize("which", ["ragged", "bench8"])
def test_deterministic_plan(which):
    """DUS_PLAN_DETERMINISTIC sums dL/dZ as 64-bit fixed point: graph
    replays and the eager step give bit-identical dL/dZ (fresh buffers each
    time), which matches the oracle to the 1e-5 bars; without the clear flag
    the result is added to what grad_Z held."""
    from tests.test_gpu_parity import ragged_case
    if which == "ragged":
        case = ragged_case(0, 0, True, seed=45)
        target = H.oracle_render(case, poses=case.poses + np.float32([[0.4, -0.2, 0.3, 0.02, 0.0, -0.01]]))
    else:
        case = synth.case_batched_c2(B=8)
        target = H.oracle_render(case, poses=case.extra["target_poses"])
    print("case", which, "ray-samples", case.ray_samples, flush=True)
    runs = _det_run(case, target) + _det_run(case, target, graph=False, replays=1)
    for gZ, gp, loss in runs[1:]:
        np.testing.assert_array_equal(gZ, runs[0][0])
        np.testing.assert_array_equal(gp, runs[0][1])
    img, ref_loss, rV, rp = _plan_reference(case, target)
    assert runs[0][2] == pytest.approx(ref_loss, rel=1e-5)
    check_grad_volume(runs[0][0], rV, f"deterministic {which}")
    check_grad_pose(runs[0][1], rp, f"deterministic {which}")
    acc = _det_run(case, target, zero=False, init=123.0, replays=1)[0][0]
    check_grad_volume(acc.astype(np.float64) - 123.0, rV.astype(np.float64), f"deterministic {which} +=")


def test_deterministic_plan_gapped_images():
    """Pose images with gaps between them (never written): the fixed-point
    bound sums the fans' own rows, so NaN bytes left in the workspace's gaps
    change nothing."""
    from paper_2508_06768_amd.render import FusedStep
    from tests.test_gpu_parity import ragged_case
    case = ragged_case(0, 0, False, seed=46)
    target = H.oracle_render(case, poses=case.poses + np.float32([[0.3, 0.2, -0.2, 0.0, 0.02, 0.01]]))
    geom, Z, P = _gpu(case)
    gap = 1001
    packed = geom.offsets.copy()
    for i in range(geom.n_poses):
        geom.fans_c[i].out_offset = int(packed[i] + gap * (i + 1))
    geom.total = int(packed[-1] + gap * (geom.n_poses + 1))
    Tg = np.zeros(geom.total, np.float32)
    for i in range(geom.n_poses):
        o = int(geom.fans_c[i].out_offset)
        Tg[o:o + packed[i + 1] - packed[i]] = target[packed[i]:packed[i + 1]]
    step = FusedStep(geom, zero_grad_z=True, deterministic=True)
    step.workspace(Z.device).fill_(0xFF)        # NaN in every FP32 word of the workspace
    gZ = torch.empty_like(Z)
    gp = torch.empty((geom.n_poses, 6), device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    step.step(Z, P, torch.from_numpy(Tg).to(DEV), loss=loss, grad_Z=gZ, grad_pose=gp)
    torch.cuda.synchronize()
    step.close()
    img, ref_loss, rV, rp = _plan_reference(case, target)
    assert loss.item() == pytest.approx(ref_loss, rel=1e-5)
    check_grad_volume(gZ.cpu().numpy(), rV, "deterministic gapped")
    check_grad_pose(gp.cpu().numpy(), rp, "deterministic gapped")


def test_schedules_agree():
    from paper_2508_06768_amd.render import get_schedule, render, render_backward, set_schedule
    from tests.test_gpu_parity import ragged_case
    case = ragged_case(0, 0, True, seed=31)
    geom, Z, P = _gpu(case)
    w = torch.from_numpy(np.random.default_rng(5).standard_normal(geom.total).astype(np.float32)).to(DEV)
    base = get_schedule()
    outs = []
    try:
        for fc, bc, xg, sr in [(4, 4, 1, 2), (8, 8, 16, 4), (16, 4, 64, 8), (8, 4, 3, 8)]:
            set_schedule(fwd_chunk=fc, bwd_chunk=bc, xcd_group=xg, scatter_rays=sr)
            img = render(Z, P, geom).cpu().numpy().astype(np.float64)
            gZ, gp = render_backward(Z, P, geom, w)
            outs.append((img, gZ.cpu().numpy().astype(np.float64), gp.cpu().numpy().astype(np.float64)))
    finally:
        set_schedule(**base)
    for img, gZ, gp in outs[1:]:
        assert H.rel_l2(img, outs[0][0]) <= 1e-7
        assert H.rel_l2(gZ, outs[0][1]) <= 1e-6
        assert H.rel_l2(gp, outs[0][2]) <= 1e-6


def test_graph_replays_agree():
    from paper_2508_06768_amd.render import FusedStep, render
    from tests.test_gpu_parity import ragged_case
    case = ragged_case(0, 0, True, seed=41)
    geom, Z, P = _gpu(case)
    T = render(Z, P + 0.3, geom).clone()
    step = FusedStep(geom, zero_grad_z=True)
    bm = torch.empty(geom.total, device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    gZ = torch.empty_like(Z)
    gp = torch.empty((geom.n_poses, 6), device=DEV)
    res = []
    for it in range(4):
        step.step(Z, P, T, bmode=bm, loss=loss, grad_Z=gZ, grad_pose=gp)
        torch.cuda.synchronize()
        res.append((bm.cpu().numpy().copy(), loss.item(), gZ.cpu().numpy().copy(), gp.cpu().numpy().copy()))
        _ = (Z * 2).sum().item()            # unrelated eager work between replays
    eager = FusedStep(geom, zero_grad_z=True, graph=False)
    eager.step(Z, P, T, bmode=bm, loss=loss, grad_Z=gZ, grad_pose=gp)
    torch.cuda.synchronize()
    ref = (bm.cpu().numpy(), loss.item(), gZ.cpu().numpy(), gp.cpu().numpy())
    # the phase-timed step launches the same kernels eagerly, on one stream
    ms = eager.step_timed(Z, P, T, bmode=bm, loss=loss, grad_Z=gZ, grad_pose=gp)
    res.append((bm.cpu().numpy().copy(), loss.item(), gZ.cpu().numpy().copy(), gp.cpu().numpy().copy()))
    # a plan held to one stream (one table, one chain of launches)
    one = FusedStep(geom, zero_grad_z=True, one_stream=True)
    for _ in range(2):
        one.step(Z, P, T, bmode=bm, loss=loss, grad_Z=gZ, grad_pose=gp)
    torch.cuda.synchronize()
    res.append((bm.cpu().numpy().copy(), loss.item(), gZ.cpu().numpy().copy(), gp.cpu().numpy().copy()))
    one.close()
    assert all(v >= 0.0 for v in ms.values()) and ms["forward"] > 0 and ms["adjoint"] > 0 and ms["scatter"] > 0
    for r in res:
        np.testing.assert_array_equal(r[0], ref[0])
        assert r[1] == pytest.approx(ref[1], rel=1e-12)
        # dL/dZ goes through the scatter's global atomics (order-dependent
        # rounding); the pose gradient is summed in a fixed order
        assert H.rel_l2(r[2], ref[2]) <= 1e-6
        np.testing.assert_array_equal(r[3], ref[3])


def test_binding_rejects_short_buffers():
    """The raw-pointer ABI cannot see sizes: the binding refuses buffers
    smaller than the geometry before anything is launched."""
    from paper_2508_06768_amd.render import FusedStep, render, render_backward
    from tests.test_gpu_parity import ragged_case
    case = ragged_case(0, 0, False, seed=43)
    geom, Z, P = _gpu(case)
    step = FusedStep(geom, zero_grad_z=True)
    T = torch.zeros(geom.total, device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    gZ = torch.zeros_like(Z)
    gp = torch.zeros((geom.n_poses, 6), device=DEV)
    with pytest.raises(ValueError, match="target"):
        step.step(Z, P, T[:-1], loss=loss, grad_Z=gZ, grad_pose=gp)
    with pytest.raises(ValueError, match="grad_Z"):
        step.step(Z, P, T, loss=loss, grad_Z=gZ.view(-1)[:-1], grad_pose=gp)
    with pytest.raises(ValueError, match="grad_pose"):
        step.step(Z, P, T, loss=loss, grad_Z=gZ, grad_pose=gp[:-1])
    with pytest.raises(ValueError, match="loss"):
        step.step(Z, P, T, loss=loss.float(), grad_Z=gZ, grad_pose=gp)
    with pytest.raises(ValueError, match="out"):
        render(Z, P, geom, out=torch.empty(geom.total - 1, device=DEV))
    with pytest.raises(ValueError, match="grad_bmode"):
        render_backward(Z, P, geom, T[:-1])
    step.close()


def test_edge_sizes():
    """Maximum samples per ray, single ray, one and two samples, an empty fan,
    and a volume with 2-voxel axes: render and adjoint, and the fused step
    (whose adjoint starts from the forward's carries and chunk states)."""
    from paper_2508_06768_amd.render import render, render_backward
    from tests.test_gpu_parity import _check_plan, _plan_reference, _run_plan
    Z = synth.brain_volume(9, 32, 1.0, semi_range=(2.0, 8.0))
    Z2 = np.ascontiguousarray(Z[:2, :2, :])                      # nz = ny = 2
    for Zv, fans, poses in [
        (Z, [synth.FanSpec(1, 16384, 0.0, 0.002, 0.0, 0)], [[15.5, 15.5, 0.0, 0.01, 0.02, 0.0]]),
        (Z, [synth.FanSpec(3, 1, 0.2, 0.5, 0.0, 0), synth.FanSpec(0, 50, 0.2, 0.5, 0.0, 1),
             synth.FanSpec(5, 2, 0.9, 0.7, 2.0, 2), synth.FanSpec(2, 300, 0.3, 0.1, 0.0, 3)],
         [[15.5, 15.5, 0.0, 0, 0, 0]] * 4),
        (Z2, [synth.FanSpec(4, 120, 1.0, 0.25, 0.0, 0)], [[15.0, 0.5, 0.5, 0.0, 1.5707, 0.0]]),
    ]:
        case = synth.Case("edge", Zv, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), np.asarray(poses, np.float32), fans,
                          synth.PhysicsSpec(speckle_on=True, blur_on=True, seed=3))
        geom, Zt, P = _gpu(case)
        print("edge case", [(f.n_rays, f.n_samples) for f in fans], Zv.shape, flush=True)
        img = render(Zt, P, geom).cpu().numpy()
        ref = H.oracle_render(case)
        if np.abs(ref).max() > 0:
            rep = H.parity_report(img, ref)
            print(rep, flush=True)
            assert rep["rel_l2"] <= 1e-5 and rep["max_abs_over_max"] <= 1e-5
        else:
            assert np.all(img == 0)
        w = np.random.default_rng(2).standard_normal(geom.total).astype(np.float32)
        gZ, gp = render_backward(Zt, P, geom, torch.from_numpy(w).to(DEV))
        rV, rp = H.oracle_backward(case, w.astype(np.float64))
        if np.abs(rV).max() > 0:
            check_grad_volume(gZ.cpu().numpy(), rV, "edge")
        check_grad_pose(gp.cpu().numpy(), rp, "edge")
        target = H.oracle_render(case, poses=case.poses + np.float32([[0.3, -0.2, 0.1, 0.0, 0.0, 0.0]]))
        _check_plan(case, _run_plan(case, target, replays=2), _plan_reference(case, target), "edge plan")
        _check_plan(case, _run_plan(case, target, replays=2, pose_only=True),
                    _plan_reference(case, target, want_volume=False), "edge pose-only plan")


def test_largest_fan():
    """One fan of DUS_MAX_RAYS (65536) rays: render, adjoint and the fused
    step against the oracle (64 samples per ray over a 48^3 volume, speckle
    and blur on; 4.2 M ray-samples in one fan, so ray, blur-block and
    scatter-block indices reach their largest per-fan values).  Signed
    coefficients: with |R| this geometry has rays next to a pole (images
    near 3e5), whose conditioning is not what is tested here."""
    from paper_2508_06768_amd import _lib
    from paper_2508_06768_amd.render import render, render_backward
    n_rays = _lib.MAX_RAYS
    Z = synth.brain_volume(31, 48, 1.0, semi_range=(3.0, 10.0))
    case = synth.Case("largest_fan", Z, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0),
                      np.array([[23.5, 24.0, 0.0, 0.05, -0.04, 0.1]], np.float32),
                      [synth.FanSpec(n_rays, 64, 1.4, 0.6, 2.0, 0)],
                      synth.PhysicsSpec(refl_mode=1, speckle_on=True, blur_on=True, seed=31))
    geom, Zt, P = _gpu(case)
    print("largest fan", n_rays, "x 64", flush=True)
    img = render(Zt, P, geom).cpu().numpy()
    rep = H.parity_report(img, H.oracle_render(case))
    print(rep, flush=True)
    assert rep["rel_l2"] <= 1e-5 and rep["max_abs_over_max"] <= 1e-5
    w = np.random.default_rng(31).standard_normal(geom.total).astype(np.float32)
    gZ, gp = render_backward(Zt, P, geom, torch.from_numpy(w).to(DEV))
    rV, rp = H.oracle_backward(case, w.astype(np.float64))
    check_grad_volume(gZ.cpu().numpy(), rV, "largest fan")
    check_grad_pose(gp.cpu().numpy(), rp, "largest fan")
    target = H.oracle_render(case, poses=case.poses + np.float32([[0.3, -0.2, 0.1, 0.01, 0.0, 0.0]]))
    _check_plan(case, _run_plan(case, target, replays=2), _plan_reference(case, target), "largest fan plan")


def test_tall_volume():
    """A 4 x 4 x 200000 column crossed lengthwise (inside it) by 16384 samples of 10 mm:
    slice indices up to 2e5, where the flat voxel index is formed from 24-bit
    products (render, adjoint and the fused step against the oracle)."""
    from paper_2508_06768_amd.render import render, render_backward
    rng = np.random.default_rng(41)
    Z = rng.uniform(1.4, 1.8, size=(200000, 4, 4)).astype(np.float32)
    case = synth.Case("tall", Z, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0),
                      np.array([[1.5, 1.6, 0.0, 0.0, 0.0, 0.0], [1.4, 1.5, 3.0, 1e-6, -1e-6, 0.2]], np.float32),
                      [synth.FanSpec(3, 16384, 1e-6, 10.0, 0.0, 0), synth.FanSpec(2, 9000, 5e-7, 20.0, 5.0, 1)],
                      synth.PhysicsSpec(refl_mode=1, alpha=0.002, speckle_on=True, blur_on=True, seed=41))
    geom, Zt, P = _gpu(case)
    print("tall volume", Z.shape, flush=True)
    img = render(Zt, P, geom).cpu().numpy()
    rep = H.parity_report(img, H.oracle_render(case))
    print(rep, flush=True)
    assert rep["rel_l2"] <= 1e-5 and rep["max_abs_over_max"] <= 1e-5
    w = np.random.default_rng(41).standard_normal(geom.total).astype(np.float32)
    gZ, gp = render_backward(Zt, P, geom, torch.from_numpy(w).to(DEV))
    rV, rp = H.oracle_backward(case, w.astype(np.float64))
    check_grad_volume(gZ.cpu().numpy(), rV, "tall volume")
    check_grad_pose(gp.cpu().numpy(), rp, "tall volume")
    target = H.oracle_render(case, poses=case.poses + np.float32([[0.2, -0.1, 3.0, 0.0, 0.0, 0.01]]))
    assert np.abs(target).max() > 0
    _check_plan(case, _run_plan(case, target, replays=2), _plan_reference(case, target), "tall volume plan")


def test_wide_slices():
    """A 4000 x 4000 x 2 volume (slices of 1.6e7 voxels, just under the 2^24
    that the 24-bit index products allow) with fans lying in its mid-plane,
    rays up to 3950 mm long across it: render, adjoint and the fused step
    against the oracle.  The rotation by 120 degrees about (1, 1, 1) turns
    the probe's depth axis into x and its lateral axis into y."""
    from paper_2508_06768_amd.render import render, render_backward
    rng = np.random.default_rng(43)
    Z = rng.uniform(1.4, 1.8, size=(2, 4000, 4000)).astype(np.float32)
    w0 = 2.0 * np.pi / 3.0 / np.sqrt(3.0)
    case = synth.Case("wide", Z, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0),
                      np.array([[5.0, 5.0, 0.5, w0, w0, w0], [8.0, 2000.0, 0.5, w0, w0, w0]], np.float32),
                      [synth.FanSpec(9, 7900, 0.5, 0.5, 0.0, 0), synth.FanSpec(4, 3000, 0.2, 1.2, 2.0, 1)],
                      synth.PhysicsSpec(refl_mode=1, alpha=0.01, speckle_on=True, blur_on=True, seed=43))
    geom, Zt, P = _gpu(case)
    print("wide slices", Z.shape, flush=True)
    img = render(Zt, P, geom).cpu().numpy()
    rep = H.parity_report(img, H.oracle_render(case))
    print(rep, flush=True)
    assert rep["rel_l2"] <= 1e-5 and rep["max_abs_over_max"] <= 1e-5
    w = np.random.default_rng(43).standard_normal(geom.total).astype(np.float32)
    gZ, gp = render_backward(Zt, P, geom, torch.from_numpy(w).to(DEV))
    rV, rp = H.oracle_backward(case, w.astype(np.float64))
    check_grad_volume(gZ.cpu().numpy(), rV, "wide slices")
    check_grad_pose(gp.cpu().numpy(), rp, "wide slices")
    target = H.oracle_render(case, poses=case.poses + np.float32([[0.3, -0.2, 0.0, 0.0, 0.0, 0.0]]))
    _check_plan(case, _run_plan(case, target, replays=2), _plan_reference(case, target), "wide slices plan")


def test_images_past_2_31_pixels():
    """65 poses of 4096 rays x 8192 samples over the 256^3 volume: 2.18e9
    pixels, so the last pose's image starts at pixel 2^31 (64-bit offsets
    through render, blur, adjoint and the pose sums; rays of 8192 samples
    also take several wavefronts each).  Checked one pose at a time, where
    the oracle can follow: the first and the last pose's images from the
    render, and their pose gradients and the loss terms of a pose-only
    fused step against a zero target."""
    from paper_2508_06768_amd.render import FusedStep, render
    B = 65
    Z = synth.brain256(1002)
    poses = synth.random_poses(np.random.default_rng(1007), B, 255.0).astype(np.float32)
    fans = [synth.FanSpec(4096, 8192, 1.2, 0.03, 0.0, p) for p in range(B)]
    # signed coefficients: with |R| some of these 246 mm rays come near a
    # pole, whose conditioning is tested elsewhere
    phys = synth.PhysicsSpec(refl_mode=1, speckle_on=True, blur_on=True, seed=1007)
    case = synth.Case("past_2_31", Z, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), poses, fans, phys)
    geom, Zt, P = _gpu(case)
    assert int(geom.offsets[B - 1]) >= 2 ** 31
    print("images past 2^31 pixels:", geom.total, flush=True)
    img = render(Zt, P, geom)

    def one(p):
        return synth.Case(f"pose{p}", Z, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), poses[p:p + 1],
                          [synth.FanSpec(4096, 8192, 1.2, 0.03, 0.0, p)], phys)

    for p in (0, B - 1):
        rep = H.parity_report(geom.image(img, p).cpu().numpy().reshape(-1), H.oracle_render(one(p)))
        print("pose", p, rep, flush=True)
        assert rep["rel_l2"] <= 1e-5 and rep["max_abs_over_max"] <= 1e-5
    del img
    step = FusedStep(geom, pose_only=True)
    T = torch.zeros(geom.total, dtype=torch.float32, device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    gp = torch.empty((B, 6), device=DEV)
    step.step(Zt, P, T, loss=loss, grad_pose=gp)
    torch.cuda.synchronize()
    step.close()
    del T
    gp = gp.cpu().numpy()
    known = 0.0
    for p in (0, B - 1):
        _, ref_loss, _, rp = _plan_reference(one(p), np.zeros(4096 * 8192), want_volume=False)
        check_grad_pose(gp[p:p + 1], rp, f"pose {p} of {B}")
        known += ref_loss
    # the loss is the sum of every pose's mean squared image: the two checked
    # poses' terms bound it from below (the others are non-negative)
    print("loss", loss.item(), "the two checked poses' terms", known, flush=True)
    assert loss.item() >= known * (1.0 - 1e-5)


def test_registration_loop():
    """Pose-only fused steps under a graph give the same pose gradient as the
    separate forward / MSE / adjoint calls, and Adam on the poses reduces the
    loss (signed-coefficient physics, small offsets)."""
    import math

    from paper_2508_06768_amd.registration import register
    from paper_2508_06768_amd.render import FusedStep, Geometry, render, render_backward
    rng = np.random.default_rng(5)
    n = 96
    Z = synth.brain_volume(77, n, 1.0, semi_range=(4.0, 18.0))
    ph = synth.PhysicsSpec(refl_mode=1, speckle_on=True, blur_on=True, seed=3)
    fans = [synth.FanSpec(64, 320, math.radians(60), 0.25, 0.0, p) for p in range(4)]
    gt = np.array([[47.5 + rng.uniform(-8, 8), 47.5 + rng.uniform(-8, 8), rng.uniform(0, 3),
                    *rng.uniform(-0.15, 0.15, 3)] for _ in range(4)], dtype=np.float32)
    init = (gt + np.concatenate([rng.uniform(-3, 3, (4, 3)),
                                 rng.uniform(-math.radians(3), math.radians(3), (4, 3))], 1)).astype(np.float32)
    geom = Geometry(Z.shape, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), fans, ph)
    Zt = torch.from_numpy(Z).to(DEV)
    T = render(Zt, torch.from_numpy(gt).to(DEV), geom).clone()
    P = torch.from_numpy(init).to(DEV)
    # one fused pose-only step vs the separate calls
    step = FusedStep(geom, pose_only=True, zero_grad_z=False)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    gp = torch.empty((4, 6), device=DEV)
    step.step(Zt, P, T, loss=loss, grad_pose=gp)
    img = render(Zt, P, geom)
    d = (img - T).double()
    grad = torch.zeros_like(d)
    ref_loss = 0.0
    for p in range(4):
        o0, o1 = int(geom.offsets[p]), int(geom.offsets[p + 1])
        ref_loss += float((d[o0:o1] ** 2).mean())
        grad[o0:o1] = 2 * d[o0:o1] / (o1 - o0)
    _, gp_ref = render_backward(Zt, P, geom, grad.float(), want_Z=False)
    torch.cuda.synchronize()
    assert loss.item() == pytest.approx(ref_loss, rel=1e-5)
    # the two GPU paths form the residual from the same FP32 image but round
    # it differently (FP32 in the step, FP64 here): agreement to 1e-4 of the
    # largest component; the step itself is held to the oracle below
    np.testing.assert_allclose(gp.cpu().numpy(), gp_ref.cpu().numpy(), rtol=1e-4,
                               atol=1e-5 * float(gp_ref.abs().max()))
    step.close()
    case = synth.Case("registration96", Z, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), init, fans, ph)
    target = H.oracle_render(case, poses=gt)
    _check_plan(case, _run_plan(case, target, replays=2, pose_only=True),
                _plan_reference(case, target, want_volume=False), "registration96 pose-only")
    res = register(Zt, geom, T, P, steps=80, lr_t=0.2, lr_w=math.radians(0.2))
    print("registration loss", res.loss_history[0], "->", res.loss_history[-1], "steps/s", res.steps_per_s,
          flush=True)
    assert res.loss_history[-1] < 0.5 * res.loss_history[0]


def test_reconstruction_loop():
    """Volume reconstruction: fused step + smoothness prior + Adam on the
    voxels lowers the loss from a blurred start (48^3, 8 poses, SIGNED
    physics) and keeps the impedance finite and inside [lo, hi].  (Eight fans
    under-determine the volume: the footprint error is reported, not
    asserted.)"""
    from scipy.ndimage import gaussian_filter

    from paper_2508_06768_amd.reconstruction import reconstruct
    from paper_2508_06768_amd.render import Geometry, footprint_mask, render
    n, h = 48, 2.0
    gt = synth.brain_volume(71, n, h, semi_range=(6.0, 30.0))
    rng = np.random.default_rng(71)
    poses_np = synth.random_poses(rng, 8, (n - 1) * h)
    fans = [synth.FanSpec(64, 128, 70 * synth.DEG, 100.0 / 128, 0.0, p) for p in range(8)]
    geom = Geometry(gt.shape, (h,) * 3, (0.0,) * 3, fans, synth.PhysicsSpec(refl_mode=1, seed=71))
    Zgt = torch.from_numpy(gt).to(DEV)
    P = torch.from_numpy(np.ascontiguousarray(poses_np, dtype=np.float32)).to(DEV)
    T = render(Zgt, P, geom).clone()
    Z0 = torch.from_numpy(gaussian_filter(gt, 1.5, mode="nearest").astype(np.float32)).to(DEV)
    mask = footprint_mask(P, geom).bool()

    def err(Z):
        return float(torch.linalg.vector_norm((Z - Zgt)[mask].double()) /
                     torch.linalg.vector_norm((Zgt - Zgt[mask].mean())[mask].double()))

    res = reconstruct(Z0, geom, P, T, steps=60, lr=2e-3, weight=1e-5)
    print("reconstruction loss", res.loss_history[0], "->", res.loss_history[-1], "error", err(Z0), "->",
          err(res.Z), "steps/s", res.steps_per_s, flush=True)
    assert np.all(np.isfinite(res.loss_history))
    assert res.loss_history[-1] < 0.85 * res.loss_history[0]
    assert bool(torch.isfinite(res.Z).all())
    assert float(res.Z.min()) >= 0.5 and float(res.Z.max()) <= 12.0


def test_table_fit_gradient_through_the_renderer():
    """End to end: intensity volume -> impedance table -> B-mode -> MSE.
    dL/d(table values), chained through the GPU render adjoint and the map
    adjoint, against central differences of the oracle's own pipeline
    (oracle map, oracle render) in FP64."""
    from scipy.ndimage import gaussian_filter

    from paper_2508_06768_amd.render import Geometry, map_impedance, map_impedance_backward, render, render_backward
    rng = np.random.default_rng(51)
    n = 32
    inten = gaussian_filter(rng.uniform(-120.0, 160.0, (n, n, n)), 1.5, mode="nearest")
    inten[8:20, 10:22, 12:18] += 60.0                       # a block with sharp faces
    inten = inten.astype(np.float32)
    xk = np.array([-100.0, -40.0, 0.0, 30.0, 60.0, 120.0], dtype=np.float32)
    zk = np.array([1.4, 1.5, 1.6, 1.7, 2.2, 3.0], dtype=np.float32)
    fan = synth.FanSpec(16, 96, 50 * synth.DEG, 0.25, 0.0, 0)
    phys = synth.PhysicsSpec(refl_mode=1)
    pose = synth.top_pose(n)[None, :]

    def oracle_image(z):
        Z, _ = O.map_impedance(inten.astype(np.float64), xk.astype(np.float64), z)
        return O.render(O.Volume(Z, (1.0,) * 3, (0.0,) * 3), pose[0].astype(np.float64), H.oracle_fan(fan),
                        H.oracle_physics(phys)).reshape(-1)

    def oracle_loss(z, T):
        return float(np.mean((oracle_image(z) - T) ** 2))

    T = oracle_image(zk.astype(np.float64) * np.array([1.0, 1.02, 0.97, 1.03, 1.0, 0.98]))
    geom = Geometry((n, n, n), (1.0,) * 3, (0.0,) * 3, [fan], phys)
    It = torch.from_numpy(inten).to(DEV)
    Pt = torch.from_numpy(pose).to(DEV)
    Z = map_impedance(It, xk, zk)
    img = render(Z, Pt, geom)
    g = (2.0 * (img.double() - torch.from_numpy(T).to(DEV)) / T.size).float()
    gZ, _ = render_backward(Z, Pt, geom, g, want_pose=False)
    _, gz = map_impedance_backward(It, xk, zk, gZ, want_intensity=False)
    gz = gz.cpu().numpy()
    h = 1e-5
    fd = np.zeros(len(xk))
    for j in range(len(xk)):
        e = np.zeros(len(xk))
        e[j] = h
        fd[j] = (oracle_loss(zk.astype(np.float64) + e, T) - oracle_loss(zk.astype(np.float64) - e, T)) / (2 * h)
    print("table gradient", gz, "fd", fd, flush=True)
    assert np.linalg.norm(gz - fd) <= 1e-3 * np.linalg.norm(fd)

