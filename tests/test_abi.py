"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, the ctypes records match the C layout, and each validation
error returns its documented status before anything is enqueued."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2508_06768_amd import _lib
from paper_2508_06768_amd._lib import DusFan, DusPhysics, DusVolume

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "diffus.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dus_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = _lib.lib()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
        assert n in _lib.SIGNATURES, f"{n} has no ctypes signature"
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (dus_\w+)", out))
    assert set(names) <= exported


def test_record_layout_matches_header(tmp_path):
    src = tmp_path / "sizes.c"
    src.write_text('#include "diffus.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(dus_volume), sizeof(dus_fan),'
                   ' sizeof(dus_physics), sizeof(dus_schedule), offsetof(dus_fan, out_offset),'
                   ' offsetof(dus_physics, seed), sizeof(dus_grid2d), offsetof(dus_grid2d, fill));'
                   ' printf("%zu %zu\\n", sizeof(dus_lut), offsetof(dus_lut, z)); return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(DusVolume), ctypes.sizeof(DusFan), ctypes.sizeof(DusPhysics),
            ctypes.sizeof(_lib.DusSchedule), DusFan.out_offset.offset, DusPhysics.seed.offset,
            ctypes.sizeof(_lib.DusGrid2d), _lib.DusGrid2d.fill.offset, ctypes.sizeof(_lib.DusLut),
            _lib.DusLut.z.offset]
    assert got == want


def _vol(n=8):
    v = DusVolume()
    v.nx = v.ny = v.nz = n
    v.spacing_mm = (ctypes.c_float * 3)(1.0, 1.0, 1.0)
    v.origin_mm = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
    return v


def _fans(specs):
    arr = (DusFan * max(len(specs), 1))()
    off = 0
    for i, (nr, ns) in enumerate(specs):
        arr[i].n_rays, arr[i].n_samples = nr, ns
        arr[i].aperture_rad, arr[i].ds_mm, arr[i].r0_mm = 1.0, 0.25, 0.0
        arr[i].out_offset = off
        off += nr * ns
    return arr


def _phys(**kw):
    p = DusPhysics()
    p.alpha_db_cm_mhz, p.f_mhz, p.spk_cell = 0.5, 5.0, 8
    p.spk_Ar, p.spk_gamma, p.spk_Ag0, p.spk_Ag1 = 0.3, 1.5, 0.2, 0.3
    p.blur_sigma0, p.blur_sigma1 = 0.5, 2.5
    for k, v in kw.items():
        setattr(p, k, v)
    return p


FAKE = ctypes.c_void_p(0x1000)     # never dereferenced: validation fails first


def _render(vol, fans, n, phys, ws=None, ws_bytes=0, Z=FAKE, poses=FAKE, out=FAKE):
    L = _lib.lib()
    return L.dus_render_bmode(Z, ctypes.byref(vol) if vol is not None else None, poses, fans, n,
                              ctypes.byref(phys) if phys is not None else None, out, None, ws, ws_bytes, None)


def test_validation_errors():
    L = _lib.lib()
    v, f, p = _vol(), _fans([(4, 100)]), _phys()
    assert _render(None, f, 1, p) == _lib.DUS_EINVAL
    assert _render(v, f, 1, None) == _lib.DUS_EINVAL
    assert _render(v, f, 1, p, Z=None) == _lib.DUS_EINVAL
    assert _render(v, f, 1, p, poses=None) == _lib.DUS_EINVAL
    assert _render(v, f, 1, p, out=None) == _lib.DUS_EINVAL
    bad = _vol()
    bad.nx = 1
    assert _render(bad, f, 1, p) == _lib.DUS_ESHAPE
    bad = _vol()
    bad.nx, bad.ny, bad.nz = 4096, 4096, 2        # slice of 2^24 voxels: beyond the 24-bit voxel index
    assert _render(bad, f, 1, p) == _lib.DUS_EUNSUPPORTED
    bad.nx, bad.ny, bad.nz = 4096, 4095, 2        # below 2^24 is accepted (validation only)
    assert L.dus_workspace_bytes(ctypes.byref(bad), f, 1, ctypes.byref(p), 0) >= 0
    bad.nx, bad.ny, bad.nz = 2, 2, 1 << 24         # 2^24 slices: beyond the 24-bit slice index
    assert _render(bad, f, 1, p) == _lib.DUS_EUNSUPPORTED
    assert L.dus_workspace_bytes(ctypes.byref(bad), f, 1, ctypes.byref(p), 0) == _lib.DUS_EUNSUPPORTED
    bad.nz = (1 << 24) - 1                          # the largest slice count accepted
    assert L.dus_workspace_bytes(ctypes.byref(bad), f, 1, ctypes.byref(p), 0) >= 0
    bad = _vol()
    bad.spacing_mm = (ctypes.c_float * 3)(1.0, 0.0, 1.0)
    assert _render(bad, f, 1, p) == _lib.DUS_EINVAL
    bad = _vol()
    bad.origin_mm = (ctypes.c_float * 3)(float("nan"), 0.0, 0.0)
    assert _render(bad, f, 1, p) == _lib.DUS_EINVAL
    assert _render(v, _fans([(4, _lib.MAX_SAMPLES + 1)]), 1, p) == _lib.DUS_ESHAPE
    assert _render(v, _fans([(-1, 10)]), 1, p) == _lib.DUS_ESHAPE
    ff = _fans([(4, 100)])
    ff[0].ds_mm = 0.0
    assert _render(v, ff, 1, p) == _lib.DUS_EINVAL
    ff = _fans([(4, 100), (4, 100)])
    ff[1].out_offset = 399          # overlaps pose 0's 400 pixels
    assert _render(v, ff, 2, p) == _lib.DUS_ESHAPE
    assert _render(v, f, -1, p) == _lib.DUS_ESHAPE
    assert _render(v, f, 1, _phys(refl_mode=2)) == _lib.DUS_EINVAL
    assert _render(v, f, 1, _phys(atten_mode=3)) == _lib.DUS_EINVAL
    assert _render(v, f, 1, _phys(reserved=1)) == _lib.DUS_EINVAL
    assert _render(v, f, 1, _phys(speckle_on=1, spk_cell=2)) == _lib.DUS_EINVAL
    assert _render(v, f, 1, _phys(alpha_db_cm_mhz=-1.0)) == _lib.DUS_EINVAL
    assert _render(v, f, 1, _phys(blur_on=1, blur_sigma1=11.0)) == _lib.DUS_EUNSUPPORTED
    # blur needs a workspace
    pb = _phys(blur_on=1)
    need = L.dus_workspace_bytes(ctypes.byref(v), f, 1, ctypes.byref(pb), 0)
    assert need >= 400 * 4
    assert _render(v, f, 1, pb) == _lib.DUS_EWORKSPACE
    assert _render(v, f, 1, pb, ws=FAKE, ws_bytes=need - 1) == _lib.DUS_EWORKSPACE
    assert _render(v, f, 1, pb, ws=ctypes.c_void_p(0x1004), ws_bytes=need) == _lib.DUS_EWORKSPACE
    # backward: grad source required
    rc = L.dus_render_bmode_backward(FAKE, ctypes.byref(v), FAKE, f, 1, ctypes.byref(p), None, FAKE, FAKE,
                                     FAKE, 1 << 20, None)
    assert rc == _lib.DUS_EINVAL
    # empty work is a no-op success, even with NULL data pointers
    assert _render(v, _fans([(0, 100)]), 1, p, Z=None, poses=None, out=None) == _lib.DUS_OK
    assert _render(v, f, 0, p, Z=None, poses=None, out=None) == _lib.DUS_OK
    assert L.dus_philox4x32_10(FAKE, -1, 0, FAKE, None) == _lib.DUS_ESHAPE
    assert L.dus_philox4x32_10(None, 4, 0, FAKE, None) == _lib.DUS_EINVAL
    assert L.dus_last_error()


def test_workspace_sizes():
    L = _lib.lib()
    v = _vol()
    f = _fans([(4, 100), (3, 50)])
    p = _phys()
    assert L.dus_workspace_bytes(ctypes.byref(v), f, 2, ctypes.byref(p), 0) == 0
    wb = L.dus_workspace_bytes(ctypes.byref(v), f, 2, ctypes.byref(p), 1)
    # the adjoint's dL/dZ per sample (550 floats), the pose accumulators
    # (12 doubles per pose) and the per-ray pose partials (9 doubles per ray)
    assert wb >= 550 * 4 + 2 * 12 * 8 + 7 * 9 * 8 and wb % 256 == 0
    pb = _phys(blur_on=1)
    wfb = L.dus_workspace_bytes(ctypes.byref(v), f, 2, ctypes.byref(pb), 0)
    assert wfb >= 550 * 4 and wfb % 256 == 0
    assert L.dus_workspace_bytes(None, f, 2, ctypes.byref(p), 0) == _lib.DUS_EINVAL


def test_plan_validation():
    L = _lib.lib()
    h = ctypes.c_void_p()
    v, f, p = _vol(), _fans([(4, 100)]), _phys()
    assert L.dus_plan_create(None, ctypes.byref(v), f, 1, ctypes.byref(p), 0) == _lib.DUS_EINVAL
    assert L.dus_plan_create(ctypes.byref(h), ctypes.byref(v), f, 1, ctypes.byref(p), 64) == _lib.DUS_EINVAL
    assert L.dus_plan_create(ctypes.byref(h), ctypes.byref(v), f, 1, ctypes.byref(_phys(refl_mode=7)), 0) \
        == _lib.DUS_EINVAL
    assert h.value is None
    assert L.dus_plan_step(None, None, None, None, None, None, None, None, None, 0, None) == _lib.DUS_EINVAL
    ms = (ctypes.c_float * len(_lib.PHASES))()
    assert L.dus_plan_step_timed(None, None, None, None, None, None, None, None, None, 0, None, ms) \
        == _lib.DUS_EINVAL
    assert L.dus_plan_workspace_bytes(None) == _lib.DUS_EINVAL
    L.dus_plan_destroy(None)


def test_status_strings():
    L = _lib.lib()
    for s in (0, -1, -2, -3, -4, -5):
        assert L.dus_status_string(s)
    assert L.dus_version() >= 1
    assert np.int32(_lib.DUS_OK) == 0


def test_schedule_validation():
    """Schedules are validated on the host; 0 fields select the defaults
    (scatter_rays 0 = automatic)."""
    L = _lib.lib()
    old = _lib.DusSchedule()
    assert L.dus_get_schedule(ctypes.byref(old)) == _lib.DUS_OK
    try:
        for bad in [(3, 0, 0, 0, 0), (0, 16, 0, 0, 0), (0, 0, 65, 0, 0), (0, 0, 0, 3, 0), (0, 0, 0, 16, 0),
                    (0, 0, 0, 0, -2), (0, 0, 0, 0, _lib.MAX_SAMPLES + 1)]:
            assert L.dus_set_schedule(ctypes.byref(_lib.DusSchedule(*bad))) == _lib.DUS_EINVAL, bad
        assert L.dus_set_schedule(ctypes.byref(_lib.DusSchedule(0, 0, 0, 0, 0))) == _lib.DUS_OK
        got = _lib.DusSchedule()
        assert L.dus_get_schedule(ctypes.byref(got)) == _lib.DUS_OK
        assert (got.fwd_chunk, got.bwd_chunk, got.xcd_group, got.scatter_rays, got.span_samples) == (0, 4, 16, 0, 4096)
        for span in (-1, 1, _lib.MAX_SAMPLES):
            assert L.dus_set_schedule(ctypes.byref(_lib.DusSchedule(16, 8, 64, 2, span))) == _lib.DUS_OK
            assert L.dus_get_schedule(ctypes.byref(got)) == _lib.DUS_OK
            assert (got.fwd_chunk, got.bwd_chunk, got.xcd_group, got.scatter_rays, got.span_samples) == (16, 8, 64, 2, span)
    finally:
        L.dus_set_schedule(ctypes.byref(old))


def test_map_impedance_validation():
    L = _lib.lib()
    lut = _lib.DusLut()
    lut.n = 1
    assert L.dus_map_impedance(FAKE, 10, ctypes.byref(lut), FAKE, None) == _lib.DUS_EINVAL
    lut.n = 3
    for j, (x, z) in enumerate(((0.0, 1.0), (1.0, 2.0), (1.0, 3.0))):      # x not increasing
        lut.x[j], lut.z[j] = x, z
    assert L.dus_map_impedance(FAKE, 10, ctypes.byref(lut), FAKE, None) == _lib.DUS_EINVAL
    lut.x[2] = 2.0
    lut.z[1] = float("inf")
    assert L.dus_map_impedance(FAKE, 10, ctypes.byref(lut), FAKE, None) == _lib.DUS_EINVAL
    lut.z[1] = 2.0
    assert L.dus_map_impedance(FAKE, -1, ctypes.byref(lut), FAKE, None) == _lib.DUS_ESHAPE
    assert L.dus_map_impedance(None, 10, ctypes.byref(lut), FAKE, None) == _lib.DUS_EINVAL
    assert L.dus_map_impedance(FAKE, 0, ctypes.byref(lut), FAKE, None) == _lib.DUS_OK
    assert L.dus_map_impedance_backward(FAKE, 10, None, FAKE, FAKE, None, None) == _lib.DUS_EINVAL
    assert L.dus_map_impedance_backward(FAKE, 10, ctypes.byref(lut), None, FAKE, None, None) == _lib.DUS_EINVAL


def test_binding_refuses_host_buffers():
    """Buffers handed to the library as raw device pointers must be CUDA
    tensors; the binding checks before any call."""
    import torch
    from paper_2508_06768_amd.render import _check_buffer
    with pytest.raises(ValueError, match="CUDA"):
        _check_buffer(torch.zeros(4), "target", 4)
    _check_buffer(None, "bmode", 4)      # optional buffers may be absent
