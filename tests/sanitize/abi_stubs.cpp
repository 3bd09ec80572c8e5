// Host-only stand-ins for the HIP runtime calls and the kernel launchers
// that abi.cpp uses, so that the ABI's validation, workspace layout, fan
// tables and plan bookkeeping can run under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU.
//
// Streams, events, graphs and graph executables are small heap objects:
// the leak checker then sees any the ABI forgets to destroy.  Each launcher
// checks the fan table it is given (counts, offsets, monotone ray ranges)
// and aborts on an inconsistency; none touches device memory.
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "../../paper_2508_06768_amd/csrc/dus_internal.h"

int g_launches = 0;

namespace {
struct Obj {
    int kind;
};

template <typename T>
T make(int kind)
{
    return reinterpret_cast<T>(new Obj{kind});
}

void drop(void *p)
{
    delete reinterpret_cast<Obj *>(p);
}

// a plan hands the launchers its side stream and both events, all created
void check_side(const dus::SideStream *side)
{
    if (side && (!side->st || !side->fork || !side->join)) {
        fprintf(stderr, "side stream or its events missing\n");
        abort();
    }
}

void check_table(const dus::FanTable &t)
{
    ++g_launches;
    if (t.n < 0 || t.n > dus::kMaxFans) {
        fprintf(stderr, "fan table with %d fans\n", t.n);
        abort();
    }
    int rays = 0;
    for (int i = 0; i < t.n; ++i) {
        const dus::FanRec &f = t.f[i];
        if (f.ray_begin != rays || f.n_rays <= 0 || f.n_samples <= 0 || f.pose < 0) {
            fprintf(stderr, "inconsistent fan record %d\n", i);
            abort();
        }
        if (i > 0 && f.n_samples > t.f[i - 1].n_samples) {
            fprintf(stderr, "fan table not sorted longest first\n");
            abort();
        }
        rays += f.n_rays;
    }
    if (rays != t.total_rays) {
        fprintf(stderr, "fan table ray count %d != %d\n", rays, t.total_rays);
        abort();
    }
}
}  // namespace

extern "C" {
hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "stub"; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int)
{
    *s = make<hipStream_t>(1);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    drop(s);
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g)
{
    *g = make<hipGraph_t>(2);
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g)
{
    drop(g);
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t, hipGraphNode_t *, char *, size_t)
{
    *e = make<hipGraphExec_t>(3);
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e)
{
    drop(e);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = make<hipEvent_t>(4);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned)
{
    *e = make<hipEvent_t>(4);
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e)
{
    drop(e);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned int) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t)
{
    *ms = 0.0f;
    return hipSuccess;
}
}

namespace dus {
hipError_t launch_forward(int, int, const VolArgs &, const PhysArgs &, const FanTable &t, const float *, float *,
                          float *, int, double *, int32_t *, double *, float *, hipStream_t, const ZeroArgs &, int,
                          const SideStream *side)
{
    check_side(side);
    check_table(t);
    return hipSuccess;
}
hipError_t launch_backward(int, int, int, const VolArgs &, const PhysArgs &, const FanTable &t, const float *, RayRec *,
                           const float *, const float *, float *, float *, double *, double *, double *,
                           const double *, const int32_t *, const double *, const float *, hipStream_t)
{
    check_table(t);
    return hipSuccess;
}
hipError_t launch_adjoint(int, int, const VolArgs &, const PhysArgs &, const FanTable &t, const float *, RayRec *,
                          const float *, const float *, float *, double *, double *, double *, const double *,
                          const int32_t *, const double *, const float *, hipStream_t, int, const SideStream *side)
{
    check_side(side);
    check_table(t);
    return hipSuccess;
}
hipError_t launch_pose_reduce(const FanTable &t, const double *, double *, hipStream_t)
{
    check_table(t);
    return hipSuccess;
}
hipError_t launch_scatter(int, int, const VolArgs &, const FanTable &t, const RayRec *, const float *, float *,
                          hipStream_t, unsigned long long *, const double *, int)
{
    check_table(t);
    return hipSuccess;
}
hipError_t launch_blur(bool, const PhysArgs &, const FanTable &t, const float *, float *, hipStream_t)
{
    check_table(t);
    return hipSuccess;
}
hipError_t launch_blur_residual(const PhysArgs &, const FanTable &t, const float *, const float *, float *, float *,
                                float *, double *, hipStream_t)
{
    check_table(t);
    return hipSuccess;
}
hipError_t launch_pose_finalize(const double *, const float *, int, float *, hipStream_t) { return hipSuccess; }
hipError_t launch_footprint(const VolArgs &, const FanTable &t, const float *, uint8_t *, hipStream_t)
{
    check_table(t);
    return hipSuccess;
}
hipError_t launch_sample(int, const VolArgs &, const FanTable &t, const float *, float *, hipStream_t)
{
    check_table(t);
    return hipSuccess;
}
hipError_t launch_scan_convert(const float *, int, int, double, double, double, int, int, double, double, double,
                               double, float, float *, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_zero_f64(double *, int64_t, hipStream_t) { return hipSuccess; }
hipError_t launch_zero_f32(float *, int64_t, hipStream_t) { return hipSuccess; }
hipError_t launch_copy_f64(const double *, double *, int64_t, hipStream_t) { return hipSuccess; }
hipError_t launch_sum_f64(const double *, int64_t, double *, hipStream_t, bool) { return hipSuccess; }
hipError_t launch_finish(const double *, int64_t, double *, const double *, const float *, int, float *, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_zero_pair(float *, int64_t, double *, int64_t, hipStream_t) { return hipSuccess; }
int64_t smooth_blocks(int nx, int ny, int nz) { return ((int64_t)nx * ny * nz + 255) / 256; }
hipError_t launch_smooth(const float *, int, int, int, float, float, float, float *, double *, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_adam(float *, const float *, float *, float *, int64_t, float, float, float, float, float, float,
                       float, float, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_philox(const uint32_t *, int64_t, uint32_t, uint32_t, uint32_t *, hipStream_t) { return hipSuccess; }
hipError_t launch_map(const float *, int64_t, const LutArgs &, float *, hipStream_t) { return hipSuccess; }
hipError_t launch_map_backward(const float *, int64_t, const LutArgs &, const float *, float *, double *, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_pixel_gain(const PhysArgs &, const FanRec &, float *, hipStream_t) { return hipSuccess; }
hipError_t launch_abs_rows(const FanTable &t, const float *, double *, hipStream_t)
{
    check_table(t);
    return hipSuccess;
}
hipError_t launch_fix_scale(const double *, int64_t, double *, hipStream_t) { return hipSuccess; }
hipError_t launch_fix_to_f32(const unsigned long long *, int64_t, const double *, float *, bool, hipStream_t)
{
    return hipSuccess;
}
hipError_t static_scratch(void **ptr)
{
    *ptr = reinterpret_cast<void *>((uintptr_t)0x7000000);     // 256-byte aligned, never dereferenced
    return hipSuccess;
}
}  // namespace dus
