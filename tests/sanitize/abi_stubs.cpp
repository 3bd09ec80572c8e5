// Host-only stand-ins for the HIP runtime calls and the kernel launchers
// that abi.cpp uses, so that the ABI's validation, workspace layout, fan
// tables and plan bookkeeping can run under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU.
//
// Streams, events, graphs and graph executables are small heap objects:
// the leak checker then sees any the ABI forgets to destroy.  Each launcher
// checks the fan table it is given (counts, offsets, monotone ray ranges)
// and aborts on an inconsistency; none touches device memory.
//
// Streams also keep a count of the work queued on them, and events remember
// the stream and count at their record, which models the fork / join rules
// of stream capture: a stream that waits on an event of the capture joins
// it, and the capture may only end once the capturing stream has waited on
// an event recorded after each joined stream's last work (else the ending
// reports an unjoined fork, as the runtime does).  stub_fail_launch(n) makes
// the n-th launch from then on fail, to drive the ABI's error paths.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../paper_2508_06768_amd/csrc/dus_internal.h"

int g_launches = 0;

namespace {
struct Obj {
    int kind;
    long ops = 0;           // stream: work queued; event: the stream's count at the record
    long joined = 0;        // stream: work the capturing stream has waited for
    bool in_capture = false;
    bool was_origin = false;
    Obj *src = nullptr;     // event: the stream it was recorded on
};

Obj g_null_stream{1};            // the null stream
Obj *g_origin = nullptr;         // the capturing stream
std::vector<Obj *> g_forked;     // streams that joined the capture
std::vector<Obj *> g_streams;    // streams alive
int g_unjoined = 0;              // captures that ended with a fork left open
long g_fail_in = 0;              // the launch, counted from now, that fails (0: none)
long g_launch_ops = 0;           // launches so far

template <typename T>
T make(int kind)
{
    return reinterpret_cast<T>(new Obj{kind});
}

void drop(void *p)
{
    delete reinterpret_cast<Obj *>(p);
}

Obj *stream(hipStream_t s)
{
    return s ? reinterpret_cast<Obj *>(s) : &g_null_stream;
}

// one kernel launch on stream s
hipError_t launch_on(hipStream_t s)
{
    ++g_launch_ops;
    if (g_fail_in > 0 && --g_fail_in == 0) return hipErrorLaunchFailure;
    ++stream(s)->ops;
    return hipSuccess;
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
    g_streams.push_back(stream(*s));
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    for (size_t i = 0; i < g_streams.size(); ++i)
        if (g_streams[i] == stream(s)) {
            g_streams.erase(g_streams.begin() + (long)i);
            break;
        }
    drop(s);
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    if (g_origin) return hipErrorIllegalState;
    g_origin = stream(s);
    g_origin->in_capture = true;
    g_origin->was_origin = true;
    g_forked.clear();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g)
{
    if (!g_origin || stream(s) != g_origin) return hipErrorIllegalState;
    bool open = false;
    for (Obj *f : g_forked) {
        open = open || (f->ops != f->joined);
        f->in_capture = false;
    }
    g_origin->in_capture = false;
    g_origin = nullptr;
    g_forked.clear();
    if (open) {
        ++g_unjoined;
        *g = nullptr;
        return hipErrorStreamCaptureUnjoined;
    }
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
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    Obj *ev = reinterpret_cast<Obj *>(e);
    ev->src = stream(s);
    ev->ops = ev->src->ops;
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int)
{
    Obj *st = stream(s), *ev = reinterpret_cast<Obj *>(e);
    if (!ev->src) return hipSuccess;                    // never recorded: nothing to wait for
    if (ev->src->in_capture && !st->in_capture) {       // a fork: s joins the capture
        st->in_capture = true;
        st->joined = st->ops;
        g_forked.push_back(st);
    }
    // waiting makes the recorded work of the event's stream done for this one
    if (ev->src != st && ev->ops > ev->src->joined && (st == g_origin || !g_origin)) ev->src->joined = ev->ops;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t)
{
    *ms = 0.0f;
    return hipSuccess;
}

// test hooks for the driver
void stub_fail_launch(long n) { g_fail_in = n; }
long stub_launches(void) { return g_launch_ops; }
int stub_unjoined_captures(void) { return g_unjoined; }
// work queued on the library's own streams (other than capturing ones)
// that no other stream has waited for: an eager step leaves none
long stub_open_work(void)
{
    long n = 0;
    for (Obj *t : g_streams)
        if (!t->was_origin) n += t->ops - t->joined;
    return n;
}
}

namespace dus {
hipError_t launch_forward(int, int, const VolArgs &, const PhysArgs &, const FanTable &t, const float *, float *,
                          float *, int, double *, int32_t *, double *, float *, hipStream_t st, const ZeroArgs &, int,
                          const SideStream *side)
{
    check_side(side);
    check_table(t);
    return launch_on(st);
}
hipError_t launch_backward(int, int, int, const VolArgs &, const PhysArgs &, const FanTable &t, const float *, RayRec *,
                           const float *, const float *, float *, float *, double *, double *, double *,
                           const double *, const int32_t *, const double *, const float *, hipStream_t st)
{
    check_table(t);
    return launch_on(st);
}
hipError_t launch_adjoint(int, int, const VolArgs &, const PhysArgs &, const FanTable &t, const float *, RayRec *,
                          const float *, const float *, float *, double *, double *, double *, const double *,
                          const int32_t *, const double *, const float *, hipStream_t st, int, const SideStream *side)
{
    check_side(side);
    check_table(t);
    return launch_on(st);
}
hipError_t launch_pose_reduce(const FanTable &t, const double *, double *, hipStream_t st)
{
    check_table(t);
    return launch_on(st);
}
hipError_t launch_scatter(int, int, const VolArgs &, const FanTable &t, const RayRec *, const float *, float *,
                          hipStream_t st, unsigned long long *, const double *, int)
{
    check_table(t);
    return launch_on(st);
}
hipError_t launch_blur(bool, const PhysArgs &, const FanTable &t, const float *, float *, hipStream_t st)
{
    check_table(t);
    return launch_on(st);
}
hipError_t launch_blur_residual(const PhysArgs &, const FanTable &t, const float *, const float *, float *, float *,
                                float *, double *, hipStream_t st)
{
    check_table(t);
    return launch_on(st);
}
hipError_t launch_pose_finalize(const double *, const float *, int, float *, hipStream_t st) { return launch_on(st); }
hipError_t launch_footprint(const VolArgs &, const FanTable &t, const float *, uint8_t *, hipStream_t st)
{
    check_table(t);
    return launch_on(st);
}
hipError_t launch_sample(int, const VolArgs &, const FanTable &t, const float *, float *, hipStream_t st)
{
    check_table(t);
    return launch_on(st);
}
hipError_t launch_scan_convert(const float *, int, int, double, double, double, int, int, double, double, double,
                               double, float, float *, hipStream_t st)
{
    return launch_on(st);
}
hipError_t launch_zero_f64(double *, int64_t, hipStream_t st) { return launch_on(st); }
hipError_t launch_zero_f32(float *, int64_t, hipStream_t st) { return launch_on(st); }
hipError_t launch_sum_f64(const double *, int64_t, double *, hipStream_t st, bool) { return launch_on(st); }
hipError_t launch_finish(const double *, int64_t, double *, const double *, const float *, int, float *, hipStream_t st)
{
    return launch_on(st);
}
hipError_t launch_zero_pair(float *, int64_t, double *, int64_t, hipStream_t st) { return launch_on(st); }
int64_t smooth_blocks(int nx, int ny, int nz) { return ((int64_t)nx * ny * nz + 255) / 256; }
hipError_t launch_smooth(const float *, int, int, int, float, float, float, float *, double *, hipStream_t st)
{
    return launch_on(st);
}
hipError_t launch_adam(float *, const float *, float *, float *, int64_t, float, float, float, float, float, float,
                       float, float, hipStream_t st)
{
    return launch_on(st);
}
hipError_t launch_philox(const uint32_t *, int64_t, uint32_t, uint32_t, uint32_t *, hipStream_t st) { return launch_on(st); }
hipError_t launch_map(const float *, int64_t, const LutArgs &, float *, hipStream_t st) { return launch_on(st); }
hipError_t launch_map_backward(const float *, int64_t, const LutArgs &, const float *, float *, double *, hipStream_t st)
{
    return launch_on(st);
}
hipError_t launch_pixel_gain(const PhysArgs &, const FanRec &, float *, hipStream_t st) { return launch_on(st); }
hipError_t launch_abs_rows(const FanTable &t, const float *, double *, hipStream_t st)
{
    check_table(t);
    return launch_on(st);
}
hipError_t launch_fix_scale(const double *, int64_t, double *, hipStream_t st) { return launch_on(st); }
hipError_t launch_fix_to_f32(const unsigned long long *, int64_t, const double *, float *, bool, hipStream_t st)
{
    return launch_on(st);
}
hipError_t static_scratch(void **ptr)
{
    *ptr = reinterpret_cast<void *>((uintptr_t)0x7000000);     // 256-byte aligned, never dereferenced
    return hipSuccess;
}
}  // namespace dus
