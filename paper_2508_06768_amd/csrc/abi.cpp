// Host side of the C ABI declared in include/diffus.h: argument validation,
// workspace layout, fan tables for batched launches, and the captured-graph
// plan of the fused forward + loss + adjoint step.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/diffus.h"
#include "dus_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int status, const char *what)
{
    g_last_error = what ? what : "";
    return status;
}

int hip_fail(hipError_t e, const char *where)
{
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return DUS_EHIP;
}

#define DUS_HIP(call, where)                                \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(e_, where);   \
    } while (0)

bool finite_f(float x) { return isfinite(x) != 0; }

constexpr int kDefaultFwdChunk = 0;       // automatic per fan table (launch_forward)
constexpr int kDefaultBwdChunk = 4;
constexpr int kDefaultXcdGroup = 16;
constexpr int kDefaultScatterRays = 0;     // automatic (launch_scatter)
constexpr int64_t kMaxImageExtent = (int64_t)1 << 48;   // image elements addressed by out_offset
constexpr int kFusedBlurRadius = 8;        // launch_blur_residual runs in one pass up to this radius

int check_volume(const dus_volume *v)
{
    if (!v) return fail(DUS_EINVAL, "volume descriptor is NULL");
    if (v->nx < 2 || v->ny < 2 || v->nz < 2) return fail(DUS_ESHAPE, "each volume axis needs >= 2 voxels");
    const long long n = (long long)v->nx * v->ny * v->nz;
    if (n >= (1ll << 31)) return fail(DUS_ESHAPE, "volume has 2^31 voxels or more");
    // the kernels' flat voxel index multiplies the slice index by the slice
    // size with 24-bit multiplies: both operands must stay below 2^24
    if ((long long)v->nx * v->ny >= (1ll << 24))
        return fail(DUS_EUNSUPPORTED, "a volume slice (nx * ny) must hold fewer than 2^24 voxels");
    if (v->nz >= (1 << 24)) return fail(DUS_EUNSUPPORTED, "a volume must have fewer than 2^24 slices (nz)");
    for (int a = 0; a < 3; ++a) {
        if (!finite_f(v->spacing_mm[a]) || !(v->spacing_mm[a] > 0.0f))
            return fail(DUS_EINVAL, "voxel spacing must be finite and > 0");
        if (!finite_f(v->origin_mm[a])) return fail(DUS_EINVAL, "volume origin must be finite");
    }
    return DUS_OK;
}

int check_physics(const dus_physics *p)
{
    if (!p) return fail(DUS_EINVAL, "physics descriptor is NULL");
    if (p->refl_mode != DUS_REFL_ABS && p->refl_mode != DUS_REFL_SIGNED)
        return fail(DUS_EINVAL, "refl_mode must be DUS_REFL_ABS or DUS_REFL_SIGNED");
    if (p->atten_mode < DUS_ATTEN_IN_SYSTEM || p->atten_mode > DUS_ATTEN_OFF)
        return fail(DUS_EINVAL, "atten_mode out of range");
    if (!finite_f(p->alpha_db_cm_mhz) || p->alpha_db_cm_mhz < 0.0f || !finite_f(p->f_mhz) || p->f_mhz < 0.0f)
        return fail(DUS_EINVAL, "attenuation parameters must be finite and >= 0");
    if (p->speckle_on != 0 && p->speckle_on != 1) return fail(DUS_EINVAL, "speckle_on must be 0 or 1");
    if (p->blur_on != 0 && p->blur_on != 1) return fail(DUS_EINVAL, "blur_on must be 0 or 1");
    if (p->reserved != 0) return fail(DUS_EINVAL, "reserved field must be 0");
    if (p->speckle_on) {
        if (p->spk_cell < 4 || p->spk_cell > (1 << 20)) return fail(DUS_EINVAL, "spk_cell must be in [4, 2^20]");
        if (!finite_f(p->spk_Ar) || !finite_f(p->spk_gamma) || !finite_f(p->spk_Ag0) || !finite_f(p->spk_Ag1) ||
            p->spk_gamma < 0.0f)
            return fail(DUS_EINVAL, "speckle parameters must be finite, gamma >= 0");
    }
    if (p->blur_on) {
        if (!finite_f(p->blur_sigma0) || !finite_f(p->blur_sigma1) || p->blur_sigma0 < 0.0f ||
            p->blur_sigma1 < 0.0f)
            return fail(DUS_EINVAL, "blur sigmas must be finite and >= 0");
        const float smax = std::max(p->blur_sigma0, p->blur_sigma1);
        if (ceilf(3.0f * smax) > (float)DUS_MAX_BLUR_RADIUS)
            return fail(DUS_EUNSUPPORTED, "blur radius ceil(3 sigma) exceeds DUS_MAX_BLUR_RADIUS");
    }
    return DUS_OK;
}

int check_fans(const dus_fan *fans, int32_t n_poses)
{
    if (n_poses < 0) return fail(DUS_ESHAPE, "n_poses < 0");
    if (n_poses > 0 && !fans) return fail(DUS_EINVAL, "fans is NULL");
    std::vector<std::pair<int64_t, int64_t>> spans;
    for (int i = 0; i < n_poses; ++i) {
        const dus_fan &f = fans[i];
        if (f.n_rays < 0 || f.n_rays > DUS_MAX_RAYS) return fail(DUS_ESHAPE, "n_rays out of range");
        if (f.n_samples < 0 || f.n_samples > DUS_MAX_SAMPLES) return fail(DUS_ESHAPE, "n_samples out of range");
        if (!finite_f(f.aperture_rad) || !finite_f(f.r0_mm) || !finite_f(f.ds_mm) || !(f.ds_mm > 0.0f))
            return fail(DUS_EINVAL, "fan geometry must be finite with ds > 0");
        if (f.out_offset < 0) return fail(DUS_ESHAPE, "out_offset < 0");
        const int64_t n = (int64_t)f.n_rays * f.n_samples;
        // image offsets and workspace sizes (several bytes per element)
        // must not overflow
        if (f.out_offset > kMaxImageExtent - n) return fail(DUS_ESHAPE, "out_offset + n_rays * n_samples exceeds 2^48");
        if (n > 0) spans.push_back({f.out_offset, f.out_offset + n});
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return fail(DUS_ESHAPE, "output blocks of two poses overlap");
    return DUS_OK;
}

int64_t image_extent(const dus_fan *fans, int32_t n_poses)
{
    int64_t e = 0;
    for (int i = 0; i < n_poses; ++i) {
        const int64_t n = (int64_t)fans[i].n_rays * fans[i].n_samples;
        if (n > 0) e = std::max(e, fans[i].out_offset + n);
    }
    return e;
}

dus::VolArgs vol_args(const float *Z, const dus_volume *v)
{
    dus::VolArgs a{};
    a.Z = Z;
    a.nx = v->nx;
    a.ny = v->ny;
    a.nz = v->nz;
    for (int i = 0; i < 3; ++i) {
        a.h[i] = v->spacing_mm[i];
        a.o[i] = v->origin_mm[i];
    }
    return a;
}

dus::PhysArgs phys_args(const dus_physics *p)
{
    dus::PhysArgs a{};
    a.alpha = p->alpha_db_cm_mhz;
    a.freq = p->f_mhz;
    a.refl = p->refl_mode;
    a.atten = p->atten_mode;
    a.speckle = p->speckle_on;
    a.cell = p->spk_cell > 0 ? p->spk_cell : 8;
    a.Ar = p->spk_Ar;
    a.gam = p->spk_gamma;
    a.Ag0 = p->spk_Ag0;
    a.Ag1 = p->spk_Ag1;
    a.blur = p->blur_on;
    a.s0 = p->blur_sigma0;
    a.s1 = p->blur_sigma1;
    a.key0 = (uint32_t)(p->seed & 0xffffffffull);
    a.key1 = (uint32_t)(p->seed >> 32);
    a.blur_rmax = p->blur_on ? (int)ceilf(3.0f * std::max(p->blur_sigma0, p->blur_sigma1)) : 0;
    if (a.blur_rmax > DUS_MAX_BLUR_RADIUS) a.blur_rmax = DUS_MAX_BLUR_RADIUS;
    return a;
}

// Fan tables of at most kMaxFans fans, each sorted longest ray first so the
// hardware dispatcher starts the longest rays first.
// Launch tables of at most kMaxFans fans each.  two_groups (a plan's two
// chains of launches): the fans are first split into two groups of about
// equal ray-samples (each fan, largest first, to the lighter group), and
// the groups' tables alternate, so that tables 0, 2, ... hold the first
// group and 1, 3, ... the second.
std::vector<dus::FanTable> build_tables(const dus_fan *fans, int32_t n_poses, bool two_groups = false)
{
    std::vector<int> pivot_begin(n_poses + 1, 0);
    for (int i = 0; i < n_poses; ++i) pivot_begin[i + 1] = pivot_begin[i] + std::max(0, fans[i].n_rays);
    std::vector<int> order;
    for (int i = 0; i < n_poses; ++i)
        if (fans[i].n_rays > 0 && fans[i].n_samples > 0) order.push_back(i);
    std::vector<std::vector<int>> grps;
    if (!two_groups) {
        for (size_t g0 = 0; g0 < order.size(); g0 += (size_t)dus::kMaxFans)
            grps.emplace_back(order.begin() + g0, order.begin() + std::min(order.size(), g0 + (size_t)dus::kMaxFans));
    } else {
        auto work = [&](int i) { return (int64_t)fans[i].n_rays * fans[i].n_samples; };
        std::vector<int> by_work = order;
        std::stable_sort(by_work.begin(), by_work.end(), [&](int a, int b) { return work(a) > work(b); });
        std::vector<int> half[2];
        // the first group (the step's own stream) starts one 64th of the
        // work ahead: the second chain begins after the fork and is joined
        // at the end, each about 10 us on the device (bench step and
        // uneven batch 1% faster, equal fans of 316 samples 1% slower)
        int64_t total = 0;
        for (int i : by_work) total += work(i);
        int64_t load[2] = {-total / 64, 0};
        for (int i : by_work) {
            const int h = (load[1] < load[0]) ? 1 : 0;
            half[h].push_back(i);
            load[h] += work(i);
        }
        std::vector<std::vector<int>> tabs_of[2];
        for (int h = 0; h < 2; ++h)
            for (size_t g0 = 0; g0 < half[h].size(); g0 += (size_t)dus::kMaxFans)
                tabs_of[h].emplace_back(half[h].begin() + g0,
                                        half[h].begin() + std::min(half[h].size(), g0 + (size_t)dus::kMaxFans));
        for (size_t k = 0; k < std::max(tabs_of[0].size(), tabs_of[1].size()); ++k)
            for (int h = 0; h < 2; ++h)
                if (k < tabs_of[h].size()) grps.push_back(tabs_of[h][k]);
    }
    std::vector<dus::FanTable> out;
    int64_t carries = 0;    // tile-carry records of all tables before this fan
    for (auto &grp : grps) {
        std::stable_sort(grp.begin(), grp.end(),
                         [&](int a, int b) { return fans[a].n_samples > fans[b].n_samples; });
        dus::FanTable t;
        memset(&t, 0, sizeof(t));
        t.n = (int)grp.size();
        int rays = 0, blks = 0;
        for (int q = 0; q < t.n; ++q) {
            const dus_fan &f = fans[grp[q]];
            dus::FanRec &r = t.f[q];
            r.n_rays = f.n_rays;
            r.n_samples = f.n_samples;
            r.aperture = f.aperture_rad;
            r.ds = f.ds_mm;
            r.r0 = f.r0_mm;
            r.speckle_id = f.speckle_id;
            r.out_offset = f.out_offset;
            r.ray_begin = rays;
            r.blk_begin = blks;
            r.pose = grp[q];
            r.pivot_begin = pivot_begin[grp[q]];
            r.carry_begin = (int32_t)carries;
            carries += dus::carry_records(f.n_rays, f.n_samples);
            rays += f.n_rays;
            blks += ((f.n_samples + 63) / 64) * ((f.n_rays + 63) / 64);
        }
        t.total_rays = rays;
        t.total_blur_blocks = blks;
        out.push_back(t);
    }
    return out;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
    size_t pre = 0, pre_bytes = 0;     // pre-blur image (forward with blur)
    size_t eb = 0, eb_bytes = 0;       // blur-transposed dL/dI (adjoint with blur)
    size_t res = 0, res_bytes = 0;     // MSE residual (plan with blur)
    size_t acc = 0, acc_bytes = 0;     // pose accumulators
    size_t rp = 0, rp_bytes = 0;       // per-ray pose partials of one table (adjoint)
    size_t zb = 0, zb_bytes = 0;       // dL/dZ per sample (adjoint)
    size_t part = 0, part_bytes = 0;   // loss partials (plan step)
    size_t car = 0, car_bytes = 0;     // tile carries, 4 doubles per record (plan step)
    size_t cex = 0, cex_bytes = 0;     // tile-carry exponents, one int32 per record
    size_t cst = 0, cst_bytes = 0;     // chunk states, kStateDoubles doubles per record
    size_t gain = 0, gain_bytes = 0;   // per-pixel gains recorded by the forward (plan step)
    size_t rays = 0, rays_bytes = 0;   // ray geometry the adjoint hands the scatter, one RayRec per ray
    size_t fix = 0, fix_bytes = 0;     // deterministic plan: 64-bit fixed-point dL/dZ per voxel
    size_t fsc = 0, fsc_bytes = 0;     // its scale (2^e, 2^-e, the bound) and the bound's partials
    size_t total = 0;
};

WsLayout layout(const dus_fan *fans, int32_t n_poses, const dus_physics *p, int mode, bool pose_only = false,
                int64_t det_voxels = 0)
{
    // mode 0: forward, 1: backward, 2: plan step (pose_only: a plan that
    // never scatters dL/dZ, so it keeps no per-sample dL/dZ)
    WsLayout L;
    const size_t img = (size_t)image_extent(fans, n_poses) * sizeof(float);
    size_t off = 0;
    if (p->blur_on && (mode == 0 || mode == 2)) {
        L.pre = off;
        L.pre_bytes = img;
        off = align_up(off + img);
    }
    if (p->blur_on && (mode == 1 || mode == 2)) {
        L.eb = off;
        L.eb_bytes = img;
        off = align_up(off + img);
    }
    // the plan keeps the MSE residual in memory only for blur radii above
    // the one-pass kernel's bound (8 rays)
    if (p->blur_on && mode == 2 && ceilf(3.0f * std::max(p->blur_sigma0, p->blur_sigma1)) > (float)kFusedBlurRadius) {
        L.res = off;
        L.res_bytes = img;
        off = align_up(off + img);
    }
    if (mode == 1 || mode == 2) {
        if (!(mode == 2 && pose_only)) {
            L.zb = off;
            L.zb_bytes = img;
            off = align_up(off + img);
        }
        L.acc = off;
        L.acc_bytes = (size_t)std::max(n_poses, 1) * dus::kPoseAcc * sizeof(double);
        off = align_up(off + L.acc_bytes);
        // every table's rays: the partials are summed after all adjoints ran
        size_t rays = 1;
        for (const auto &t : build_tables(fans, n_poses)) rays += (size_t)t.total_rays;
        L.rp = off;
        L.rp_bytes = rays * dus::kRayPart * sizeof(double);
        off = align_up(off + L.rp_bytes);
        if (!(mode == 2 && pose_only)) {
            L.rays = off;
            L.rays_bytes = rays * sizeof(dus::RayRec);
            off = align_up(off + L.rays_bytes);
        }
    }
    if (mode == 2) {
        // one partial per blur block or per ray of every table: at most the
        // larger of the two for every fan, however the fans are grouped in
        // tables (a plan regroups them when its schedule changes)
        size_t n = 0;
        for (int32_t i = 0; i < n_poses; ++i) {
            const dus_fan &f = fans[i];
            if (f.n_rays <= 0 || f.n_samples <= 0) continue;
            const size_t bb = (size_t)((f.n_samples + 63) / 64) * (size_t)((f.n_rays + 63) / 64);
            n += std::max(bb, (size_t)f.n_rays);
        }
        L.part = off;
        L.part_bytes = std::max<size_t>(n, 1) * sizeof(double);
        off = align_up(off + L.part_bytes);
        size_t rec = 0;
        for (int32_t i = 0; i < n_poses; ++i)
            if (fans[i].n_rays > 0 && fans[i].n_samples > 0)
                rec += (size_t)dus::carry_records(fans[i].n_rays, fans[i].n_samples);
        L.car = off;
        L.car_bytes = std::max<size_t>(rec, 1) * 4 * sizeof(double);
        off = align_up(off + L.car_bytes);
        L.cex = off;
        L.cex_bytes = std::max<size_t>(rec, 1) * sizeof(int32_t);
        off = align_up(off + L.cex_bytes);
        L.cst = off;
        L.cst_bytes = std::max<size_t>(rec, 1) * dus::kStateDoubles * sizeof(double);
        off = align_up(off + L.cst_bytes);
        if (p->speckle_on || p->atten_mode == DUS_ATTEN_POST_HOC) {
            L.gain = off;
            L.gain_bytes = img;
            off = align_up(off + img);
        }
    }
    if (mode == 2 && det_voxels > 0 && !pose_only) {
        L.fix = off;
        L.fix_bytes = (size_t)det_voxels * sizeof(unsigned long long);
        off = align_up(off + L.fix_bytes);
        L.fsc = off;
        size_t rays = 0;
        for (const auto &t : build_tables(fans, n_poses)) rays += (size_t)t.total_rays;
        L.fsc_bytes = (4 + rays) * sizeof(double);
        off = align_up(off + L.fsc_bytes);
    }
    L.total = off;
    return L;
}

int check_ws(void *ws, size_t ws_bytes, size_t need)
{
    if (need == 0) return DUS_OK;
    if (!ws) return fail(DUS_EWORKSPACE, "workspace is NULL but the call needs one");
    if (ws_bytes < need) return fail(DUS_EWORKSPACE, "workspace too small");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(DUS_EWORKSPACE, "workspace must be 256-byte aligned");
    return DUS_OK;
}

int check_common(const float *Z, const dus_volume *vol, const float *poses, const dus_fan *fans,
                 int32_t n_poses, const dus_physics *phys)
{
    int s;
    if ((s = check_volume(vol)) != DUS_OK) return s;
    if ((s = check_physics(phys)) != DUS_OK) return s;
    if ((s = check_fans(fans, n_poses)) != DUS_OK) return s;
    if (n_poses > 0 && image_extent(fans, n_poses) > 0) {
        if (!Z) return fail(DUS_EINVAL, "Z is NULL");
        if (!poses) return fail(DUS_EINVAL, "poses is NULL");
    }
    return DUS_OK;
}

// ---- enqueue helpers shared by the direct calls and the plan ----
struct Sched {
    int fwd_chunk = kDefaultFwdChunk;
    int bwd_chunk = kDefaultBwdChunk;
    int xcd_group = kDefaultXcdGroup;
    int scatter_rays = kDefaultScatterRays;
    int span_samples = dus::kSpanSamples;
};

Sched g_sched;     // schedule of the direct (non-plan) calls

int make_sched(const dus_schedule *sc, Sched &n)
{
    n.fwd_chunk = sc->fwd_chunk ? sc->fwd_chunk : kDefaultFwdChunk;
    n.bwd_chunk = sc->bwd_chunk ? sc->bwd_chunk : kDefaultBwdChunk;
    n.xcd_group = sc->xcd_group ? sc->xcd_group : kDefaultXcdGroup;
    n.scatter_rays = sc->scatter_rays ? sc->scatter_rays : kDefaultScatterRays;
    if (n.scatter_rays != 0 && n.scatter_rays != 2 && n.scatter_rays != 4 && n.scatter_rays != 8)
        return fail(DUS_EINVAL, "scatter_rays must be 0 (automatic), 2, 4 or 8");
    if (n.fwd_chunk != 0 && n.fwd_chunk != 4 && n.fwd_chunk != 8 && n.fwd_chunk != 16)
        return fail(DUS_EINVAL, "fwd_chunk must be 0 (automatic), 4, 8 or 16");
    if (n.bwd_chunk != 4 && n.bwd_chunk != 8) return fail(DUS_EINVAL, "bwd_chunk must be 4 or 8");
    if (n.xcd_group < 1 || n.xcd_group > 64) return fail(DUS_EINVAL, "xcd_group must be in [1, 64]");
    n.span_samples = sc->span_samples ? sc->span_samples : dus::kSpanSamples;
    if (n.span_samples != -1 && (n.span_samples < 1 || n.span_samples > DUS_MAX_SAMPLES))
        return fail(DUS_EINVAL, "span_samples must be 0 (default), -1 (never) or in [1, DUS_MAX_SAMPLES]");
    return DUS_OK;
}

// zero: buffers the first forward launch clears besides rendering
int enqueue_forward(const Sched &sc, const dus::VolArgs &va, const dus::PhysArgs &pa,
                    const std::vector<dus::FanTable> &tabs, const float *poses, float *out,
                    float *min_pivot, hipStream_t st, double *carry = nullptr, int32_t *carry_exp = nullptr,
                    double *cstate = nullptr, float *gain = nullptr, const dus::ZeroArgs &zero = dus::ZeroArgs{},
                    const dus::SideStream *side = nullptr)
{
    bool first = true;
    for (const auto &t : tabs) {
        if (t.total_rays <= 0) continue;
        DUS_HIP(dus::launch_forward(sc.fwd_chunk, sc.xcd_group, va, pa, t, poses, out, min_pivot, 0, carry,
                                    carry_exp, cstate, gain, st, first ? zero : dus::ZeroArgs{}, sc.span_samples,
                                    side),
                "forward kernel launch");
        first = false;
    }
    return DUS_OK;
}

}  // namespace

struct dus_plan {
    dus_volume vol;
    std::vector<dus_fan> fans;
    dus_physics phys;
    int32_t flags;
    Sched sched;
    std::vector<dus::FanTable> tabs;
    WsLayout ws;
    int64_t extent;
    hipStream_t cap = nullptr;
    // second stream, forked from the step's stream and joined back into it:
    // the second chain of launches (half the tables), or, when some ray is
    // long, the launches of the long rays beside the one-wavefront ones
    dus::SideStream side{};
    hipEvent_t cleared = nullptr;   // the first table's forward has cleared dL/dZ and the pose sums
    bool two_chains = false;        // the tables alternate between two chains of launches
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    const void *key[9] = {};
    size_t key_ws_bytes = 0;
    int device = -1;
};


namespace {

// Whether a plan's step runs as two chains of launches on two streams, the
// fans split in two groups of about equal work, so that one chain's kernels
// fill the other's tails: not for the deterministic plan (one chain), nor
// for a plan held to one stream, nor when some ray is long enough for
// several wavefronts (its launches take the second stream), nor for a
// single fan.
bool plan_two_chains(const dus_plan *p)
{
    int nonempty = 0;
    bool long_rays = false;
    for (const auto &f : p->fans) {
        if (f.n_rays <= 0 || f.n_samples <= 0) continue;
        ++nonempty;
        long_rays = long_rays || (p->sched.span_samples > 0 && f.n_samples >= p->sched.span_samples);
    }
    return !(nonempty < 2 || long_rays || (p->flags & (DUS_PLAN_DETERMINISTIC | DUS_PLAN_ONE_STREAM)));
}

}  // namespace

extern "C" {

const char *dus_status_string(int s)
{
    switch (s) {
    case DUS_OK: return "ok";
    case DUS_EINVAL: return "invalid argument";
    case DUS_ESHAPE: return "invalid shape";
    case DUS_EWORKSPACE: return "workspace missing or too small";
    case DUS_EHIP: return "HIP runtime error";
    case DUS_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *dus_last_error(void) { return g_last_error.c_str(); }

int dus_version(void) { return 1; }

int64_t dus_workspace_bytes(const dus_volume *vol, const dus_fan *fans, int32_t n_poses,
                            const dus_physics *phys, int32_t with_backward)
{
    int s;
    if ((s = check_volume(vol)) != DUS_OK) return s;
    if ((s = check_physics(phys)) != DUS_OK) return s;
    if ((s = check_fans(fans, n_poses)) != DUS_OK) return s;
    return (int64_t)layout(fans, n_poses, phys, with_backward ? 1 : 0).total;
}

int dus_render_bmode(const float *Z, const dus_volume *vol, const float *poses, const dus_fan *fans,
                     int32_t n_poses, const dus_physics *phys, float *bmode, float *ray_min_pivot,
                     void *ws, size_t ws_bytes, void *stream)
{
    int s;
    if ((s = check_common(Z, vol, poses, fans, n_poses, phys)) != DUS_OK) return s;
    const int64_t extent = image_extent(fans, n_poses);
    if (extent > 0 && !bmode) return fail(DUS_EINVAL, "bmode is NULL");
    const WsLayout L = layout(fans, n_poses, phys, 0);
    if ((s = check_ws(ws, ws_bytes, L.total)) != DUS_OK) return s;
    if (extent == 0) return DUS_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const auto tabs = build_tables(fans, n_poses);
    const dus::VolArgs va = vol_args(Z, vol);
    const dus::PhysArgs pa = phys_args(phys);
    const Sched sc = g_sched;
    float *dst = phys->blur_on ? reinterpret_cast<float *>((char *)ws + L.pre) : bmode;
    if ((s = enqueue_forward(sc, va, pa, tabs, poses, dst, ray_min_pivot, st)) != DUS_OK) return s;
    if (phys->blur_on)
        for (const auto &t : tabs) DUS_HIP(dus::launch_blur(false, pa, t, dst, bmode, st), "blur kernel launch");
    return DUS_OK;
}

int dus_render_bmode_backward(const float *Z, const dus_volume *vol, const float *poses,
                              const dus_fan *fans, int32_t n_poses, const dus_physics *phys,
                              const float *grad_bmode, float *grad_Z, float *grad_pose, void *ws,
                              size_t ws_bytes, void *stream)
{
    int s;
    if ((s = check_common(Z, vol, poses, fans, n_poses, phys)) != DUS_OK) return s;
    const int64_t extent = image_extent(fans, n_poses);
    if (extent > 0 && !grad_bmode) return fail(DUS_EINVAL, "grad_bmode is NULL");
    const WsLayout L = layout(fans, n_poses, phys, 1);
    if ((s = check_ws(ws, ws_bytes, L.total)) != DUS_OK) return s;
    if (!grad_Z && !grad_pose) return DUS_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *acc = reinterpret_cast<double *>((char *)ws + L.acc);
    if (grad_pose) DUS_HIP(dus::launch_zero_f64(acc, (int64_t)n_poses * dus::kPoseAcc, st), "zero kernel launch");
    if (extent > 0) {
        const auto tabs = build_tables(fans, n_poses);
        const dus::VolArgs va = vol_args(Z, vol);
        const dus::PhysArgs pa = phys_args(phys);
        const Sched sc = g_sched;
        const float *src = grad_bmode;
        if (phys->blur_on) {
            float *eb = reinterpret_cast<float *>((char *)ws + L.eb);
            for (const auto &t : tabs) DUS_HIP(dus::launch_blur(true, pa, t, grad_bmode, eb, st), "blur^T kernel launch");
            src = eb;
        }
        double *rpart = reinterpret_cast<double *>((char *)ws + L.rp);
        int64_t r0 = 0;
        for (const auto &t : tabs) {
            DUS_HIP(dus::launch_backward(sc.bwd_chunk, sc.xcd_group, sc.scatter_rays, va, pa, t, poses,
                                         reinterpret_cast<dus::RayRec *>((char *)ws + L.rays) + r0, src, nullptr,
                                         grad_Z ? reinterpret_cast<float *>((char *)ws + L.zb) : nullptr, grad_Z,
                                         grad_pose ? acc : nullptr, rpart + dus::kRayPart * r0, nullptr, nullptr,
                                         nullptr, nullptr, nullptr, st),
                    "adjoint kernel launch");
            r0 += t.total_rays;
        }
        if (grad_pose) {
            r0 = 0;
            for (const auto &t : tabs) {
                DUS_HIP(dus::launch_pose_reduce(t, rpart + dus::kRayPart * r0, acc, st), "pose reduction kernel");
                r0 += t.total_rays;
            }
        }
    }
    if (grad_pose) DUS_HIP(dus::launch_pose_finalize(acc, poses, n_poses, grad_pose, st), "pose kernel launch");
    return DUS_OK;
}

int dus_render_bmode_backward_static(const float *Z, const dus_volume *vol, const float *poses,
                                     const dus_fan *fans, int32_t n_poses, const dus_physics *phys,
                                     const float *grad_bmode, float *grad_Z, float *grad_pose, void *stream)
{
    static_assert(DUS_STATIC_SCRATCH_BYTES == dus::kStaticScratchBytes, "static scratch size");
    int s;
    if ((s = check_common(Z, vol, poses, fans, n_poses, phys)) != DUS_OK) return s;
    const WsLayout L = layout(fans, n_poses, phys, 1);
    if (L.total > dus::kStaticScratchBytes) {
        char msg[160];
        snprintf(msg, sizeof(msg), "this call needs %zu bytes of scratch; the static scratch holds %zu",
                 L.total, dus::kStaticScratchBytes);
        return fail(DUS_EUNSUPPORTED, msg);
    }
    void *ws = nullptr;
    if (L.total > 0) DUS_HIP(dus::static_scratch(&ws), "static scratch address");
    return dus_render_bmode_backward(Z, vol, poses, fans, n_poses, phys, grad_bmode, grad_Z, grad_pose, ws,
                                     ws ? dus::kStaticScratchBytes : 0, stream);
}

int dus_philox4x32_10(const uint32_t *counters, int64_t n, uint64_t seed, uint32_t *out, void *stream)
{
    if (n < 0) return fail(DUS_ESHAPE, "n < 0");
    if (n == 0) return DUS_OK;
    if (!counters || !out) return fail(DUS_EINVAL, "NULL pointer");
    DUS_HIP(dus::launch_philox(counters, n, (uint32_t)(seed & 0xffffffffull), (uint32_t)(seed >> 32), out,
                               reinterpret_cast<hipStream_t>(stream)),
            "philox kernel launch");
    return DUS_OK;
}

int dus_pixel_gain(const dus_fan *fan, const dus_physics *phys, float *out, void *stream)
{
    int s;
    if ((s = check_physics(phys)) != DUS_OK) return s;
    if ((s = check_fans(fan, 1)) != DUS_OK) return s;
    if ((int64_t)fan->n_rays * fan->n_samples == 0) return DUS_OK;
    if (!out) return fail(DUS_EINVAL, "out is NULL");
    if (fan->n_samples > 65535 * 256) return fail(DUS_ESHAPE, "too many samples");
    dus::FanRec r{};
    r.n_rays = fan->n_rays;
    r.n_samples = fan->n_samples;
    r.aperture = fan->aperture_rad;
    r.ds = fan->ds_mm;
    r.r0 = fan->r0_mm;
    r.speckle_id = fan->speckle_id;
    DUS_HIP(dus::launch_pixel_gain(phys_args(phys), r, out, reinterpret_cast<hipStream_t>(stream)),
            "gain kernel launch");
    return DUS_OK;
}

int dus_footprint_mask(const dus_volume *vol, const float *poses, const dus_fan *fans, int32_t n_poses,
                       uint8_t *mask, void *stream)
{
    int s;
    if ((s = check_volume(vol)) != DUS_OK) return s;
    if ((s = check_fans(fans, n_poses)) != DUS_OK) return s;
    if (image_extent(fans, n_poses) == 0) return DUS_OK;
    if (!poses || !mask) return fail(DUS_EINVAL, "NULL pointer");
    const dus::VolArgs va = vol_args(nullptr, vol);
    for (const auto &t : build_tables(fans, n_poses))
        DUS_HIP(dus::launch_footprint(va, t, poses, mask, reinterpret_cast<hipStream_t>(stream)),
                "footprint kernel launch");
    return DUS_OK;
}

int dus_sample_volume(const float *Z, const dus_volume *vol, const float *poses, const dus_fan *fans,
                      int32_t n_poses, float *out, void *stream)
{
    int s;
    if ((s = check_volume(vol)) != DUS_OK) return s;
    if ((s = check_fans(fans, n_poses)) != DUS_OK) return s;
    if (image_extent(fans, n_poses) == 0) return DUS_OK;
    if (!Z || !poses || !out) return fail(DUS_EINVAL, "NULL pointer");
    const dus::VolArgs va = vol_args(Z, vol);
    for (const auto &t : build_tables(fans, n_poses))
        DUS_HIP(dus::launch_sample(g_sched.xcd_group, va, t, poses, out, reinterpret_cast<hipStream_t>(stream)),
                "sample kernel launch");
    return DUS_OK;
}

int dus_scan_convert(const float *bmode, const dus_fan *fan, const dus_grid2d *grid, float *out, void *stream)
{
    if (!fan || !grid) return fail(DUS_EINVAL, "fan and grid are required");
    int s;
    if ((s = check_fans(fan, 1)) != DUS_OK) return s;
    if (fan->n_rays < 2 || fan->n_samples < 2) return fail(DUS_ESHAPE, "scan conversion needs n_rays >= 2 and n_samples >= 2");
    if (!(fan->aperture_rad > 0.0f)) return fail(DUS_EINVAL, "scan conversion needs aperture_rad > 0");
    if (grid->nx < 0 || grid->nz < 0) return fail(DUS_ESHAPE, "grid nx, nz must be >= 0");
    if ((int64_t)grid->nx * grid->nz > ((int64_t)1 << 31)) return fail(DUS_ESHAPE, "grid too large");
    if (!(grid->dx_mm > 0.0f) || !(grid->dz_mm > 0.0f) || !finite_f(grid->dx_mm) || !finite_f(grid->dz_mm) ||
        !finite_f(grid->x0_mm) || !finite_f(grid->z0_mm))
        return fail(DUS_EINVAL, "grid pitch must be finite and > 0, origin finite");
    if ((int64_t)grid->nx * grid->nz == 0) return DUS_OK;
    if (!bmode || !out) return fail(DUS_EINVAL, "NULL pointer");
    DUS_HIP(dus::launch_scan_convert(bmode + fan->out_offset, fan->n_rays, fan->n_samples, fan->aperture_rad, fan->r0_mm,
                                     fan->ds_mm, grid->nx, grid->nz, grid->x0_mm, grid->z0_mm, grid->dx_mm, grid->dz_mm,
                                     grid->fill, out, reinterpret_cast<hipStream_t>(stream)),
            "scan conversion kernel launch");
    return DUS_OK;
}

int64_t dus_smoothness_workspace_bytes(const dus_volume *vol)
{
    int s;
    if ((s = check_volume(vol)) != DUS_OK) return s;
    return (int64_t)align_up((size_t)std::max<int64_t>(dus::smooth_blocks(vol->nx, vol->ny, vol->nz), 1) *
                             sizeof(double));
}

int dus_smoothness(const float *Z, const dus_volume *vol, float weight, float *grad_Z, double *loss, void *ws,
                   size_t ws_bytes, void *stream)
{
    int s;
    if ((s = check_volume(vol)) != DUS_OK) return s;
    if (!finite_f(weight) || weight < 0.0f) return fail(DUS_EINVAL, "weight must be finite and >= 0");
    if (!Z || !grad_Z) return fail(DUS_EINVAL, "Z and grad_Z are required");
    const int64_t need = dus_smoothness_workspace_bytes(vol);
    if ((s = check_ws(ws, ws_bytes, (size_t)need)) != DUS_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const float wx = weight / (vol->spacing_mm[0] * vol->spacing_mm[0]);
    const float wy = weight / (vol->spacing_mm[1] * vol->spacing_mm[1]);
    const float wz = weight / (vol->spacing_mm[2] * vol->spacing_mm[2]);
    double *part = reinterpret_cast<double *>(ws);
    DUS_HIP(dus::launch_smooth(Z, vol->nx, vol->ny, vol->nz, wx, wy, wz, grad_Z, part, st), "smoothness kernel launch");
    if (loss)
        DUS_HIP(dus::launch_sum_f64(part, dus::smooth_blocks(vol->nx, vol->ny, vol->nz), loss, st, true),
                "smoothness sum kernel launch");
    return DUS_OK;
}

int dus_adam_step(float *x, const float *grad, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
                  float eps, int32_t t, float lo, float hi, void *stream)
{
    if (n < 0) return fail(DUS_ESHAPE, "n < 0");
    if (n == 0) return DUS_OK;
    if (!x || !grad || !m || !v) return fail(DUS_EINVAL, "NULL pointer");
    if (t < 1) return fail(DUS_EINVAL, "t must be >= 1");
    if (!finite_f(lr) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !finite_f(eps) || eps < 0.0f || !(lo <= hi))
        return fail(DUS_EINVAL, "bad Adam parameters");
    const float c1 = (float)(1.0 - pow((double)beta1, (double)t));
    const float c2 = (float)(1.0 - pow((double)beta2, (double)t));
    DUS_HIP(dus::launch_adam(x, grad, m, v, n, lr, beta1, beta2, eps, c1, c2, lo, hi,
                             reinterpret_cast<hipStream_t>(stream)),
            "Adam kernel launch");
    return DUS_OK;
}

static int lut_args(const dus_lut *lut, dus::LutArgs &a)
{
    if (!lut) return fail(DUS_EINVAL, "lut is NULL");
    static_assert(DUS_MAX_KNOTS == dus::kMaxKnots, "knot limit");
    if (lut->n < 2 || lut->n > DUS_MAX_KNOTS) return fail(DUS_EINVAL, "lut needs 2..DUS_MAX_KNOTS knots");
    a = dus::LutArgs{};
    a.n = lut->n;
    for (int j = 0; j < lut->n; ++j) {
        if (!finite_f(lut->x[j]) || !finite_f(lut->z[j])) return fail(DUS_EINVAL, "lut values must be finite");
        if (j > 0 && !(lut->x[j] > lut->x[j - 1])) return fail(DUS_EINVAL, "lut x must be strictly increasing");
        a.x[j] = lut->x[j];
        a.z[j] = lut->z[j];
    }
    return DUS_OK;
}

int dus_map_impedance(const float *intensity, int64_t n_vox, const dus_lut *lut, float *Z, void *stream)
{
    dus::LutArgs a;
    int s;
    if ((s = lut_args(lut, a)) != DUS_OK) return s;
    if (n_vox < 0) return fail(DUS_ESHAPE, "n_vox < 0");
    if (n_vox == 0) return DUS_OK;
    if (!intensity || !Z) return fail(DUS_EINVAL, "NULL pointer");
    DUS_HIP(dus::launch_map(intensity, n_vox, a, Z, reinterpret_cast<hipStream_t>(stream)), "map kernel launch");
    return DUS_OK;
}

int dus_map_impedance_backward(const float *intensity, int64_t n_vox, const dus_lut *lut, const float *grad_Z,
                               float *grad_intensity, double *grad_z, void *stream)
{
    dus::LutArgs a;
    int s;
    if ((s = lut_args(lut, a)) != DUS_OK) return s;
    if (n_vox < 0) return fail(DUS_ESHAPE, "n_vox < 0");
    if (n_vox == 0 || (!grad_intensity && !grad_z)) return DUS_OK;
    if (!intensity || !grad_Z) return fail(DUS_EINVAL, "NULL pointer");
    DUS_HIP(dus::launch_map_backward(intensity, n_vox, a, grad_Z, grad_intensity, grad_z,
                                     reinterpret_cast<hipStream_t>(stream)),
            "map adjoint kernel launch");
    return DUS_OK;
}

// ---------------------------------------------------------------------------
// plan: batched fused forward + MSE + adjoint, replayed from a HIP graph
// ---------------------------------------------------------------------------
int dus_plan_create(dus_plan **out, const dus_volume *vol, const dus_fan *fans, int32_t n_poses,
                    const dus_physics *phys, int32_t flags)
{
    if (!out) return fail(DUS_EINVAL, "out is NULL");
    *out = nullptr;
    int s;
    if ((s = check_volume(vol)) != DUS_OK) return s;
    if ((s = check_physics(phys)) != DUS_OK) return s;
    if ((s = check_fans(fans, n_poses)) != DUS_OK) return s;
    if (flags & ~(DUS_PLAN_POSE_ONLY | DUS_PLAN_ZERO_GRAD_Z | DUS_PLAN_NO_GRAPH | DUS_PLAN_DETERMINISTIC |
                  DUS_PLAN_ONE_STREAM))
        return fail(DUS_EINVAL, "unknown plan flag");
    dus_plan *p = new (std::nothrow) dus_plan();
    if (!p) return fail(DUS_EINVAL, "out of host memory");
    p->vol = *vol;
    p->fans.assign(fans, fans + n_poses);
    p->phys = *phys;
    p->flags = flags;
    p->two_chains = plan_two_chains(p);
    p->tabs = build_tables(fans, n_poses, p->two_chains);
    p->ws = layout(fans, n_poses, phys, 2, (flags & DUS_PLAN_POSE_ONLY) != 0,
                   (flags & DUS_PLAN_DETERMINISTIC) ? (int64_t)vol->nx * vol->ny * vol->nz : 0);
    p->extent = image_extent(fans, n_poses);
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->side.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->side.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->side.join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->cleared, hipEventDisableTiming);
    if (e != hipSuccess) {
        dus_plan_destroy(p);
        return hip_fail(e, "plan streams and events");
    }
    *out = p;
    return DUS_OK;
}

int64_t dus_plan_workspace_bytes(const dus_plan *p)
{
    if (!p) return fail(DUS_EINVAL, "plan is NULL");
    return (int64_t)p->ws.total;
}

static void plan_drop_graph(dus_plan *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

int dus_plan_set_schedule(dus_plan *p, const dus_schedule *sc)
{
    if (!p || !sc) return fail(DUS_EINVAL, "NULL pointer");
    Sched n;
    int s;
    if ((s = make_sched(sc, n)) != DUS_OK) return s;
    p->sched = n;
    plan_drop_graph(p);
    const bool two = plan_two_chains(p);
    if (two != p->two_chains) {
        p->two_chains = two;
        p->tabs = build_tables(p->fans.data(), (int32_t)p->fans.size(), two);
    }
    return DUS_OK;
}

int dus_set_schedule(const dus_schedule *sc)
{
    if (!sc) return fail(DUS_EINVAL, "NULL pointer");
    Sched n;
    int s;
    if ((s = make_sched(sc, n)) != DUS_OK) return s;
    g_sched = n;
    return DUS_OK;
}

int dus_get_schedule(dus_schedule *sc)
{
    if (!sc) return fail(DUS_EINVAL, "NULL pointer");
    sc->fwd_chunk = g_sched.fwd_chunk;
    sc->bwd_chunk = g_sched.bwd_chunk;
    sc->xcd_group = g_sched.xcd_group;
    sc->scatter_rays = g_sched.scatter_rays;
    sc->span_samples = g_sched.span_samples;
    return DUS_OK;
}

int dus_plan_get_schedule(const dus_plan *p, dus_schedule *sc)
{
    if (!p || !sc) return fail(DUS_EINVAL, "NULL pointer");
    sc->fwd_chunk = p->sched.fwd_chunk;
    sc->bwd_chunk = p->sched.bwd_chunk;
    sc->xcd_group = p->sched.xcd_group;
    sc->scatter_rays = p->sched.scatter_rays;
    sc->span_samples = p->sched.span_samples;
    return DUS_OK;
}

// ev (optional): DUS_NUM_PHASES + 1 events recorded at the phase boundaries
static int plan_enqueue_body(dus_plan *p, const float *Z, const float *poses, const float *target, float *bmode,
                             double *loss, float *grad_Z, float *grad_pose, void *ws, hipStream_t st,
                             hipEvent_t *ev, bool &forked)
{
    auto mark = [&](int i) -> hipError_t { return ev ? hipEventRecord(ev[i], st) : hipSuccess; };
    const dus::VolArgs va = vol_args(Z, &p->vol);
    const dus::PhysArgs pa = phys_args(&p->phys);
    const int n_poses = (int)p->fans.size();
    double *acc = reinterpret_cast<double *>((char *)ws + p->ws.acc);
    double *rpart = reinterpret_cast<double *>((char *)ws + p->ws.rp);
    float *gZ = (p->flags & DUS_PLAN_POSE_ONLY) ? nullptr : grad_Z;
    float *zbar = p->ws.zb_bytes ? reinterpret_cast<float *>((char *)ws + p->ws.zb) : nullptr;
    dus::RayRec *rays = p->ws.rays_bytes ? reinterpret_cast<dus::RayRec *>((char *)ws + p->ws.rays) : nullptr;
    double *part = reinterpret_cast<double *>((char *)ws + p->ws.part);
    int64_t n_part = 0;
    const Sched &sc = p->sched;
    // the forward records its tile carries, chunk states and per-pixel
    // gains; the adjoint starts from them
    double *car = reinterpret_cast<double *>((char *)ws + p->ws.car);
    int32_t *cex = reinterpret_cast<int32_t *>((char *)ws + p->ws.cex);
    double *cst = reinterpret_cast<double *>((char *)ws + p->ws.cst);
    float *gain = p->ws.gain_bytes ? reinterpret_cast<float *>((char *)ws + p->ws.gain) : nullptr;
    const bool blur = p->phys.blur_on != 0;
    const bool fwd = blur || bmode;               // the forward kernel runs
    // the pose accumulators and dL/dZ are cleared by the forward kernel's
    // wavefronts (when it runs and renders something), else by a fill kernel
    const int64_t n_vox = (int64_t)p->vol.nx * p->vol.ny * p->vol.nz;
    // deterministic plan: dL/dZ is summed in the fixed-point buffer (cleared
    // every step) and written into grad_Z at the end
    unsigned long long *fix = (gZ && p->ws.fix_bytes) ? reinterpret_cast<unsigned long long *>((char *)ws + p->ws.fix)
                                                      : nullptr;
    double *fsc = fix ? reinterpret_cast<double *>((char *)ws + p->ws.fsc) : nullptr;
    dus::ZeroArgs zero{};
    if (fix) {
        zero.a = reinterpret_cast<float *>(fix);
        zero.na = 2 * n_vox;
    } else {
        zero.a = gZ;
        zero.na = (gZ && (p->flags & DUS_PLAN_ZERO_GRAD_Z)) ? n_vox : 0;
    }
    zero.b = acc;
    zero.nb = grad_pose ? (int64_t)n_poses * dus::kPoseAcc : 0;
    const bool fwd_clears = fwd && p->extent > 0;
    // two chains: the tables alternate between the step's stream and the
    // plan's second stream (forked after the clears, joined before the end).
    // One chain for the phase-timed step, for the deterministic plan (its
    // scale needs every table's dL/dZ before any scatter), and when some ray
    // is long (plan_two_chains; the second stream then takes the long rays'
    // launches: a third stream forked from the second one crashed the host
    // process in graph capture)
    const bool two = (ev == nullptr) && p->tabs.size() >= 2 && !fix && p->two_chains;
    auto tst = [&](size_t i) { return (two && (i % 2)) ? p->side.st : st; };
    // the long rays' launches take the second stream unless the step keeps
    // to one stream (one-stream plan, phase-timed step) or it carries the
    // second chain
    const dus::SideStream *side = (two || ev || (p->flags & DUS_PLAN_ONE_STREAM)) ? nullptr : &p->side;
    DUS_HIP(mark(DUS_PHASE_CLEAR), "event");
    if (!fwd_clears) DUS_HIP(dus::launch_zero_pair(zero.a, zero.na, zero.b, zero.nb, st), "zero kernel");
    if (two) {
        DUS_HIP(hipEventRecord(p->side.fork, st), "fork event");
        DUS_HIP(hipStreamWaitEvent(p->side.st, p->side.fork, 0), "fork wait");
        forked = true;
    }
    DUS_HIP(mark(DUS_PHASE_FORWARD), "event");
    if (fwd) {
        float *img = blur ? reinterpret_cast<float *>((char *)ws + p->ws.pre) : bmode;
        for (size_t i = 0; i < p->tabs.size(); ++i) {
            const auto &t = p->tabs[i];
            if (t.total_rays <= 0) continue;
            // the first table's forward clears dL/dZ and the pose sums
            DUS_HIP(dus::launch_forward(sc.fwd_chunk, sc.xcd_group, va, pa, t, poses, img, nullptr, 0, car, cex, cst,
                                        gain, tst(i), (i == 0 && fwd_clears) ? zero : dus::ZeroArgs{},
                                        sc.span_samples, side),
                    "forward kernel launch");
            if (i == 0 && two && fwd_clears) DUS_HIP(hipEventRecord(p->cleared, st), "clear event");
        }
    }
    DUS_HIP(mark(DUS_PHASE_BLUR_LOSS), "event");
    const float *eb = nullptr;
    if (blur) {
        const float *pre = reinterpret_cast<float *>((char *)ws + p->ws.pre);
        float *res = p->ws.res_bytes ? reinterpret_cast<float *>((char *)ws + p->ws.res) : nullptr;
        float *ebw = reinterpret_cast<float *>((char *)ws + p->ws.eb);
        for (size_t i = 0; i < p->tabs.size(); ++i) {
            const auto &t = p->tabs[i];
            DUS_HIP(dus::launch_blur_residual(pa, t, pre, target, bmode, res, ebw, loss ? part + n_part : nullptr,
                                              tst(i)),
                    "blur/loss kernel");
            n_part += t.total_blur_blocks;
        }
        eb = ebw;
    }
    DUS_HIP(mark(DUS_PHASE_ADJOINT), "event");
    // with blur the adjoint starts from B^T of the residual; without it, the
    // adjoint forms the residual and the loss partials itself
    const bool adj = blur ? (gZ || grad_pose) : true;
    int64_t r0 = 0;        // rays of the tables before this one (pose partials)
    if (adj)
        for (size_t i = 0; i < p->tabs.size(); ++i) {
            const auto &t = p->tabs[i];
            // dL/dZ per sample is stored only for the scatter
            DUS_HIP(dus::launch_adjoint(sc.bwd_chunk, sc.xcd_group, va, pa, t, poses, gZ ? rays + r0 : nullptr, eb,
                                        blur ? nullptr : target,
                                        gZ ? zbar : nullptr,
                                        grad_pose ? acc : nullptr, rpart + dus::kRayPart * r0,
                                        (!blur && loss) ? part + n_part : nullptr,
                                        fwd ? car : nullptr, fwd ? cex : nullptr, fwd ? cst : nullptr,
                                        fwd ? gain : nullptr, tst(i), sc.span_samples, side),
                    "adjoint kernel");
            if (!blur) n_part += t.total_rays;
            r0 += t.total_rays;
        }
    // the second chain's scatters and pose sums wait for the first table's
    // forward, which clears what they add to
    if (two && fwd_clears) DUS_HIP(hipStreamWaitEvent(p->side.st, p->cleared, 0), "clear wait");
    DUS_HIP(mark(DUS_PHASE_SCATTER), "event");
    if (adj && gZ) {
        if (fix) {
            r0 = 0;
            for (const auto &t : p->tabs) {
                DUS_HIP(dus::launch_abs_rows(t, zbar, fsc + 4 + r0, st), "fixed-point bound kernel");
                r0 += t.total_rays;
            }
            DUS_HIP(dus::launch_fix_scale(fsc + 4, r0, fsc, st), "fixed-point scale kernel");
        }
        r0 = 0;
        for (size_t i = 0; i < p->tabs.size(); ++i) {
            const auto &t = p->tabs[i];
            // two chains: two scatters at a time share the wavefront budget
            DUS_HIP(dus::launch_scatter(sc.scatter_rays, sc.xcd_group, va, t, rays + r0, zbar, gZ, tst(i), fix, fsc,
                                        two ? 16384 : 32768),
                    "scatter kernel");
            r0 += t.total_rays;
        }
        if (fix)
            DUS_HIP(dus::launch_fix_to_f32(fix, n_vox, fsc, gZ, (p->flags & DUS_PLAN_ZERO_GRAD_Z) != 0, st),
                    "fixed-point conversion kernel");
    }
    DUS_HIP(mark(DUS_PHASE_FINISH), "event");
    if (adj && grad_pose) {
        r0 = 0;
        for (size_t i = 0; i < p->tabs.size(); ++i) {
            const auto &t = p->tabs[i];
            DUS_HIP(dus::launch_pose_reduce(t, rpart + dus::kRayPart * r0, acc, tst(i)), "pose reduction kernel");
            r0 += t.total_rays;
        }
    }
    if (two) {
        DUS_HIP(hipEventRecord(p->side.join, p->side.st), "join event");
        DUS_HIP(hipStreamWaitEvent(st, p->side.join, 0), "join wait");
    }
    DUS_HIP(dus::launch_finish(part, n_part, loss, acc, poses, n_poses, grad_pose, st), "loss and pose kernel");
    DUS_HIP(mark(DUS_NUM_PHASES), "event");
    return DUS_OK;
}

static int plan_enqueue(dus_plan *p, const float *Z, const float *poses, const float *target, float *bmode,
                        double *loss, float *grad_Z, float *grad_pose, void *ws, hipStream_t st,
                        hipEvent_t *ev = nullptr)
{
    bool forked = false;
    const int s = plan_enqueue_body(p, Z, poses, target, bmode, loss, grad_Z, grad_pose, ws, st, ev, forked);
    if (s != DUS_OK && forked) {
        // the second stream is joined back also when a launch failed: a
        // capture must not end with a fork left open, and the caller's
        // stream must wait for what the second stream already holds
        (void)hipEventRecord(p->side.join, p->side.st);
        (void)hipStreamWaitEvent(st, p->side.join, 0);
    }
    return s;
}

int dus_plan_step(dus_plan *p, const float *Z, const float *poses, const float *target, float *bmode,
                  double *loss, float *grad_Z, float *grad_pose, void *ws, size_t ws_bytes, void *stream)
{
    if (!p) return fail(DUS_EINVAL, "plan is NULL");
    int s;
    if ((s = check_ws(ws, ws_bytes, p->ws.total)) != DUS_OK) return s;
    if (p->extent > 0) {
        if (!Z || !poses || !target) return fail(DUS_EINVAL, "Z, poses and target are required");
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (p->flags & DUS_PLAN_NO_GRAPH) return plan_enqueue(p, Z, poses, target, bmode, loss, grad_Z, grad_pose, ws, st);
    const void *key[9] = {Z, poses, target, bmode, loss, grad_Z, grad_pose, ws, nullptr};
    bool same = p->exec != nullptr && p->key_ws_bytes == ws_bytes;
    for (int i = 0; i < 8 && same; ++i) same = (key[i] == p->key[i]);
    if (!same) {
        plan_drop_graph(p);
        DUS_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal), "begin capture");
        s = plan_enqueue(p, Z, poses, target, bmode, loss, grad_Z, grad_pose, ws, p->cap);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(p->cap, &g);
        if (s != DUS_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        p->graph = g;
        e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            plan_drop_graph(p);
            return hip_fail(e, "graph instantiate");
        }
        memcpy(p->key, key, sizeof(key));
        p->key_ws_bytes = ws_bytes;
    }
    DUS_HIP(hipGraphLaunch(p->exec, st), "graph launch");
    return DUS_OK;
}

int dus_plan_step_timed(dus_plan *p, const float *Z, const float *poses, const float *target, float *bmode,
                        double *loss, float *grad_Z, float *grad_pose, void *ws, size_t ws_bytes, void *stream,
                        float *ms)
{
    if (!p) return fail(DUS_EINVAL, "plan is NULL");
    if (!ms) return fail(DUS_EINVAL, "ms is NULL");
    int s;
    if ((s = check_ws(ws, ws_bytes, p->ws.total)) != DUS_OK) return s;
    if (p->extent > 0 && (!Z || !poses || !target)) return fail(DUS_EINVAL, "Z, poses and target are required");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t ev[DUS_NUM_PHASES + 1] = {};
    int made = 0;
    hipError_t e = hipSuccess;
    for (; made <= DUS_NUM_PHASES; ++made)
        if ((e = hipEventCreate(&ev[made])) != hipSuccess) break;
    if (e == hipSuccess) {
        s = plan_enqueue(p, Z, poses, target, bmode, loss, grad_Z, grad_pose, ws, st, ev);
        if (s == DUS_OK) {
            e = hipEventSynchronize(ev[DUS_NUM_PHASES]);
            for (int i = 0; i < DUS_NUM_PHASES && e == hipSuccess; ++i) e = hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]);
        }
    }
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    if (s != DUS_OK) return s;
    if (e != hipSuccess) return hip_fail(e, "phase events");
    return DUS_OK;
}

void dus_plan_destroy(dus_plan *p)
{
    if (!p) return;
    plan_drop_graph(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->side.st) (void)hipStreamDestroy(p->side.st);
    if (p->side.fork) (void)hipEventDestroy(p->side.fork);
    if (p->side.join) (void)hipEventDestroy(p->side.join);
    if (p->cleared) (void)hipEventDestroy(p->cleared);
    delete p;
}

}  // extern "C"
