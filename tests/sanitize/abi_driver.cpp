// Drives every entry point of include/diffus.h through its host-side logic
// (validation, workspace layout, fan tables, plan capture bookkeeping) with
// valid and invalid arguments.  Linked with abi_stubs.cpp instead of the HIP
// runtime and the kernels, and built with -fsanitize=address,undefined: the
// device pointers below are never dereferenced by the host code.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/diffus.h"

extern int g_launches;
extern "C" {
void stub_fail_launch(long n);
long stub_launches(void);
int stub_unjoined_captures(void);
long stub_open_work(void);
}

namespace {
int failures = 0;

void expect(bool ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s (%s)\n", what, dus_last_error());
        ++failures;
    }
}

template <typename T>
T *dev(uintptr_t a)
{
    return reinterpret_cast<T *>(a);
}

dus_volume volume(int nx, int ny, int nz)
{
    dus_volume v;
    memset(&v, 0, sizeof(v));
    v.nx = nx;
    v.ny = ny;
    v.nz = nz;
    for (int a = 0; a < 3; ++a) v.spacing_mm[a] = 1.0f;
    return v;
}

dus_physics physics(int speckle, int blur)
{
    dus_physics p;
    memset(&p, 0, sizeof(p));
    p.alpha_db_cm_mhz = 0.5f;
    p.f_mhz = 5.0f;
    p.speckle_on = speckle;
    p.spk_cell = 8;
    p.spk_Ar = 0.3f;
    p.spk_gamma = 1.5f;
    p.spk_Ag0 = 0.2f;
    p.spk_Ag1 = 0.3f;
    p.blur_on = blur;
    p.blur_sigma0 = 0.5f;
    p.blur_sigma1 = 2.5f;
    p.seed = 7;
    return p;
}

std::vector<dus_fan> fans(int n, int rays, int samples)
{
    std::vector<dus_fan> f((size_t)n);
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        f[i].n_rays = rays + (i % 3);
        f[i].n_samples = samples + 37 * (i % 5);
        f[i].aperture_rad = 1.0f;
        f[i].ds_mm = 0.25f;
        f[i].r0_mm = 0.0f;
        f[i].speckle_id = i;
        f[i].out_offset = off;
        off += (int64_t)f[i].n_rays * f[i].n_samples;
    }
    return f;
}

const uintptr_t kZ = 0x1000000, kPoses = 0x2000000, kImg = 0x3000000, kGrad = 0x4000000, kWs = 0x5000000;
}  // namespace

int main()
{
    for (int s = 1; s >= -6; --s) expect(dus_status_string(s) != nullptr, "status string");
    expect(dus_version() >= 1, "version");

    const dus_volume v = volume(48, 40, 36);
    for (int spk = 0; spk < 2; ++spk)
        for (int blur = 0; blur < 2; ++blur) {
            const dus_physics p = physics(spk, blur);
            for (int nf : {1, 3, 64, 70}) {
                std::vector<dus_fan> f = fans(nf, 5, 100);
                for (int wb = 0; wb < 2; ++wb) {
                    const int64_t ws = dus_workspace_bytes(&v, f.data(), nf, &p, wb);
                    expect(ws >= 0, "workspace bytes");
                }
                const int64_t wsf = dus_workspace_bytes(&v, f.data(), nf, &p, 0);
                expect(dus_render_bmode(dev<float>(kZ), &v, dev<float>(kPoses), f.data(), nf, &p, dev<float>(kImg),
                                        dev<float>(kGrad), dev<void>(kWs), (size_t)wsf, nullptr) == DUS_OK,
                       "render");
                const int64_t wsb = dus_workspace_bytes(&v, f.data(), nf, &p, 1);
                expect(dus_render_bmode_backward(dev<float>(kZ), &v, dev<float>(kPoses), f.data(), nf, &p,
                                                 dev<float>(kImg), dev<float>(kGrad), dev<float>(kGrad + 0x100000),
                                                 dev<void>(kWs), (size_t)wsb, nullptr) == DUS_OK,
                       "backward");
                expect(dus_render_bmode_backward(dev<float>(kZ), &v, dev<float>(kPoses), f.data(), nf, &p,
                                                 dev<float>(kImg), nullptr, dev<float>(kGrad + 0x100000),
                                                 dev<void>(kWs), (size_t)wsb, nullptr) == DUS_OK,
                       "backward pose only");
                expect(dus_render_bmode_backward_static(dev<float>(kZ), &v, dev<float>(kPoses), f.data(), nf, &p,
                                                        dev<float>(kImg), dev<float>(kGrad),
                                                        dev<float>(kGrad + 0x100000), nullptr) == DUS_OK,
                       "backward, static scratch");
                for (int flags : {0, (int)DUS_PLAN_POSE_ONLY, (int)DUS_PLAN_ZERO_GRAD_Z, (int)DUS_PLAN_NO_GRAPH,
                                  (int)(DUS_PLAN_ZERO_GRAD_Z | DUS_PLAN_NO_GRAPH), (int)DUS_PLAN_DETERMINISTIC,
                                  (int)(DUS_PLAN_DETERMINISTIC | DUS_PLAN_ZERO_GRAD_Z | DUS_PLAN_NO_GRAPH),
                                  (int)DUS_PLAN_ONE_STREAM, (int)(DUS_PLAN_ONE_STREAM | DUS_PLAN_NO_GRAPH)}) {
                    dus_plan *plan = nullptr;
                    expect(dus_plan_create(&plan, &v, f.data(), nf, &p, flags) == DUS_OK, "plan create");
                    const int64_t wsp = dus_plan_workspace_bytes(plan);
                    expect(wsp >= 0, "plan workspace");
                    for (int rep = 0; rep < 3; ++rep) {
                        // a changed pointer captures a new graph
                        expect(dus_plan_step(plan, dev<float>(kZ), dev<float>(kPoses), dev<float>(kImg),
                                             rep == 2 ? dev<float>(kImg + 0x800000) : nullptr, dev<double>(kGrad),
                                             (flags & DUS_PLAN_POSE_ONLY) ? nullptr : dev<float>(kGrad + 0x200000),
                                             dev<float>(kGrad + 0x100000), dev<void>(kWs), (size_t)wsp,
                                             nullptr) == DUS_OK,
                               "plan step");
                    }
                    float ms[DUS_NUM_PHASES];
                    expect(dus_plan_step_timed(plan, dev<float>(kZ), dev<float>(kPoses), dev<float>(kImg), nullptr,
                                               dev<double>(kGrad), nullptr, dev<float>(kGrad + 0x100000),
                                               dev<void>(kWs), (size_t)wsp, nullptr, ms) == DUS_OK,
                           "plan step timed");
                    dus_schedule sc = {16, 8, 3, 4};
                    expect(dus_plan_set_schedule(plan, &sc) == DUS_OK, "plan schedule");
                    dus_schedule got;
                    expect(dus_plan_get_schedule(plan, &got) == DUS_OK && got.fwd_chunk == 16, "plan get schedule");
                    expect(dus_plan_step(plan, dev<float>(kZ), dev<float>(kPoses), dev<float>(kImg), nullptr,
                                         nullptr, nullptr, nullptr, dev<void>(kWs), (size_t)wsp - 1,
                                         nullptr) == DUS_EWORKSPACE,
                           "plan short workspace");
                    dus_plan_destroy(plan);
                }
            }
        }
    dus_plan_destroy(nullptr);

    // a launch that fails inside a two-chain step (captured, and eager): the
    // step reports it, every fork into the second stream is joined back (the
    // capture ends cleanly; eagerly, no work is left on the second stream
    // that the caller's stream does not wait for), and the plan then steps
    // as before
    {
        const dus_physics pf = physics(1, 1);
        std::vector<dus_fan> ff = fans(4, 5, 100);
        for (int flags : {0, (int)DUS_PLAN_NO_GRAPH, (int)(DUS_PLAN_NO_GRAPH | DUS_PLAN_POSE_ONLY)}) {
            dus_plan *plan = nullptr;
            expect(dus_plan_create(&plan, &v, ff.data(), 4, &pf, flags) == DUS_OK, "plan create (failures)");
            const int64_t wsp = dus_plan_workspace_bytes(plan);
            uintptr_t img = kImg;
            auto step = [&]() {
                img += 0x1000;              // a new image pointer: the graph is captured again
                return dus_plan_step(plan, dev<float>(kZ), dev<float>(kPoses), dev<float>(kImg + 0x800000),
                                     dev<float>(img), dev<double>(kGrad),
                                     (flags & DUS_PLAN_POSE_ONLY) ? nullptr : dev<float>(kGrad + 0x200000),
                                     dev<float>(kGrad + 0x100000), dev<void>(kWs), (size_t)wsp, nullptr);
            };
            const long l0 = stub_launches();
            expect(step() == DUS_OK, "step before failures");
            const long per_step = stub_launches() - l0;
            expect(per_step >= 8, "a two-chain step launches its kernels");
            for (long k = 1; k <= per_step; ++k) {
                stub_fail_launch(k);
                expect(step() == DUS_EHIP, "failed launch reported");
                stub_fail_launch(0);
                expect(stub_unjoined_captures() == 0, "capture ended with every fork joined");
                expect(stub_open_work() == 0, "no work left unjoined on the second stream");
                expect(step() == DUS_OK, "step after a failed one");
            }
            dus_plan_destroy(plan);
        }
    }

    // invalid requests: a negative status, nothing launched
    const dus_physics p = physics(1, 1);
    std::vector<dus_fan> f = fans(2, 4, 50);
    const int before = g_launches;
    dus_volume bad = volume(2, 2, 1 << 24);
    expect(dus_render_bmode(dev<float>(kZ), &bad, dev<float>(kPoses), f.data(), 2, &p, dev<float>(kImg), nullptr,
                            dev<void>(kWs), 1 << 30, nullptr) == DUS_EUNSUPPORTED,
           "nz limit");
    bad = volume(1 << 12, 1 << 12, 2);
    expect(dus_workspace_bytes(&bad, f.data(), 2, &p, 0) == DUS_EUNSUPPORTED, "slice limit");
    bad = volume(1 << 11, 1 << 11, 1 << 10);
    expect(dus_workspace_bytes(&bad, f.data(), 2, &p, 0) == DUS_ESHAPE, "2^31 voxels");
    std::vector<dus_fan> g = f;
    g[1].out_offset = INT64_MAX - 10;            // the block's end does not fit int64
    expect(dus_workspace_bytes(&v, g.data(), 2, &p, 0) == DUS_ESHAPE, "offset overflow");
    g = f;
    g[0].n_samples = DUS_MAX_SAMPLES + 1;
    expect(dus_workspace_bytes(&v, g.data(), 2, &p, 0) == DUS_ESHAPE, "too many samples");
    g = f;
    g[0].n_rays = DUS_MAX_RAYS;
    g[0].n_samples = DUS_MAX_SAMPLES;
    g[1].out_offset = (int64_t)DUS_MAX_RAYS * DUS_MAX_SAMPLES;
    expect(dus_workspace_bytes(&v, g.data(), 2, &p, 1) > 0, "largest fan");
    dus_physics q = p;
    q.blur_sigma1 = 1e30f;
    expect(dus_workspace_bytes(&v, f.data(), 2, &q, 0) == DUS_EUNSUPPORTED, "huge blur");
    q = p;
    q.spk_cell = 1 << 30;
    expect(dus_workspace_bytes(&v, f.data(), 2, &q, 0) == DUS_EINVAL, "huge cell");
    dus_plan *plan = reinterpret_cast<dus_plan *>(1);
    expect(dus_plan_create(&plan, &v, f.data(), 2, &p, 1 << 10) == DUS_EINVAL && plan == nullptr, "plan flag");
    std::vector<dus_fan> big = fans(1, 4096, 2048);          // 8 M ray-samples: beyond the static scratch
    expect(dus_render_bmode_backward_static(dev<float>(kZ), &v, dev<float>(kPoses), big.data(), 1, &p,
                                            dev<float>(kImg), dev<float>(kGrad), nullptr, nullptr) == DUS_EUNSUPPORTED,
           "static scratch too small");
    expect(g_launches == before, "nothing launched on invalid requests");

    // the smaller entry points
    dus_grid2d grid = {64, 48, -10.0f, 0.0f, 0.5f, 0.5f, 0.0f};
    expect(dus_scan_convert(dev<float>(kImg), &f[0], &grid, dev<float>(kGrad), nullptr) == DUS_OK, "scan convert");
    grid.nx = 1 << 20;
    grid.nz = 1 << 20;
    expect(dus_scan_convert(dev<float>(kImg), &f[0], &grid, dev<float>(kGrad), nullptr) == DUS_ESHAPE, "big grid");
    const int64_t sws = dus_smoothness_workspace_bytes(&v);
    expect(sws > 0 && dus_smoothness(dev<float>(kZ), &v, 0.1f, dev<float>(kGrad), nullptr, dev<void>(kWs),
                                     (size_t)sws, nullptr) == DUS_OK,
           "smoothness");
    expect(dus_adam_step(dev<float>(kZ), dev<float>(kGrad), dev<float>(kImg), dev<float>(kWs), 1000, 0.1f, 0.9f,
                         0.999f, 1e-8f, 3, 0.5f, 12.0f, nullptr) == DUS_OK,
           "adam");
    expect(dus_adam_step(dev<float>(kZ), dev<float>(kGrad), dev<float>(kImg), dev<float>(kWs), 1000, 0.1f, 0.9f,
                         0.999f, 1e-8f, 0, 0.5f, 12.0f, nullptr) == DUS_EINVAL,
           "adam step 0");
    dus_lut lut;
    memset(&lut, 0, sizeof(lut));
    lut.n = DUS_MAX_KNOTS;
    for (int j = 0; j < DUS_MAX_KNOTS; ++j) {
        lut.x[j] = (float)j;
        lut.z[j] = 1.0f + 0.01f * (float)j;
    }
    expect(dus_map_impedance(dev<float>(kImg), 4096, &lut, dev<float>(kZ), nullptr) == DUS_OK, "map");
    expect(dus_map_impedance_backward(dev<float>(kImg), 4096, &lut, dev<float>(kGrad), dev<float>(kZ),
                                      dev<double>(kWs), nullptr) == DUS_OK,
           "map adjoint");
    lut.n = DUS_MAX_KNOTS + 1;
    expect(dus_map_impedance(dev<float>(kImg), 4096, &lut, dev<float>(kZ), nullptr) == DUS_EINVAL, "lut size");
    expect(dus_footprint_mask(&v, dev<float>(kPoses), f.data(), 2, dev<uint8_t>(kGrad), nullptr) == DUS_OK,
           "footprint");
    expect(dus_sample_volume(dev<float>(kZ), &v, dev<float>(kPoses), f.data(), 2, dev<float>(kImg), nullptr) == DUS_OK,
           "sample");
    expect(dus_philox4x32_10(dev<uint32_t>(kImg), 100, 5, dev<uint32_t>(kGrad), nullptr) == DUS_OK, "philox");
    expect(dus_pixel_gain(&f[0], &p, dev<float>(kImg), nullptr) == DUS_OK, "gain");
    dus_schedule sc = {8, 4, 16, 0}, got;
    expect(dus_set_schedule(&sc) == DUS_OK && dus_get_schedule(&got) == DUS_OK, "schedule");
    sc.bwd_chunk = 16;
    expect(dus_set_schedule(&sc) == DUS_EINVAL, "bad schedule");

    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("abi driver: ok, %d launches\n", g_launches);
    return 0;
}
