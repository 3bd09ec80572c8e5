// Internal launch records shared by the HIP kernels and the host ABI layer.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace dus {

// Fans per launch: the fan table travels in the kernel arguments.
constexpr int kMaxFans = 64;
// rays of at least span_samples samples (kSpanSamples by default; <= 0:
// none) are walked by kSpanWaves wavefronts each, which take consecutive
// tiles of the ray together (forward and plan adjoint); shorter rays by one
// wavefront
constexpr int kSpanSamples = 4096;
constexpr int kSpanWaves = 8;

struct FanRec {
    int32_t n_rays, n_samples;
    float aperture, ds, r0;
    int32_t speckle_id;
    int64_t out_offset;     // element offset of the [n_rays][n_samples] image
    int32_t ray_begin;      // first launch-wide ray index of this fan
    int32_t blk_begin;      // first blur block of this fan
    int32_t pose;           // row of the poses array
    int32_t pivot_begin;    // pose-major index of this fan's first ray
    int32_t carry_begin;    // first tile-carry record of this fan's first ray
    int32_t unit_begin;     // first wavefront of this fan in a scatter launch (set by launch_scatter)
};
static_assert(sizeof(FanRec) == 56, "FanRec layout");

// Tile carries: the forward kernel records, at every 256-sample boundary of
// a ray, the carried row vector and determinant (v0, v1, D) and the sample
// before the boundary, in the scale of the forward tile that holds the
// boundary.  Each record's exponent gives that scale relative to the
// previous record's: zero inside a forward tile, the tile's renormalisation
// (a power of two) at its first record.  The adjoint then starts its
// reverse sweep from these records instead of re-running the forward.
constexpr int kCarryBlock = 256;
inline int64_t carry_records(int32_t n_rays, int32_t n_samples)
{
    return (int64_t)n_rays * ((n_samples + kCarryBlock - 1) / kCarryBlock);
}

// Chunk states: the forward kernel also records (v0, v1, D) at every 4th
// sample, in the frame of that sample's carry record, so that the adjoint
// needs neither its own chunk products nor its prefix scan.  Each carry
// record owns kStatesPerBlock states stored component-major (all v0, all v1,
// all D): 3 * 64 doubles per record.
constexpr int kStateStride = 4;
constexpr int kStatesPerBlock = kCarryBlock / kStateStride;
constexpr int kStateDoubles = 3 * kStatesPerBlock;

struct FanTable {
    int32_t n;              // fans in this launch
    int32_t total_rays;
    int32_t total_blur_blocks;
    int32_t ray0;           // forward and adjoint, one wavefront per ray: rays below ray0 are
                            // another launch's (their wavefronts return at once)
    FanRec f[kMaxFans];
};

// A ray's geometry, written by the adjoint kernel (which sets it up from the
// pose and the fan) for the dL/dZ scatter: sample k sits at voxel coordinate
// u0 + k du.
struct RayRec {
    double u0[3], du[3];
};
static_assert(sizeof(RayRec) == 48, "RayRec layout");

struct VolArgs {
    const float *Z;
    int32_t nx, ny, nz, pad_;
    float h[3];
    float o[3];
};

struct PhysArgs {
    float alpha, freq;
    int32_t refl, atten;
    int32_t speckle, cell;
    float Ar, gam, Ag0, Ag1;
    int32_t blur;
    float s0, s1;
    uint32_t key0, key1;
    int32_t blur_rmax;      // ceil(3 * max sigma), <= DUS_MAX_BLUR_RADIUS
};

// Per-pose accumulator of the adjoint: dL/dt (3) and dL/dR (9), FP64.
constexpr int kPoseAcc = 12;
// Per-ray partial of the adjoint: dL/dt (3) and the two non-zero columns of
// dL/dR (the ray direction has no y component in the probe frame), FP64.
constexpr int kRayPart = 9;

// Launch wrappers (kernels.hip).  All enqueue on `st` and return the HIP
// error of the launch.
// carry / carry_exp: optional tile-carry records (4 doubles / 1 int each);
// cstate: optional chunk states (kStateDoubles per carry record; needs carry);
// gain: optional per-pixel gain (speckle x post-hoc attenuation) output
// Buffers a kernel clears on the side (a[0..na) and b[0..nb) set to zero)
// A second stream for the launch of the long rays (several wavefronts per
// ray), forked from and joined back into the launch stream with two events,
// so that it runs beside the one-wavefront launch of the other rays.
struct SideStream {
    hipStream_t st;
    hipEvent_t fork, join;
};

struct ZeroArgs {
    float *a;
    long long na;
    double *b;
    long long nb;
};

// zero: cleared by the forward's wavefronts besides their rays (the fused
// step's dL/dZ and pose accumulators), or {} for none
hipError_t launch_forward(int chunk, int xcd_group, const VolArgs &v, const PhysArgs &p,
                          const FanTable &t, const float *poses, float *out,
                          float *min_pivot, int pivot_base, double *carry, int32_t *carry_exp,
                          double *cstate, float *gain, hipStream_t st, const ZeroArgs &zero = ZeroArgs{},
                          int span_samples = kSpanSamples, const SideStream *side = nullptr);
// adjoint: dL/dZ per sample into zbar (image layout), then its scatter; in
// the fused form (target given) loss receives one partial per ray.  With
// pose_acc (a flag here), pose_part receives kRayPart doubles per ray of the
// table; launch_pose_reduce then adds them into the pose accumulators.
// rays: one RayRec per ray of the table, written by the adjoint when zbar is
// (the scatter reads them)
hipError_t launch_backward(int chunk, int xcd_group, int scatter_rays, const VolArgs &v,
                           const PhysArgs &p, const FanTable &t, const float *poses, RayRec *rays,
                           const float *gsrc, const float *target, float *zbar, float *gZ,
                           double *pose_acc, double *pose_part, double *loss, const double *carry,
                           const int32_t *carry_exp, const double *cstate, const float *gain,
                           hipStream_t st);
// the two halves of launch_backward: the adjoint scan (dL/dZ per sample into
// zbar, pose sums, fused loss partials) and the scatter of zbar into gZ
hipError_t launch_adjoint(int chunk, int xcd_group, const VolArgs &v, const PhysArgs &p,
                          const FanTable &t, const float *poses, RayRec *rays, const float *gsrc,
                          const float *target, float *zbar, double *pose_acc, double *pose_part, double *loss,
                          const double *carry, const int32_t *carry_exp, const double *cstate,
                          const float *gain, hipStream_t st, int span_samples = kSpanSamples,
                          const SideStream *side = nullptr);
// pose_acc[pose] += the sum of the table's per-ray partials, one wavefront
// per fan (fixed order)
hipError_t launch_pose_reduce(const FanTable &t, const double *pose_part, double *pose_acc, hipStream_t st);
// fix (nullable): deterministic mode, 64-bit fixed-point sums at the scale
// fscale[0] (launch_fix_scale) instead of FP32 atomics into gZ; wave_target:
// about how many wavefronts the depth segments should make (that of the
// launches running at the same time)
hipError_t launch_scatter(int scatter_rays, int xcd_group, const VolArgs &v, const FanTable &t,
                          const RayRec *rays, const float *zbar, float *gZ, hipStream_t st,
                          unsigned long long *fix = nullptr, const double *fscale = nullptr,
                          int wave_target = 32768);
// deterministic dL/dZ: part[r] = the sum of |zbar| along the table's ray r
// (one double per ray); fscale[2] = the sum of part[0..n), fscale[0..1] =
// 2^e and 2^-e from it; the conversion of the fixed-point sums into gZ
// (overwritten or added)
hipError_t launch_abs_rows(const FanTable &t, const float *zbar, double *part, hipStream_t st);
hipError_t launch_fix_scale(const double *part, int64_t n, double *fscale, hipStream_t st);
hipError_t launch_fix_to_f32(const unsigned long long *fix, int64_t n, const double *fscale, float *gZ,
                             bool overwrite, hipStream_t st);
hipError_t launch_blur(bool transpose, const PhysArgs &p, const FanTable &t, const float *in,
                       float *out, hipStream_t st);
// image = B pre (optional), ebar = B^T (2 (image - target) / P); loss
// receives one MSE partial per blur block (total_blur_blocks entries)
hipError_t launch_blur_residual(const PhysArgs &p, const FanTable &t, const float *pre,
                                const float *target, float *image, float *resid, float *ebar,
                                double *loss, hipStream_t st);
hipError_t launch_pose_finalize(const double *acc, const float *poses, int n_poses,
                                float *grad_pose, hipStream_t st);
hipError_t launch_footprint(const VolArgs &v, const FanTable &t, const float *poses, uint8_t *mask,
                            hipStream_t st);
// impedance at every ray sample (image layout)
hipError_t launch_sample(int xcd_group, const VolArgs &v, const FanTable &t, const float *poses, float *out,
                         hipStream_t st);
// one fan's polar image onto an nz x nx grid of the probe's x-z plane
hipError_t launch_scan_convert(const float *img, int n_rays, int n_samples, double aperture, double r0,
                               double ds, int nx, int nz, double x0, double z0, double dx, double dz,
                               float fill, float *out, hipStream_t st);
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t st);
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t st);
// *out = sum of the n partials (the loss of the fused step)
hipError_t launch_sum_f64(const double *part, int64_t n, double *out, hipStream_t st, bool accumulate = false);
// loss = sum of the partials (if loss) and grad = the finalised pose
// gradients (if grad), in one launch
hipError_t launch_finish(const double *part, int64_t n_part, double *loss, const double *acc, const float *poses,
                         int n_poses, float *grad, hipStream_t st);
// a[0..na) = 0 and b[0..nb) = 0 in one launch
hipError_t launch_zero_pair(float *a, int64_t na, double *b, int64_t nb, hipStream_t st);
// smoothness prior of the reconstruction: per-axis weights w / h^2; one
// energy partial per block of 256 voxels (smooth_blocks of them)
int64_t smooth_blocks(int nx, int ny, int nz);
hipError_t launch_smooth(const float *Z, int nx, int ny, int nz, float wx, float wy, float wz, float *gZ,
                         double *part, hipStream_t st);
// Adam with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t, result clamped to [lo, hi]
hipError_t launch_adam(float *x, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, float lo, float hi, hipStream_t st);
hipError_t launch_philox(const uint32_t *ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t *out,
                         hipStream_t st);
// impedance mapping: piecewise-linear table from intensity to impedance
constexpr int kMaxKnots = 64;
struct LutArgs {
    int n;                      // knots, 2..kMaxKnots, x strictly increasing
    float x[kMaxKnots];
    float z[kMaxKnots];
};
hipError_t launch_map(const float *in, int64_t n, const LutArgs &lut, float *Z, hipStream_t st);
// grad_in (nullable): overwritten; grad_z (nullable): += per knot (FP64)
hipError_t launch_map_backward(const float *in, int64_t n, const LutArgs &lut, const float *gZ, float *grad_in,
                               double *grad_z, hipStream_t st);
hipError_t launch_pixel_gain(const PhysArgs &p, const FanRec &f, float *out, hipStream_t st);

// Static device scratch of the allocation-free entry points (a file-scope
// __device__ array of kernels.hip): *ptr receives its device address on the
// current device, looked up on the first call per device.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
hipError_t static_scratch(void **ptr);

}  // namespace dus
