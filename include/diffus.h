/*
 * diffus.h -- C ABI of the MI355X (gfx950) DiffUS fan-beam renderer.
 *
 * The renderer follows arXiv 2508.06768 ("DiffUS: Differentiable Ultrasound
 * Rendering from Volumetric Imaging"):
 *   - Sec. 2.1, Eq. 1: interface coefficients R = |Z2-Z1|/(Z1+Z2),
 *     T = 2 Z2/(Z1+Z2) (a signed-R mode is offered as an option);
 *   - Sec. 2.1: straight rays, uniform attenuation;
 *   - Sec. 2.3, Eq. 2-4: coupled forward/backward amplitudes per ray, solved
 *     for every truncation depth k (Sec. 2.4) -- here by an O(S) composition
 *     of the per-interface 2x2 transfer maps, computed in FP64;
 *   - Sec. 2.4: fan of rays from one virtual transducer, pixel = first
 *     difference of the depth-resolved echo, optional depth-dependent speckle
 *     and lateral blur;
 *   - Sec. 1 / abstract: differentiable, for registration and reconstruction:
 *     gradients with respect to the impedance volume and the probe pose.
 *
 * Conventions
 *   Volume Z[nz][ny][nx] FP32 (MRayl, > 0, finite), x fastest.  Voxel (i,j,k)
 *   has its centre at origin + (i hx, j hy, k hz) mm.  Sampling is trilinear
 *   with clamp-to-edge.
 *   Pose p: 6 FP32 values (t_x, t_y, t_z [mm], w_x, w_y, w_z [rad]) mapping a
 *   probe point q to world t + R(w) q, R(w) = exp([w]x).  In the probe frame
 *   ray j of a fan of n rays has direction (sin th_j, 0, cos th_j),
 *   th_j = -A/2 + j A/(n-1) (th = 0 when n = 1); sample k sits at
 *   s_k = r0 + k ds.
 *   B-mode image of pose p: FP32 [n_rays][n_samples] starting at element
 *   fans[p].out_offset of the output array; pixel k of a ray is the echo of
 *   the interface between samples k-1 and k (pixel 0 is 0).
 *
 * Memory and streams
 *   Pointers named Z, poses, bmode, grad_*, target, ws, counters, out are
 *   DEVICE pointers; dus_volume / dus_fan / dus_physics arguments are HOST
 *   pointers.  The caller owns every buffer, including the workspace; the
 *   library never allocates device memory in a render call and never
 *   synchronises the stream: all work is enqueued on `stream` (a
 *   hipStream_t; NULL is the default stream).  Plans (dus_plan_*) own a
 *   captured HIP graph and a private capture stream.
 *
 * Errors
 *   Host-side validation runs before anything is enqueued; on failure a
 *   negative dus_status is returned and nothing is enqueued.  HIP failures
 *   return DUS_EHIP; dus_last_error() gives the detail (per thread).
 *   Numerical hazards are not errors: NaN/Inf propagate.  With the |R|
 *   convention of Eq. 1 the per-ray system can approach singularity (a
 *   pole of the echo); ray_min_pivot reports how close each ray came.
 */
#ifndef DIFFUS_H
#define DIFFUS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DUS_OK = 0,
    DUS_EINVAL = -1,       /* null pointer, bad enum, non-finite parameter */
    DUS_ESHAPE = -2,       /* sizes out of range or inconsistent */
    DUS_EWORKSPACE = -3,   /* workspace missing or too small */
    DUS_EHIP = -4,         /* a HIP runtime call failed */
    DUS_EUNSUPPORTED = -5  /* valid request the library does not handle */
} dus_status;

enum { DUS_REFL_ABS = 0, DUS_REFL_SIGNED = 1 };
enum { DUS_ATTEN_IN_SYSTEM = 0, DUS_ATTEN_POST_HOC = 1, DUS_ATTEN_OFF = 2 };

/* Limits checked by validation. */
#define DUS_MAX_SAMPLES 16384      /* samples per ray */
#define DUS_MAX_RAYS 65536         /* rays per fan */
#define DUS_MAX_BLUR_RADIUS 32     /* ceil(3 * max(sigma0, sigma1)) */

typedef struct {
    int32_t nx, ny, nz;            /* voxels per axis, each >= 2, and nx * ny * nz < 2^31
                                      (else DUS_ESHAPE); nx * ny < 2^24 and nz < 2^24
                                      (else DUS_EUNSUPPORTED) */
    float spacing_mm[3];           /* > 0 */
    float origin_mm[3];            /* world position of voxel (0,0,0)'s centre */
} dus_volume;

typedef struct {
    int32_t n_rays;                /* >= 0 (0: the pose renders nothing) */
    int32_t n_samples;             /* >= 0, <= DUS_MAX_SAMPLES */
    float aperture_rad;            /* full fan angle, finite */
    float ds_mm;                   /* depth step, > 0 */
    float r0_mm;                   /* apex-to-first-sample distance, finite */
    int32_t speckle_id;            /* speckle stream of this fan (counter word 2) */
    int64_t out_offset;            /* element offset of this pose's image, >= 0;
                                      out_offset + n_rays * n_samples <= 2^48 */
} dus_fan;

typedef struct {
    float alpha_db_cm_mhz;         /* attenuation, >= 0 */
    float f_mhz;                   /* centre frequency, >= 0 */
    int32_t refl_mode;             /* DUS_REFL_ABS (Eq. 1 as printed) or DUS_REFL_SIGNED */
    int32_t atten_mode;            /* DUS_ATTEN_* */
    int32_t speckle_on;            /* 0/1 */
    int32_t spk_cell;              /* radial speckle cell, samples, >= 4 */
    float spk_Ar, spk_gamma;       /* radial amplitude and depth exponent */
    float spk_Ag0, spk_Ag1;        /* granular amplitude at zero and full depth */
    int32_t blur_on;               /* 0/1 */
    float blur_sigma0, blur_sigma1;/* lateral blur sigma (rays) at first/last depth */
    int32_t reserved;              /* must be 0 */
    uint64_t seed;                 /* Philox key = (seed low, seed high) */
} dus_physics;

/* Status text and the last HIP error detail of the calling thread. */
const char *dus_status_string(int status);
const char *dus_last_error(void);
int dus_version(void);

/*
 * Workspace size in bytes for dus_render_bmode (with_backward = 0) or for
 * dus_render_bmode_backward (with_backward = 1) with these arguments.
 * Returns a negative dus_status on invalid arguments.
 */
int64_t dus_workspace_bytes(const dus_volume *vol, const dus_fan *fans, int32_t n_poses,
                            const dus_physics *phys, int32_t with_backward);

/*
 * Forward render (Sec. 2.3-2.4) of n_poses fans in one batched launch.
 *   Z        device, FP32 [nz][ny][nx]
 *   poses    device, FP32 [n_poses][6]
 *   fans     host, n_poses records; output blocks must not overlap
 *   bmode    device, FP32; pose p writes [n_rays][n_samples] at out_offset
 *   ray_min_pivot  device, FP32 [total rays] in pose-major ray order, or
 *            NULL.  Per ray: min_k |P_{k+1}[1][1] / P_k[1][1]|, the pivots of
 *            the top-down elimination of the truncated systems (ratios of
 *            consecutive determinants of Eq. 4); 0 means a singular system,
 *            and a ray of one sample (no interface) reports +inf.
 *   ws       device workspace of at least dus_workspace_bytes(..., 0) bytes
 *            (may be NULL when that size is 0)
 */
int dus_render_bmode(const float *Z, const dus_volume *vol, const float *poses,
                     const dus_fan *fans, int32_t n_poses, const dus_physics *phys,
                     float *bmode, float *ray_min_pivot, void *ws, size_t ws_bytes,
                     void *stream);

/*
 * Exact gradient of dus_render_bmode (hand-written adjoint).  The paper
 * builds the renderer to be differentiable so that B-mode losses can drive
 * slice-to-volume registration (a gradient with respect to the probe pose)
 * and volumetric reconstruction (a gradient with respect to the impedance
 * volume): Sec. 1 and Sec. 4.  This call differentiates every step of
 * Sec. 2.3-2.4 as dus_render_bmode computes it: the Eq. 1 coefficients of
 * the trilinear samples, the depth-resolved solves of Eq. 2-4, the first
 * differences, attenuation, speckle gains and the lateral blur.
 *   grad_bmode  device FP32, dL/d(bmode), same layout as bmode
 *   grad_Z      device FP32 [nz][ny][nx] or NULL: dL/dZ is ADDED (+=)
 *   grad_pose   device FP32 [n_poses][6] or NULL: dL/dpose, OVERWRITTEN
 *   ws          at least dus_workspace_bytes(..., 1) bytes
 * The forward is recomputed inside; nothing from dus_render_bmode is reused.
 * grad_Z accumulation uses FP32 atomics (order-dependent rounding).
 */
int dus_render_bmode_backward(const float *Z, const dus_volume *vol, const float *poses,
                              const dus_fan *fans, int32_t n_poses, const dus_physics *phys,
                              const float *grad_bmode, float *grad_Z, float *grad_pose,
                              void *ws, size_t ws_bytes, void *stream);

/*
 * dus_render_bmode_backward for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and results, with the workspace taken
 * from a static device array of DUS_STATIC_SCRATCH_BYTES per GPU instead of
 * a caller buffer.  The caller still passes every input and output.  The
 * call allocates nothing: the array is part of the library's code object,
 * and each GPU that runs the library holds its own copy until the process
 * ends (its address is looked up on the first call on each device).
 * Returns DUS_EUNSUPPORTED when dus_workspace_bytes(..., 1) exceeds
 * DUS_STATIC_SCRATCH_BYTES.  Every call on one GPU shares that GPU's array,
 * which keeps the last call's contents (each call overwrites what it
 * reads): calls that overlap on one GPU (on different streams, or from
 * different threads) race and must be serialised by the caller.
 */
#define DUS_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
int dus_render_bmode_backward_static(const float *Z, const dus_volume *vol, const float *poses,
                                     const dus_fan *fans, int32_t n_poses, const dus_physics *phys,
                                     const float *grad_bmode, float *grad_Z, float *grad_pose, void *stream);

/*
 * Philox4x32-10 (Salmon et al., SC'11), the generator of the speckle
 * multipliers (Sec. 2.4).  counters: device uint32 [n][4]; out: device
 * uint32 [n][4]; key = (seed low 32 bits, seed high 32 bits).
 */
int dus_philox4x32_10(const uint32_t *counters, int64_t n, uint64_t seed, uint32_t *out,
                      void *stream);

/*
 * Per-pixel gain applied to the raw echo of one fan: post-hoc attenuation
 * (atten_mode POST_HOC) times the speckle multiplier (speckle_on), Sec. 2.4.
 * out: device FP32 [n_rays][n_samples].
 */
int dus_pixel_gain(const dus_fan *fan, const dus_physics *phys, float *out, void *stream);

/*
 * Sampling-only render (the "sampling" row of Table 1, Sec. 3): pixel k of
 * ray j is the impedance at the ray sample itself (trilinear, clamp-to-edge,
 * the positions of dus_render_bmode), with no reflection, attenuation,
 * speckle or blur.  Same arguments and image layout as dus_render_bmode;
 * out: device FP32.  Needs no workspace.
 */
int dus_sample_volume(const float *Z, const dus_volume *vol, const float *poses, const dus_fan *fans,
                      int32_t n_poses, float *out, void *stream);

/*
 * Scan conversion for display (the fan images of Fig. 3): the polar image of
 * one fan (rows = rays at angles -A/2 .. A/2, columns = depths r0 + k ds) is
 * resampled onto a Cartesian grid in the probe's x-z plane.  Output pixel
 * (iz, ix) sits at x = x0 + ix dx, z = z0 + iz dz (mm, probe frame: x
 * lateral, z along the beam axis); with r = |(x, z)| and theta = atan2(x, z)
 * its polar indices are j = (theta + A/2)(n_rays - 1)/A and k = (r - r0)/ds,
 * and its value is the bilinear interpolation of the polar image (along
 * depth, then along the rays) for 0 <= j <= n_rays - 1 and
 * 0 <= k <= n_samples - 1, else `fill`.  Needs n_rays >= 2, n_samples >= 2.
 *   bmode  device FP32, the fan's image at fan->out_offset
 *   out    device FP32 [nz][nx]
 */
typedef struct {
    int32_t nx, nz;          /* output pixels along x and z */
    float x0_mm, z0_mm;      /* position of pixel (0, 0) */
    float dx_mm, dz_mm;      /* pixel pitch (> 0) */
    float fill;              /* value outside the fan */
} dus_grid2d;

int dus_scan_convert(const float *bmode, const dus_fan *fan, const dus_grid2d *grid, float *out, void *stream);

/*
 * Volume reconstruction (the second use of the gradient that the paper names,
 * Sec. 1 and Sec. 4: recovering Z from B-modes): a smoothness prior on Z,
 *   R(Z) = weight * sum over the axes a, over the neighbour pairs
 *          (v, v + e_a) inside the volume, of ((Z[v + e_a] - Z[v]) / h_a)^2,
 * and an Adam update.  dus_smoothness adds dR/dZ to grad_Z (device FP32,
 * +=) and R to *loss (device FP64 scalar or NULL, +=).  Workspace:
 * dus_smoothness_workspace_bytes(vol) bytes (per-block energy partials),
 * 256-byte aligned.
 */
int64_t dus_smoothness_workspace_bytes(const dus_volume *vol);
int dus_smoothness(const float *Z, const dus_volume *vol, float weight, float *grad_Z, double *loss,
                   void *ws, size_t ws_bytes, void *stream);

/*
 * One Adam step (Kingma and Ba, ICLR 2015) on n FP32 parameters in place:
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   x = clamp(x - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), lo, hi),
 * t >= 1 the step count.  With lo > 0 it keeps an impedance volume positive
 * (Eq. 1 needs Z > 0).  x, m, v are updated; grad is read.
 */
int dus_adam_step(float *x, const float *grad, float *m, float *v, int64_t n, float lr, float beta1,
                  float beta2, float eps, int32_t t, float lo, float hi, void *stream);

/*
 * Impedance mapping (Sec. 2.2: the paper turns MRI or CT intensities into an
 * impedance volume voxel by voxel, with a learned or tabulated map).  Here
 * the map is a piecewise-linear table of n knots (x_j, z_j), x strictly
 * increasing, constant beyond its ends:
 *   Z = z_0 for v <= x_0,  z_{n-1} for v >= x_{n-1},
 *   Z = z_j + t (z_{j+1} - z_j), t = (v - x_j) / (x_{j+1} - x_j) for
 *   x_j <= v < x_{j+1}; NaN stays NaN.
 * The renderer needs Z > 0, which positive z_j give.  The table is a HOST
 * record (2 <= n <= DUS_MAX_KNOTS, finite values, else DUS_EINVAL);
 * intensities and Z are DEVICE FP32 arrays of n_vox elements.  The
 * calibration itself (the paper's training pairs and MLP) is not given.
 */
#define DUS_MAX_KNOTS 64
typedef struct {
    int32_t n;
    float x[DUS_MAX_KNOTS];        /* intensities, strictly increasing */
    float z[DUS_MAX_KNOTS];        /* impedances (MRayl) */
} dus_lut;

int dus_map_impedance(const float *intensity, int64_t n_vox, const dus_lut *lut, float *Z, void *stream);

/*
 * Adjoint of dus_map_impedance for dL/dZ (device FP32, n_vox):
 *   grad_intensity (device FP32 or NULL, overwritten):
 *     dL/dZ (z_{j+1} - z_j) / (x_{j+1} - x_j) inside the table (the segment to
 *     the right at a knot), 0 beyond its ends;
 *   grad_z (device FP64 [lut->n] or NULL, +=): dL/dz_j summed over the voxels.
 */
int dus_map_impedance_backward(const float *intensity, int64_t n_vox, const dus_lut *lut, const float *grad_Z,
                               float *grad_intensity, double *grad_z, void *stream);

/*
 * Footprint of the rendering: mask[v] = 1 for every voxel v that is a corner
 * of the trilinear stencil of some sample of some ray (other entries are left
 * untouched).  mask: device uint8 [nz][ny][nx].  Used to count the distinct
 * voxels a render must read (the compulsory volume traffic).
 */
int dus_footprint_mask(const dus_volume *vol, const float *poses, const dus_fan *fans,
                       int32_t n_poses, uint8_t *mask, void *stream);

/*
 * Batched fused step: forward, loss = sum over poses of mean((I - target)^2),
 * adjoint.  One step is one iteration of the gradient-based registration or
 * reconstruction the paper names as the renderer's purpose (Sec. 1, Sec. 4):
 * the B-modes of many probe poses are rendered as in Sec. 2.3-2.4 (Eq. 1-4,
 * fan geometry, attenuation, speckle, blur), compared with target images,
 * and the loss is differentiated with respect to the impedance volume and
 * the poses (as dus_render_bmode_backward does).  The paper prints no loss;
 * the mean squared error per pose is this library's choice.  A plan fixes
 * the volume shape, the fans and the physics; each dus_plan_step replays one
 * captured HIP graph on `stream`.
 */
typedef struct dus_plan dus_plan;

enum {
    DUS_PLAN_POSE_ONLY = 1,   /* grad_Z is neither needed nor touched */
    DUS_PLAN_ZERO_GRAD_Z = 2, /* the step clears grad_Z itself (fill kernel) */
    DUS_PLAN_NO_GRAPH = 4,    /* launch eagerly instead of replaying a graph */
    DUS_PLAN_DETERMINISTIC = 8, /* dL/dZ bit-identical from step to step: summed as 64-bit fixed
                                   point (scale 2^e set per step from the sum of |dL/dZ| over all
                                   samples, so no sum can overflow) and rounded once to FP32,
                                   instead of FP32 atomics; costs 8 B per voxel of workspace */
    DUS_PLAN_ONE_STREAM = 16   /* every launch on the step's stream, the fans in tables of up to 64
                                  (by default a plan of two or more fans runs them as two chains of
                                  launches, half the fans each, on the step's stream and a second
                                  one, and long rays' launches beside the others) */
};

/* Ray-to-wavefront schedule; 0 fields select the library default. */
typedef struct {
    int32_t fwd_chunk;        /* interfaces per lane per tile, forward: 4, 8 or 16; 0 (the default)
                                 picks 8 per fan table, or 4 when the table's rays fill 512-sample
                                 tiles more than 7% worse than 256-sample ones */
    int32_t bwd_chunk;        /* same for the adjoint: 4 or 8 */
    int32_t xcd_group;        /* consecutive rays kept on one XCD: 1..64 */
    int32_t scatter_rays;     /* neighbouring rays per wavefront (one LDS box) in the dL/dZ scatter:
                                 2, 4 or 8; 0 (the default) picks 8, or 2 when even the shortest
                                 depth segments would give fewer than 2048 wavefronts */
    int32_t span_samples;     /* rays of at least this many samples are walked by several
                                 wavefronts each, which take consecutive tiles of the ray together
                                 (forward; the plan's adjoint): 1..DUS_MAX_SAMPLES, 0 (the default)
                                 for 4096, -1 for never.  Results do not depend on it, except for
                                 the rounding of the pose gradient and of the fused loss */
} dus_schedule;

/* Process-wide schedule used by dus_render_bmode / dus_render_bmode_backward
 * (plans carry their own).  Not thread-safe against concurrent render calls. */
int dus_set_schedule(const dus_schedule *sched);
int dus_get_schedule(dus_schedule *sched);

/*
 * A plan for the fused step above: the volume record, the n_poses fan
 * records and the physics (all HOST, copied into the plan) are validated as
 * for dus_render_bmode, and flags is a combination of DUS_PLAN_*.  *out
 * receives the plan (NULL on failure); the caller destroys it with
 * dus_plan_destroy.  Creating a plan allocates host memory, two HIP streams
 * (graph capture; the launches of rays of at least span_samples samples,
 * forked from and joined back into the step's stream) and two events on the
 * current device, never device memory.
 */
int dus_plan_create(dus_plan **out, const dus_volume *vol, const dus_fan *fans,
                    int32_t n_poses, const dus_physics *phys, int32_t flags);
/* The plan's workspace holds, besides the images of the step, what the
 * forward hands to the adjoint: per ray, 4 doubles + 1 int32 per 256-sample
 * block (tile carries), (v0, v1, D) as 3 doubles per 4 samples (chunk
 * states), one FP32 gain per pixel (with speckle or post-hoc attenuation),
 * and 9 doubles of pose partials: about 10 B per ray-sample, on top of the
 * step's images (4 B per pixel each: the pre-blur image, the residual and
 * its blur transpose with blur on, and the per-sample dL/dZ, which a
 * DUS_PLAN_POSE_ONLY plan does not keep). */
int64_t dus_plan_workspace_bytes(const dus_plan *plan);
int dus_plan_set_schedule(dus_plan *plan, const dus_schedule *sched);
int dus_plan_get_schedule(const dus_plan *plan, dus_schedule *sched);
/*
 * One fused step of the plan (Sec. 2.3-2.4 forward, MSE, adjoint; see above)
 * on `stream`: the first call, and any call whose pointers or workspace size
 * differ from the previous call's, captures a new HIP graph; the others
 * replay it.  Unless the plan was created with DUS_PLAN_ONE_STREAM, the step
 * also runs launches on the plan's second stream (two chains of launches,
 * or the long rays' launches), forked from `stream` and joined back into it
 * before the step's last launch, so the step is ordered on `stream` all the
 * same; two steps of one plan must not run at the same time.  Z and poses
 * as for dus_render_bmode; the workspace has at least
 * dus_plan_workspace_bytes(plan) bytes, 256-byte aligned.
 *   target   device FP32, same layout as bmode
 *   bmode    device FP32 or NULL: the rendered image is also written
 *   loss     device FP64 scalar or NULL: receives the loss (overwritten)
 *   grad_Z   device FP32 or NULL (+=; cleared first with DUS_PLAN_ZERO_GRAD_Z)
 *   grad_pose device FP32 [n_poses][6] or NULL (overwritten)
 */
int dus_plan_step(dus_plan *plan, const float *Z, const float *poses, const float *target,
                  float *bmode, double *loss, float *grad_Z, float *grad_pose,
                  void *ws, size_t ws_bytes, void *stream);

/*
 * Phases of a plan step, in launch order (measurement and tracing):
 *   CLEAR      fill kernel for the pose accumulators and grad_Z, when the
 *              forward kernel does not run (else its wavefronts clear them)
 *   FORWARD    forward kernel (pixels, tile carries, per-pixel gains)
 *   BLUR_LOSS  blur, MSE residual and loss partials, blur transpose (blur on)
 *   ADJOINT    adjoint scan kernel (dL/dZ per sample, pose sums; with blur
 *              off it also forms the loss partials)
 *   SCATTER    trilinear scatter of dL/dZ into grad_Z
 *   FINISH     loss reduction and pose-gradient kernel
 */
enum {
    DUS_PHASE_CLEAR = 0,
    DUS_PHASE_FORWARD = 1,
    DUS_PHASE_BLUR_LOSS = 2,
    DUS_PHASE_ADJOINT = 3,
    DUS_PHASE_SCATTER = 4,
    DUS_PHASE_FINISH = 5,
    DUS_NUM_PHASES = 6
};

/*
 * dus_plan_step without graph replay and on `stream` alone (one chain of
 * launches), with a HIP event recorded on `stream` at every phase boundary.
 * Same arguments and results as dus_plan_step;
 * ms[DUS_PHASE_*] receives each phase's duration in milliseconds (0 for a
 * phase the step does not run).  Blocks the calling thread until the step
 * has finished on the device.  Creates and destroys its events (no device
 * memory is allocated).
 */
int dus_plan_step_timed(dus_plan *plan, const float *Z, const float *poses, const float *target,
                        float *bmode, double *loss, float *grad_Z, float *grad_pose,
                        void *ws, size_t ws_bytes, void *stream, float *ms);
void dus_plan_destroy(dus_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* DIFFUS_H */
