// HIP kernels of the DiffUS fan-beam renderer for MI355X (gfx950, CDNA4).
//
// Method: arXiv 2508.06768.  Per ray, Eq. 1 coefficients between consecutive
// trilinear samples, the coupled amplitude system of Eq. 2-4 solved for every
// truncation depth (Sec. 2.4), pixel = first difference of the echo d_0^(k),
// fan geometry, speckle and depth-dependent lateral blur (Sec. 2.4).
//
// The truncated systems are solved through the 2x2 transfer maps of the
// back-substitution: with Gamma = d/g,
//   Gamma_i = (A Gamma_{i+1} + R) / (B Gamma_{i+1} + 1),
//   M_i = [[A, R], [B, 1]],  A = a^2 (T T' - R R'),  B = -a^2 R',
// and P_k = M_0 ... M_{k-1}.  Only the bottom row v_k = [0 1] P_k and
// D_k = det P_k are needed:
//   e_{k+1} = R_k D_k / (v_k[1] v_{k+1}[1]),  v_{k+1}[1] = v_k[0] R_k + v_k[1],
// which is the exact first difference P01/P11 |_{k+1} - P01/P11 |_k without
// subtracting nearly equal numbers.  With R = rho and R' = s rho (s = +1 for
// the |R| of Eq. 1, -1 for the signed coefficient), T T' = 1 - rho^2, so one
// number per interface describes M.
//
// Layout of the work: one wavefront per ray.  A ray is cut into tiles of
// T = 64 C samples.  Phase 1 gathers 64 consecutive samples per instruction
// (good L1/L2 locality), computes rho in FP64 and parks it in LDS.  Phase 2
// gives each lane C consecutive interfaces: chunk product, 6-step wavefront
// scan of 2x2 products, carry between tiles, walk emitting pixels into LDS.
// Phase 3 stores the tile coalesced, applying post-hoc attenuation and
// speckle.  The recurrence runs in FP64 (full rate on CDNA4 vector ALUs): the
// |R| convention makes the system nearly singular on some rays, where FP32
// would lose the 1e-5 agreement with the reference.
//
// The adjoint kernel recomputes the forward (no stored state), runs the
// reverse recurrence as an associative affine suffix scan over lanes, and
// scatters dL/dZ into the volume gradient with FP32 atomics; pose gradients
// are reduced per ray in FP64.
#include <algorithm>
#include <math.h>
#include <mutex>
#include <stdint.h>

#include "../../include/diffus.h"
#include "dus_internal.h"

namespace dus {
namespace {

// --------------------------------------------------------------------------
// wavefront helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ double lane_read(double x, int l)
{
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// a wave-uniform double made visibly uniform to the compiler (kept in SGPRs)
__device__ __forceinline__ double uniform(double x)
{
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b & 0xffffffffll));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
    return x;
}

__device__ __forceinline__ double wave_min(double x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x = fmin(x, __shfl_xor(x, d));
    return x;
}

// FP64 reciprocal: hardware estimate refined by one Newton step (the step
// squares the estimate's relative error: below 2^-44 even for a
// single-precision estimate)
__device__ __forceinline__ double rcp64(double b)
{
    const double r = __builtin_amdgcn_rcp(b);
    return fma(fma(-b, r, 1.0), r, r);
}

// partial unroll of the sample-gather loops: enough independent gathers in
// flight without holding every tile sample in registers
#ifndef GATHER_UNROLL
#define GATHER_UNROLL 4
#endif

// LDS index padding: doubles (one pad word per 16) and floats (per 32)
__device__ __forceinline__ int pad8(int i) { return i + (i >> 4); }
__device__ __forceinline__ int pad4(int i) { return i + (i >> 5); }

// blocks are handed to the 8 XCDs round-robin; keep runs of `grp`
// consecutive rays (neighbours in the fan, sharing voxels) on one XCD's L2
__device__ __forceinline__ int remap_block(int b, int G, int grp)
{
    if (grp <= 1) return b;
    const int super = 8 * grp;
    const int full = (G / super) * super;
    if (b >= full) return b;
    const int s = b / super, r = b - s * super;
    return s * super + (r & 7) * grp + (r >> 3);
}

__device__ __forceinline__ int find_fan(const FanTable &t, int g)
{
    int lo = 0, hi = t.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.f[mid].ray_begin <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_blur_fan(const FanTable &t, int b)
{
    int lo = 0, hi = t.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.f[mid].blk_begin <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// --------------------------------------------------------------------------
// geometry: probe pose -> per-ray affine sample positions in voxel units
// --------------------------------------------------------------------------
__device__ void rotation(const double w[3], double R[9])
{
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = sqrt(th2);
    double A, B;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
    }
    // R = I + A [w]x + B [w]x^2, [w]x^2 = w w^T - |w|^2 I
    R[0] = 1.0 + B * (w[0] * w[0] - th2);
    R[1] = -A * w[2] + B * w[0] * w[1];
    R[2] = A * w[1] + B * w[0] * w[2];
    R[3] = A * w[2] + B * w[1] * w[0];
    R[4] = 1.0 + B * (w[1] * w[1] - th2);
    R[5] = -A * w[0] + B * w[1] * w[2];
    R[6] = -A * w[1] + B * w[2] * w[0];
    R[7] = A * w[0] + B * w[2] * w[1];
    R[8] = 1.0 + B * (w[2] * w[2] - th2);
}

struct Ray {
    double u0[3], du[3];   // voxel coordinate of sample 0 and per-sample step
    double a2;             // round-trip amplitude over one step
    double dirx, dirz;     // probe-frame direction (y component is 0)
    double r0, ds;
    // orthonormal basis, world frame: the ray's direction D, its in-plane
    // normal T = R (cz, 0, -sx) and the fan plane's normal N = R (0, 1, 0)
    double bd[3], bt[3], bn[3];
};

// wave_uniform: every lane of the wavefront traces the same ray (its
// parameters are then kept in scalar registers)
__device__ __forceinline__ void setup_ray(const VolArgs &v, const PhysArgs &p, const FanRec &fr,
                                          const float *__restrict__ poses, int j, Ray &ray,
                                          bool wave_uniform = true)
{
    const float *ps = poses + 6 * (size_t)fr.pose;
    const double t[3] = {ps[0], ps[1], ps[2]};
    const double w[3] = {ps[3], ps[4], ps[5]};
    double R[9];
    rotation(w, R);
    const double A = fr.aperture;
    const double th = fr.n_rays > 1 ? -0.5 * A + (double)j * A / (double)(fr.n_rays - 1) : 0.0;
    const double sx = sin(th), cz = cos(th);
    const double d[3] = {R[0] * sx + R[2] * cz, R[3] * sx + R[5] * cz, R[6] * sx + R[8] * cz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ray.bd[a] = d[a];
        ray.bt[a] = R[3 * a] * cz - R[3 * a + 2] * sx;
        ray.bn[a] = R[3 * a + 1];
    }
    const double r0 = fr.r0, ds = fr.ds;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double ih = 1.0 / (double)v.h[a];
        ray.u0[a] = (t[a] + r0 * d[a] - (double)v.o[a]) * ih;
        ray.du[a] = ds * d[a] * ih;
    }
    const double amp = (p.atten == 0)
                           ? pow(10.0, -(double)p.alpha * (double)p.freq * (ds / 10.0) / 20.0)
                           : 1.0;
    ray.a2 = amp * amp;
    ray.dirx = sx;
    ray.dirz = cz;
    ray.r0 = r0;
    ray.ds = ds;
    if (!wave_uniform) return;
    // every lane computed the same values: keep them in scalar registers
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ray.u0[a] = uniform(ray.u0[a]);
        ray.du[a] = uniform(ray.du[a]);
    }
    ray.a2 = uniform(ray.a2);
    ray.dirx = uniform(ray.dirx);
    ray.dirz = uniform(ray.dirz);
    ray.r0 = uniform(ray.r0);
    ray.ds = uniform(ray.ds);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ray.bd[a] = uniform(ray.bd[a]);
        ray.bt[a] = uniform(ray.bt[a]);
        ray.bn[a] = uniform(ray.bn[a]);
    }
}

// cell index (clamped) and fraction along one axis; NaN positions clamp to 0.
// INSIDE: the caller knows u lies in [0, n-1), where the clamps change
// nothing.  u >= 0 in both cases, so truncation is the floor.
template <bool INSIDE>
__device__ __forceinline__ void axis_cell(double u, int n, int &i0, double &f)
{
    const double uc = INSIDE ? u : fmin(fmax(u, 0.0), (double)(n - 1));
    const int i = INSIDE ? (int)uc : min((int)uc, n - 2);
    i0 = i;
    // inside, u - floor(u) is exact and one instruction
    f = INSIDE ? __builtin_amdgcn_fract(uc) : uc - (double)i;
}

struct Stencil {
    int idx;               // flat index of the (x0, y0, z0) corner
    int ix, iy, iz;        // that corner's voxel coordinates
    double fx, fy, fz;
};

// a slice of the volume holds fewer than 2^24 voxels (checked on the host),
// so the flat index takes two independent 24-bit multiplies
template <bool INSIDE = false>
__device__ __forceinline__ Stencil stencil_at(const VolArgs &v, const Ray &ray, int k)
{
    Stencil s;
    const double kk = (double)k;
    axis_cell<INSIDE>(fma(kk, ray.du[0], ray.u0[0]), v.nx, s.ix, s.fx);
    axis_cell<INSIDE>(fma(kk, ray.du[1], ray.u0[1]), v.ny, s.iy, s.fy);
    axis_cell<INSIDE>(fma(kk, ray.du[2], ray.u0[2]), v.nz, s.iz, s.fz);
    s.idx = (int)(__umul24((unsigned)s.iz, (unsigned)(v.nx * v.ny)) + __umul24((unsigned)s.iy, (unsigned)v.nx)) + s.ix;
    return s;
}

// every sample k in [ka, kb] lies in [0, n-1) on every axis: the position is
// affine in k and its FP64 rounding is monotone, so the two ends decide
__device__ __forceinline__ bool segment_inside(const VolArgs &v, const Ray &ray, int ka, int kb)
{
    const int n[3] = {v.nx, v.ny, v.nz};
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double ua = fma((double)ka, ray.du[a], ray.u0[a]);
        const double ub = fma((double)kb, ray.du[a], ray.u0[a]);
        const double hi = (double)(n[a] - 1);
        in = in && (ua >= 0.0) && (ua < hi) && (ub >= 0.0) && (ub < hi);
    }
    return in;
}

__device__ __forceinline__ double lerp(double a, double b, double t) { return fma(t, b - a, a); }

// trilinear value (lerp along x, then y, then z), FP64 from FP32 corners
__device__ __forceinline__ double trilinear(const float *__restrict__ Z, int nx, int sxy,
                                            const Stencil &s, double *grad)
{
    const float *p = Z + s.idx;
    const double c000 = p[0], c100 = p[1];
    const double c010 = p[nx], c110 = p[nx + 1];
    const double c001 = p[sxy], c101 = p[sxy + 1];
    const double c011 = p[sxy + nx], c111 = p[sxy + nx + 1];
    const double a00 = lerp(c000, c100, s.fx), a10 = lerp(c010, c110, s.fx);
    const double a01 = lerp(c001, c101, s.fx), a11 = lerp(c011, c111, s.fx);
    const double b0 = lerp(a00, a10, s.fy), b1 = lerp(a01, a11, s.fy);
    if (grad) {
        const double gx0 = lerp(c100 - c000, c110 - c010, s.fy);
        const double gx1 = lerp(c101 - c001, c111 - c011, s.fy);
        grad[0] = lerp(gx0, gx1, s.fz);
        grad[1] = lerp(a10 - a00, a11 - a01, s.fz);
        grad[2] = b1 - b0;
    }
    return lerp(b0, b1, s.fz);
}

// Eq. 1 reflection coefficient between samples zl (shallower) and zr; dq
// (optional) receives d rho/d zr = dq zl and d rho/d zl = -dq zr, i.e.
// dq = 2 s / (zl + zr)^2 with s = sign(zr - zl) (ABS, sign(0) = 0) or 1
__device__ __forceinline__ double iface_rho(double zl, double zr, bool absm, double *dq = nullptr)
{
    const double sum = zl + zr, dif = zr - zl;
    const double is = rcp64(sum);
    const double q = dif * is;
    const double r = fma(fma(-sum, q, dif), is, q);
    if (dq) {
        const double sg = absm ? ((zr > zl) ? 1.0 : ((zr < zl) ? -1.0 : 0.0)) : 1.0;
        *dq = 2.0 * sg * is * is;
    }
    return absm ? fabs(r) : r;
}

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the unit-mean Rayleigh variate
// --------------------------------------------------------------------------
__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32 x 32 -> 64-bit product per multiplier (low and high words)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// unit-mean Rayleigh: sqrt(-2 ln u) sqrt(2/pi) = sqrt(-(4 ln 2 / pi) log2 u);
// u in [2^-24, 1] is a normal number, so the hardware log2 and square root
// (about 1 ulp) apply directly
__device__ __forceinline__ float rayleigh(uint32_t x)
{
    const float u = (float)((x >> 8) + 1u) * 0x1p-24f;
    return __builtin_amdgcn_sqrtf(-0.88254240061060638f * __builtin_amdgcn_logf(u));
}

// granular variates of samples 4 ctr .. 4 ctr + 3 of ray j
__device__ __forceinline__ void granular4(const PhysArgs &p, int ctr, int j, int sid, float x[4])
{
    uint32_t w[4];
    philox((uint32_t)ctr, (uint32_t)j, (uint32_t)sid, 0u, p.key0, p.key1, w);
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = rayleigh(w[q]);
}

// radial cell values covering the tile [t0, t0+T): s_xir[c - t0/cell]
template <int T>
__device__ __forceinline__ void speckle_radial(const PhysArgs &p, int t0, int j, int sid, int lane, float *s_xir)
{
    const int cell = p.cell;
    const int c_lo = t0 / cell, c_hi = (t0 + T - 1) / cell + 1;
    for (int b = (c_lo >> 2) + lane; b <= (c_hi >> 2); b += 64) {
        uint32_t w[4];
        philox((uint32_t)b, (uint32_t)j, (uint32_t)sid, 1u, p.key0, p.key1, w);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = 4 * b + q;
            if (c >= c_lo && c <= c_hi) s_xir[c - c_lo] = rayleigh(w[q]);
        }
    }
}

// Speckle inputs of one tile [t0, t0+T): granular variates per pixel and the
// radial cell values covering the tile.
template <int T>
__device__ __forceinline__ void speckle_fill(const PhysArgs &p, int t0, int j, int sid, int lane,
                                             float *s_xig, float *s_xir)
{
    for (int bb = lane; bb < T / 4; bb += 64) {
        float x[4];
        granular4(p, (t0 >> 2) + bb, j, sid, x);
        *reinterpret_cast<float4 *>(s_xig + 4 * bb) = make_float4(x[0], x[1], x[2], x[3]);
    }
    speckle_radial<T>(p, t0, j, sid, lane, s_xir);
}

// per-launch constants of pixel_gain: 1/(S-1) and 1/cell
struct GainK {
    float inv_sm1, inv_cell;
};

__device__ __forceinline__ GainK gain_consts(const PhysArgs &p, int S)
{
    return GainK{S > 1 ? 1.0f / (float)(S - 1) : 0.0f, 1.0f / (float)p.cell};
}

// speckle multiplier of a pixel at depth fraction zeta, cell fraction fr
// between the radial cell values x0 and x1, granular variate xg.  zeta^gam
// with zeta in [1/(S-1), 1] (a normal number); a power below 2^-126 may
// flush to zero, which leaves the FP32 gain unchanged.
__device__ __forceinline__ float speckle_mult(const PhysArgs &p, float zeta, float fr, float x0, float x1,
                                              float xg)
{
    const float xr = (1.0f - fr) * x0 + fr * x1;
    float pw;
    if (zeta > 0.0f) pw = __builtin_amdgcn_exp2f(p.gam * __builtin_amdgcn_logf(zeta));
    else pw = (p.gam == 0.0f) ? 1.0f : 0.0f;
    return 1.0f + p.Ar * pw * (xr - 1.0f) + (p.Ag0 + p.Ag1 * zeta) * (xg - 1.0f);
}

// radial cell c = k div cell and remainder r of sample k (exact: the
// reciprocal's quotient is corrected by one step either way)
__device__ __forceinline__ void cell_of(const PhysArgs &p, const GainK &gk, int k, int &c, int &r)
{
    const int cell = p.cell;
    c = (int)((float)k * gk.inv_cell);
    r = k - c * cell;
    if (r < 0) { --c; r += cell; }
    if (r >= cell) { ++c; r -= cell; }
}

// Gain of pixel k: post-hoc attenuation (POST) times speckle (SPK), with xg
// the pixel's granular variate and s_xir the radial cell values of the tile
// starting at t0.  zeta = k/(S-1) and the cell fraction come from reciprocals
// (within an ulp of the quotients); the cell index is exact.
template <bool SPK, bool POST>
__device__ __forceinline__ float pixel_gain(const PhysArgs &p, const GainK &gk, int k, int t0, float postc,
                                            float xg, const float *s_xir)
{
    float g = 1.0f;
    if (POST) g = exp2f((float)((double)k * (double)postc));
    if (SPK) {
        int c, r;
        cell_of(p, gk, k, c, r);
        const int c_lo = t0 / p.cell;
        g *= speckle_mult(p, (float)k * gk.inv_sm1, (float)r * gk.inv_cell, s_xir[c - c_lo], s_xir[c + 1 - c_lo], xg);
    }
    return g;
}

// the same with the post-hoc switch read at run time
template <bool SPK>
__device__ __forceinline__ float pixel_gain_rt(const PhysArgs &p, const GainK &gk, int k, int t0, float postc,
                                               float xg, const float *s_xir)
{
    return (p.atten == 1) ? pixel_gain<SPK, true>(p, gk, k, t0, postc, xg, s_xir)
                          : pixel_gain<SPK, false>(p, gk, k, t0, postc, xg, s_xir);
}

__device__ __forceinline__ float posthoc_coef(const PhysArgs &p, float ds)
{
    // 10^(-2 alpha f (k ds / 10) / 20) = 2^(k * postc)
    return (float)(-(double)p.alpha * (double)p.freq * (double)ds / 100.0 * 3.321928094887362);
}

// --------------------------------------------------------------------------
// phase 1: gather samples [t0, t0+T) of a ray, interface rho of (k-1, k)
// into s_rho[pad8(k - t0)]; optionally keep the samples in s_z, and the
// last sample of every 256-sample block in s_zc (tile carries).  W (the
// caller's wavefronts per ray) only keeps the callers' instances apart: the
// compiler then derives each caller's index ranges from that caller alone.
// --------------------------------------------------------------------------
template <int C, bool KEEPZ, bool KEEPG, bool INSIDE, int W>
__device__ __forceinline__ void gather_tile_body(const VolArgs &v, const Ray &ray, int t0, int S,
                                                 bool absm, int lane, double &zprev, double *s_rho,
                                                 double *s_z, float *s_g, double *s_zc, double *s_dq)
{
    constexpr int T = 64 * C;
    const int sxy = v.nx * v.ny;
    // 1 / h once per tile, not an FP64 division per sample and axis
    double ih[3] = {0.0, 0.0, 0.0};
    if (KEEPG) {
#pragma unroll
        for (int a = 0; a < 3; ++a) ih[a] = 1.0 / (double)v.h[a];
    }
#pragma unroll GATHER_UNROLL
    for (int jj = 0; jj < C; ++jj) {
        const int i = jj * 64 + lane;
        const int k = t0 + i;
        const Stencil st = stencil_at<INSIDE>(v, ray, min(k, S - 1));
        double gu[3];
        const double z = trilinear(v.Z, v.nx, sxy, st, KEEPG ? gu : nullptr);
        double zm = __shfl_up(z, 1);
        if (lane == 0) zm = zprev;
        zprev = lane_read(z, 63);
        // interface (k-1, k); outside [1, S) rho = 0 and dq = 0
        const bool ok = (k >= 1) && (k < S);
        double dq = 0.0;
        double rho = iface_rho(zm, z, absm, KEEPZ ? &dq : nullptr);
        rho = ok ? rho : 0.0;
        dq = ok ? dq : 0.0;
        s_rho[pad8(i)] = rho;
        if (KEEPZ) {
            s_z[pad8(i)] = z;
            s_dq[pad8(i)] = dq;
        }
        if (s_zc && lane == 63 && (jj & 3) == 3) s_zc[jj >> 2] = z;
        if (KEEPG) {
            // dZ/dp per mm (dZ/du / h, zero along an axis where the sample
            // lies outside the volume: clamped), kept in FP32 as its
            // components along the ray and across it (the ray's basis), so
            // that the rounding of the large component along the ray stays
            // along the ray, where it cannot reach the rotation gradient
            const double kk = (double)min(k, S - 1);
            const int n[3] = {v.nx, v.ny, v.nz};
            double gw[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double u = fma(kk, ray.du[a], ray.u0[a]);
                const bool inside = INSIDE || ((u >= 0.0) && (u <= (double)(n[a] - 1)));
                gw[a] = inside ? gu[a] * ih[a] : 0.0;
            }
            s_g[i] = (float)fma(gw[0], ray.bd[0], fma(gw[1], ray.bd[1], gw[2] * ray.bd[2]));
            s_g[T + i] = (float)fma(gw[0], ray.bt[0], fma(gw[1], ray.bt[1], gw[2] * ray.bt[2]));
            s_g[2 * T + i] = (float)fma(gw[0], ray.bn[0], fma(gw[1], ray.bn[1], gw[2] * ray.bn[2]));
        }
    }
}

template <int C, bool KEEPZ, bool KEEPG = false, int W = 1>
__device__ __forceinline__ void gather_tile(const VolArgs &v, const Ray &ray, int t0, int S,
                                            bool absm, int lane, double &zprev, double *s_rho,
                                            double *s_z, float *s_g = nullptr, double *s_zc = nullptr,
                                            double *s_dq = nullptr)
{
    // a tile whose samples all lie inside the volume skips the clamps (the
    // ray is the same on every lane, so the branch is uniform)
    if (segment_inside(v, ray, t0, min(t0 + 64 * C - 1, S - 1)))
        gather_tile_body<C, KEEPZ, KEEPG, true, W>(v, ray, t0, S, absm, lane, zprev, s_rho, s_z, s_g, s_zc, s_dq);
    else
        gather_tile_body<C, KEEPZ, KEEPG, false, W>(v, ray, t0, S, absm, lane, zprev, s_rho, s_z, s_g, s_zc, s_dq);
}

// transfer map of interface rho (first column and determinant; the second
// column is (rho, 1)).  VALID = false (interfaces outside [1, S), rho = 0):
// the identity.
struct Map {
    double m00, m10, det;
};

__device__ __forceinline__ Map make_map(double r, double a2, double sgn, bool valid)
{
    Map m;
    const double r2 = r * r;
    m.m00 = valid ? a2 * (1.0 - r2 - sgn * r2) : 1.0;
    m.m10 = -a2 * sgn * r;
    m.det = valid ? a2 * (1.0 - r2) : 1.0;
    return m;
}

// The forward takes every interface's map unselected: with rho = 0 it is
// diag(a^2, 1), which leaves v1 alone and scales D by a^2.  Past the last
// sample that changes nothing stored; the interface before sample 0 is the
// first step of every ray, and its a^2 is taken out of the starting D
// (d_start).  Dropping the selects cuts the forward's walk and chunk
// product; the adjoint keeps them (its registers stay within 3 waves).
__device__ __forceinline__ Map make_map(double r, double a2, double sgn) { return make_map(r, a2, sgn, true); }

// D at the start of a ray for the unselected maps: D = 1 after the first step
__device__ __forceinline__ double d_start(double a2) { return 1.0 / a2; }

struct Mat {
    double a, b, c, d;     // [[a, b], [c, d]]
};

__device__ __forceinline__ Mat matmul(const Mat &x, const Mat &y)
{
    Mat r;
    r.a = fma(x.a, y.a, x.b * y.c);
    r.b = fma(x.a, y.b, x.b * y.d);
    r.c = fma(x.c, y.a, x.d * y.c);
    r.d = fma(x.c, y.b, x.d * y.d);
    return r;
}

__device__ __forceinline__ Mat shfl_up_mat(const Mat &m, int d)
{
    Mat r;
    r.a = __shfl_up(m.a, d);
    r.b = __shfl_up(m.b, d);
    r.c = __shfl_up(m.c, d);
    r.d = __shfl_up(m.d, d);
    return r;
}

// chunk product Q = M_first ... M_last of a lane's C interfaces, and det;
// SEL: identity maps outside [1, S) (the adjoint), else unselected maps
template <int C, bool SEL>
__device__ __forceinline__ void chunk_product(const double *s_rho, int base, int t0, int S,
                                              double a2, double sgn, Mat &Q, double &qd)
{
    Q = Mat{1.0, 0.0, 0.0, 1.0};
    qd = 1.0;
    // unrolled: the C LDS reads issue together
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const int k = t0 + base + i;
        const double r = s_rho[pad8(base + i)];
        const Map m = make_map(r, a2, sgn, !SEL || ((k >= 1) && (k < S)));
        const double n00 = fma(Q.a, m.m00, Q.b * m.m10);
        const double n01 = fma(Q.a, r, Q.b);
        const double n10 = fma(Q.c, m.m00, Q.d * m.m10);
        const double n11 = fma(Q.c, r, Q.d);
        Q = Mat{n00, n01, n10, n11};
        qd *= m.det;
    }
}

// exclusive left-to-right product scan over the 64 lanes; also returns the
// wave total (inclusive product of lane 63)
__device__ __forceinline__ void scan_exclusive(int lane, Mat Q, double qd, Mat &X, double &xd,
                                               Mat &Tot, double &td)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const Mat o = shfl_up_mat(Q, d);
        const double od = __shfl_up(qd, d);
        if (lane >= d) {
            Q = matmul(o, Q);
            qd = od * qd;
        }
    }
    Tot = Mat{lane_read(Q.a, 63), lane_read(Q.b, 63), lane_read(Q.c, 63), lane_read(Q.d, 63)};
    td = lane_read(qd, 63);
    X = shfl_up_mat(Q, 1);
    xd = __shfl_up(qd, 1);
    if (lane == 0) {
        X = Mat{1.0, 0.0, 0.0, 1.0};
        xd = 1.0;
    }
}

// scale the carried row vector by a power of two (exact; pixels are
// homogeneous of degree 0 in (v, sqrt(D)))
__device__ __forceinline__ int renorm_exp(double c0, double c1)
{
    const double m = fmax(fabs(c0), fabs(c1));
    if (!(m > 0.0) || !isfinite(m)) return 0;
    return ilogb(m);
}

// --------------------------------------------------------------------------
// forward kernel
//
// W = 1: one wavefront per ray walks its tiles in order.  W > 1 (rays of
// many tiles): W wavefronts share a ray and take W consecutive tiles at a
// time.  A tile's gather, chunk products and lane scan need nothing from the
// tiles before it; only the state carried into its walk does, and that is
// the state at the round's start pushed through the scan totals of the
// tiles before it (one 1x2 by 2x2 product and a power-of-two renormalisation
// per tile, in the order and with the operations of W = 1, so the results
// are the same bit for bit).  The sample before the tile comes from its own
// trilinear lookup instead of the previous tile's gather.
// --------------------------------------------------------------------------
template <int C, bool SPK, int W>
__global__ __launch_bounds__(64 * W) void k_forward(VolArgs v, PhysArgs p, FanTable tab,
                                                    const float *__restrict__ poses,
                                                    float *__restrict__ out, float *__restrict__ minpiv,
                                                    int pivot_base, double *__restrict__ carry,
                                                    int32_t *__restrict__ carry_exp,
                                                    double *__restrict__ cstate,
                                                    float *__restrict__ gain_out, int xgrp, ZeroArgs zero)
{
    constexpr int T = 64 * C;
    static_assert(T % kCarryBlock == 0, "tiles hold whole carry blocks");
    static_assert(C % kStateStride == 0, "chunks hold whole state strides");
    constexpr int NB = T / kCarryBlock;     // carry blocks per tile
    constexpr int LB = kCarryBlock / C;     // lanes per carry block
    __shared__ double s_rho_w[W][T + T / 16];
    __shared__ double s_zc_w[W][NB];
    __shared__ float s_xir_w[W][SPK ? T / 4 + 8 : 1];
    __shared__ double s_tot[W > 1 ? W : 1][5];     // scan totals of a round's tiles
    __shared__ double s_piv[W > 1 ? W : 1];

    const int lane = (W == 1) ? (int)threadIdx.x : (int)(threadIdx.x & 63);
    const int wv = (W == 1) ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    double *s_rho = s_rho_w[wv];
    double *s_zc = s_zc_w[wv];
    float *s_xir = s_xir_w[wv];
    if (zero.na > 0 || zero.nb > 0) {
        // the step's clears, spread over the forward's wavefronts: the stores
        // drain while the wavefront renders its ray
        const long long stride = (long long)gridDim.x * 64 * W;
        const long long i0 = (long long)blockIdx.x * 64 * W + threadIdx.x;
        if ((reinterpret_cast<uintptr_t>(zero.a) & 15) == 0) {
            float4 *a4 = reinterpret_cast<float4 *>(zero.a);
            const long long n4 = zero.na / 4;
            for (long long i = i0; i < n4; i += stride) a4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            for (long long i = 4 * n4 + i0; i < zero.na; i += stride) zero.a[i] = 0.0f;
        } else {
            for (long long i = i0; i < zero.na; i += stride) zero.a[i] = 0.0f;
        }
        for (long long i = i0; i < zero.nb; i += stride) zero.b[i] = 0.0;
    }
    const int g = remap_block(blockIdx.x, gridDim.x, xgrp);
    if (W == 1 && g < tab.ray0) return;          // walked by several wavefronts in another launch
    const int fi = find_fan(tab, g);
    const FanRec fr = tab.f[fi];
    const int j = g - fr.ray_begin;
    const int S = fr.n_samples;
    Ray ray;
    setup_ray(v, p, fr, poses, j, ray);
    const bool absm = (p.refl == 0);
    const double sgn = absm ? 1.0 : -1.0;
    const double a2 = ray.a2;
    const float postc = posthoc_coef(p, fr.ds);
    const GainK gk = gain_consts(p, fr.n_samples);
    const long long obase = fr.out_offset + (long long)j * S;

    // state carried into the round (W > 1) or the tile (W = 1)
    double c0 = 0.0, c1 = 1.0, cD = d_start(a2), zprev = 0.0;
    double piv = 1e300;
    const bool want_piv = (minpiv != nullptr);
    const int nblk = (S + kCarryBlock - 1) / kCarryBlock;
    const long long crec = (long long)fr.carry_begin + (long long)j * nblk;
    int first_rel = 0;      // exponent of this tile's carry relative to the previous record

    for (int r0 = 0; r0 < S; r0 += W * T) {
        const int t0 = r0 + wv * T;
        const bool act = (W == 1) || (t0 < S);      // uniform over the wavefront
        if (W > 1 && act && t0 > 0) {
            const Stencil st = stencil_at<false>(v, ray, t0 - 1);
            zprev = trilinear(v.Z, v.nx, v.nx * v.ny, st, nullptr);
        }
        const double zstart = zprev;
        if (act) {
            gather_tile<C, false, false, W>(v, ray, t0, S, absm, lane, zprev, s_rho, nullptr, nullptr,
                                  carry ? s_zc : nullptr);
            if (SPK) speckle_radial<T>(p, t0, j, fr.speckle_id, lane, s_xir);
        }
        __syncthreads();

        const int base = lane * C;
        Mat Q, X, Tot;
        double qd, xd, td;
        double tc0 = c0, tc1 = c1, tcD = cD;        // the state carried into this tile
        int trel = first_rel;
        if (act) {
            chunk_product<C, false>(s_rho, base, t0, S, a2, sgn, Q, qd);
            scan_exclusive(lane, Q, qd, X, xd, Tot, td);
        }
        if (W > 1) {
            if (act && lane == 0) {
                s_tot[wv][0] = Tot.a;
                s_tot[wv][1] = Tot.b;
                s_tot[wv][2] = Tot.c;
                s_tot[wv][3] = Tot.d;
                s_tot[wv][4] = td;
            }
            __syncthreads();
            // the round's carry through the tiles before this one; then on
            // through the rest of the round for the next round's carry
            for (int u = 0; u < W; ++u) {
                if (u == wv) {
                    tc0 = c0;
                    tc1 = c1;
                    tcD = cD;
                    trel = first_rel;
                }
                if (r0 + u * T >= S) break;
                const double n0 = fma(c0, s_tot[u][0], c1 * s_tot[u][2]);
                const double n1 = fma(c0, s_tot[u][1], c1 * s_tot[u][3]);
                const double nD = cD * s_tot[u][4];
                const int ex = renorm_exp(n0, n1);
                c0 = ldexp(n0, -ex);
                c1 = ldexp(n1, -ex);
                cD = ldexp(nD, -2 * ex);
                first_rel = ex;
            }
        }
        if (act) {
            double v0 = fma(tc0, X.a, tc1 * X.c);
            double v1 = fma(tc0, X.b, tc1 * X.d);
            double D = tcD * xd;
            if (carry) {
                // state at the start of carry block m = lane / LB (lanes on a
                // block boundary), in the tile's frame: inside a tile the
                // records share one scale, so only a tile's first record carries
                // an exponent (relative to the previous record)
                const int m = lane / LB;
                const int kb = t0 + m * kCarryBlock;
                if ((lane % LB) == 0 && kb < S) {
                    const long long r = crec + kb / kCarryBlock;
                    double *q = carry + 4 * r;
                    q[0] = v0;
                    q[1] = v1;
                    // the ray's first record in the adjoint's convention (identity
                    // map before sample 0): D = 1
                    q[2] = (kb == 0) ? 1.0 : D;
                    q[3] = (m == 0) ? zstart : s_zc[m - 1];
                    carry_exp[r] = (m == 0) ? trel : 0;
                }
            }
            // chunk states for the adjoint: the lane's C samples lie in one
            // carry block (the ray's first state is taken in the adjoint's
            // convention by the adjoint itself)
            double *qs = nullptr;
            if (cstate && (t0 + base) / kCarryBlock < nblk)
                qs = cstate + (crec + (t0 + base) / kCarryBlock) * kStateDoubles + ((t0 + base) % kCarryBlock) / kStateStride;
            float pix[C];
#pragma unroll
            for (int i = 0; i < C; ++i) {
                // branch-free: outside [1, S) rho = 0, so the pixel is 0 and v1
                // unchanged (make_map)
                const int k = t0 + base + i;
                // the chunk states and the gains below are read once, by the
                // adjoint after the blur: non-temporal stores keep them from
                // displacing the volume and the images in the caches
                if ((i % kStateStride) == 0 && qs) {
                    __builtin_nontemporal_store(v0, qs + i / kStateStride);
                    __builtin_nontemporal_store(v1, qs + kStatesPerBlock + i / kStateStride);
                    __builtin_nontemporal_store(D, qs + 2 * kStatesPerBlock + i / kStateStride);
                }
                const double r = s_rho[pad8(base + i)];
                const Map m = make_map(r, a2, sgn);
                const double v1n = fma(v0, r, v1);
                // the pixel leaves in FP32: the hardware FP64 reciprocal, without
                // the Newton step, is accurate well beyond that
                pix[i] = (float)(r * D * __builtin_amdgcn_rcp(v1 * v1n));
                if (want_piv) piv = (k >= 1 && k < S) ? fmin(piv, fabs(v1n * rcp64(v1))) : piv;
                const double v0n = fma(v0, m.m00, v1 * m.m10);
                v0 = v0n;
                v1 = v1n;
                D *= m.det;
            }
            if (W == 1) {
                // carry to the next tile, renormalised by a power of two
                const double n0 = fma(c0, Tot.a, c1 * Tot.c);
                const double n1 = fma(c0, Tot.b, c1 * Tot.d);
                const double nD = cD * td;
                const int ex = renorm_exp(n0, n1);
                c0 = ldexp(n0, -ex);
                c1 = ldexp(n1, -ex);
                cD = ldexp(nD, -2 * ex);
                first_rel = ex;
            }
            // per-pixel gains and the stores, in the lane's chunk order (the
            // lane's C samples start at a multiple of 4: its granular variates
            // are C/4 whole Philox blocks)
            float gn[C];
#pragma unroll
            for (int i = 0; i < C; ++i) gn[i] = 1.0f;
            if (SPK) {
#pragma unroll
                for (int q = 0; q < C / 4; ++q) {
                    float x[4];
                    granular4(p, ((t0 + base) >> 2) + q, j, fr.speckle_id, x);
#pragma unroll
                    for (int u = 0; u < 4; ++u) gn[4 * q + u] = x[u];
                }
                // the lane's samples are consecutive: the radial cell index of the
                // first is exact (cell_of), the others step it
                int c, r;
                cell_of(p, gk, t0 + base, c, r);
                c -= t0 / p.cell;          // index into s_xir
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int k = t0 + base + i;
                    float g = speckle_mult(p, (float)k * gk.inv_sm1, (float)r * gk.inv_cell, s_xir[c], s_xir[c + 1], gn[i]);
                    if (p.atten == 1) g *= exp2f((float)((double)k * (double)postc));
                    gn[i] = g;
                    const bool wrap = (r + 1 == p.cell);
                    c += wrap ? 1 : 0;
                    r = wrap ? 0 : r + 1;
                }
            } else if (p.atten == 1) {
#pragma unroll
                for (int i = 0; i < C; ++i)
                    gn[i] = pixel_gain<false, true>(p, gk, t0 + base + i, t0, postc, 1.0f, s_xir);
            }
            const bool has_gain = SPK || p.atten == 1;
            const long long o = obase + t0 + base;
            const bool vec = ((reinterpret_cast<uintptr_t>(out + o) & 15) == 0) &&
                             (!gain_out || (reinterpret_cast<uintptr_t>(gain_out + o) & 15) == 0);
            if (vec && t0 + base + C <= S) {
#pragma unroll
                for (int q = 0; q < C / 4; ++q) {
                    const int i = 4 * q;
                    *reinterpret_cast<float4 *>(out + o + i) =
                        make_float4(pix[i] * gn[i], pix[i + 1] * gn[i + 1], pix[i + 2] * gn[i + 2], pix[i + 3] * gn[i + 3]);
                    if (has_gain && gain_out) {
                        float *gq = gain_out + o + i;
                        __builtin_nontemporal_store(gn[i], gq);
                        __builtin_nontemporal_store(gn[i + 1], gq + 1);
                        __builtin_nontemporal_store(gn[i + 2], gq + 2);
                        __builtin_nontemporal_store(gn[i + 3], gq + 3);
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    if (t0 + base + i < S) {
                        out[o + i] = pix[i] * gn[i];
                        if (has_gain && gain_out) gain_out[o + i] = gn[i];
                    }
                }
            }
        }
        __syncthreads();
    }
    if (want_piv) {
        piv = wave_min(piv);
        if (W == 1) {
            if (lane == 0) minpiv[pivot_base + fr.pivot_begin + j] = (float)piv;
        } else {
            if (lane == 0) s_piv[wv] = piv;
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int u = 1; u < W; ++u) piv = fmin(piv, s_piv[u]);
                minpiv[pivot_base + fr.pivot_begin + j] = (float)piv;
            }
        }
    }
}

// --------------------------------------------------------------------------
// adjoint kernel
// --------------------------------------------------------------------------
// Reverse recurrence per interface step (state before the step: v0, v1, D;
// adjoint after the step: l0, l1, lD = dL/d(v0', v1', D')):
//   v0' = v0 A + v1 B,  v1' = v0 R + v1,  D' = D E,  e = R D / (v1 v1')
// gives l_before = l_after J + f with J = diag(M^T, E) and forcing f from
// de/d(state); the rho adjoint collects dA, dB, dR, dE and de/dR = D/v1'^2.
struct Adj {
    double l0, l1, lD;
};

// W = 1: one wavefront per ray walks its tiles from the deepest up.  W > 1
// (rays of many tiles, with the forward's carry records and chunk states):
// W wavefronts share a ray and take W consecutive tiles at a time.  Walk 1
// and the lanes' suffix composition need nothing from the deeper tiles; the
// adjoint entering each tile is the round's incoming adjoint pushed through
// the deeper tiles' affine maps (lane 1's suffix map, then lane 0's chunk
// map, then the frame's power of two: the operations of W = 1, in its
// order, so the results are the same bit for bit).  The sample after a
// tile and its interface's dL/dZ factor come from the neighbouring
// wavefront's LDS; the pose sums and the loss are added over the W
// wavefronts in a fixed order.
template <int C, bool SPK, bool FUSED, int W>
__global__ __launch_bounds__(64 * W) void k_backward(VolArgs v, PhysArgs p, FanTable tab,
                                                 const float *__restrict__ poses,
                                                 RayRec *__restrict__ rays_out,
                                                 const float *__restrict__ gsrc,
                                                 const float *__restrict__ target,
                                                 float *__restrict__ zbar,
                                                 double *__restrict__ pose_part,
                                                 double *__restrict__ loss_acc,
                                                 const double *__restrict__ carry,
                                                 const int32_t *__restrict__ carry_exp,
                                                 const double *__restrict__ cstate,
                                                 const float *__restrict__ gain_in, int xgrp)
{
    constexpr int T = 64 * C;
    constexpr int kMaxTiles = (DUS_MAX_SAMPLES + T - 1) / T;
    static_assert(W == 1 || !SPK, "several wavefronts per ray take the forward's gains");
    static_assert(T % kCarryBlock == 0, "tiles hold whole carry blocks");
    constexpr int NB = T / kCarryBlock;
    // walks unrolled where the registers allow three wavefronts per SIMD
    constexpr int kWalkUnroll = (C <= 4 && !SPK && !FUSED) ? C : 1;
    __shared__ float s_g_w[W][3 * T];     // dZ/dp of every sample of the tile, in the ray's basis
    __shared__ double s_rho_w[W][T + T / 16];
    __shared__ double s_z_w[W][T + T / 16];
    __shared__ double s_dq_w[W][T + T / 16];   // d rho / dZ factor of every interface of the tile
    __shared__ float s_eb_w[W][T + T / 32];
    __shared__ float s_gain_w[W][FUSED ? T + T / 32 : 1];
    __shared__ float s_xig[SPK ? T : 1];
    __shared__ float s_xir[SPK ? T / 4 + 8 : 1];
    __shared__ double s_carry[kMaxTiles][4];
    __shared__ int s_cexp[kMaxTiles];
    __shared__ double s_x[W > 1 ? W : 1][16];   // a round's tiles: lane 1's suffix map, lane 0's chunk map
    __shared__ double s_red[W > 1 ? W : 1][7];  // per-wavefront pose sums and loss

    const int lane = (W == 1) ? (int)threadIdx.x : (int)(threadIdx.x & 63);
    const int wv = (W == 1) ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    float *s_g = s_g_w[wv];
    double *s_rho = s_rho_w[wv];
    double *s_z = s_z_w[wv];
    double *s_dq = s_dq_w[wv];
    float *s_eb = s_eb_w[wv];
    float *s_gain = s_gain_w[wv];
    const int g = remap_block(blockIdx.x, gridDim.x, xgrp);
    if (W == 1 && g < tab.ray0) return;          // walked by several wavefronts in another launch
    const int fi = find_fan(tab, g);
    const FanRec fr = tab.f[fi];
    const int j = g - fr.ray_begin;
    const int S = fr.n_samples;
    if (S <= 0) return;
    Ray ray;
    setup_ray(v, p, fr, poses, j, ray);
    if (rays_out && threadIdx.x == 0) {
        // the ray's geometry for the scatter
        RayRec r;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r.u0[a] = ray.u0[a];
            r.du[a] = ray.du[a];
        }
        rays_out[g] = r;
    }
    const bool absm = (p.refl == 0);
    const double sgn = absm ? 1.0 : -1.0;
    const double a2 = ray.a2;
    const float postc = posthoc_coef(p, fr.ds);
    const GainK gk = gain_consts(p, fr.n_samples);
    const long long obase = fr.out_offset + (long long)j * S;
    const int ntiles = (S + T - 1) / T;
    const double inv_npix = 1.0 / ((double)fr.n_rays * (double)S);

    const int nblk = (S + kCarryBlock - 1) / kCarryBlock;
    const long long rb = (long long)fr.carry_begin + (long long)j * nblk;
    __shared__ int s_bexp[(DUS_MAX_SAMPLES + kCarryBlock - 1) / kCarryBlock];
    if (carry) {
        // tile starts from the forward kernel's carry records; the exponent
        // of tile t relative to tile t - 1 sums those of its carry blocks
        for (int b = threadIdx.x; b < nblk; b += 64 * W) {
            s_bexp[b] = carry_exp[rb + b];
            if (b % NB == 0) {
                const double *q = carry + 4 * (rb + b);
                s_carry[b / NB][0] = q[0];
                s_carry[b / NB][1] = q[1];
                s_carry[b / NB][2] = q[2];
                s_carry[b / NB][3] = q[3];
            }
        }
        __syncthreads();
        // A tile's frame is its first record renormalised by a power of two
        // (the forward's records share one scale inside a forward tile).
        // Thread t takes tile t (ntiles <= 64): s_cexp[t] becomes the exponent
        // of tile t's frame relative to tile t - 1's, and s_bexp[b] that of
        // block b's record relative to its tile's frame.
        const int t = threadIdx.x;
        int et = 0, cex = 0, rel[NB];
        if (t < ntiles) {
            et = renorm_exp(s_carry[t][0], s_carry[t][1]);
            if (t > 0) {
                cex = et - renorm_exp(s_carry[t - 1][0], s_carry[t - 1][1]);
#pragma unroll
                for (int q = 0; q < NB; ++q) cex += s_bexp[(t - 1) * NB + 1 + q];
            }
            rel[0] = -et;
#pragma unroll
            for (int u = 1; u < NB; ++u) rel[u] = rel[u - 1] + s_bexp[t * NB + u];
        }
        __syncthreads();
        if (t < ntiles) {
            s_carry[t][0] = ldexp(s_carry[t][0], -et);
            s_carry[t][1] = ldexp(s_carry[t][1], -et);
            s_carry[t][2] = ldexp(s_carry[t][2], -2 * et);
            s_cexp[t] = cex;
#pragma unroll
            for (int u = 0; u < NB; ++u) s_bexp[t * NB + u] = rel[u];
        }
    } else if (W == 1) {
        // forward sweep: state at every tile start (several wavefronts per
        // ray take the forward's carry records instead)
        double c0 = 0.0, c1 = 1.0, cD = 1.0, zprev = 0.0;
        for (int t = 0; t < ntiles; ++t) {
            if (lane == 0) {
                s_carry[t][0] = c0;
                s_carry[t][1] = c1;
                s_carry[t][2] = cD;
                s_carry[t][3] = zprev;
            }
            if (t + 1 == ntiles) break;
            const int t0 = t * T;
            gather_tile<C, false>(v, ray, t0, S, absm, lane, zprev, s_rho, nullptr);
            __syncthreads();
            Mat Q, X, Tot;
            double qd, xd, td;
            chunk_product<C, true>(s_rho, lane * C, t0, S, a2, sgn, Q, qd);
            scan_exclusive(lane, Q, qd, X, xd, Tot, td);
            const double n0 = fma(c0, Tot.a, c1 * Tot.c);
            const double n1 = fma(c0, Tot.b, c1 * Tot.d);
            const double nD = cD * td;
            const int ex = renorm_exp(n0, n1);
            c0 = ldexp(n0, -ex);
            c1 = ldexp(n1, -ex);
            cD = ldexp(nD, -2 * ex);
            if (lane == 0) s_cexp[t + 1] = ex;
            __syncthreads();
        }
    }
    __syncthreads();

    // reverse sweep (W > 1: rounds of W tiles, wavefront w taking tile rt - w)
    Adj lam{0.0, 0.0, 0.0};        // adjoint of the state at the end of the (round's deepest) tile
    double rbar_next = 0.0;        // dL/dZ factor of the interface just after that tile
    double z_next = 0.0;           // first sample of the tile after it
    double loss = 0.0;
    double gsum[3] = {0.0, 0.0, 0.0}, gssum[3] = {0.0, 0.0, 0.0};
    for (int rt = ntiles - 1; rt >= 0; rt -= W) {
        // uniform over the wavefront; an idle wavefront of the last round
        // repeats tile 0 and stores nothing
        const bool act = (W == 1) || (rt - wv >= 0);
        const int t = act ? rt - wv : 0;
        const int t0 = t * T;
        const double zstart = s_carry[t][3];
        double zprev = zstart;
        const int base = lane * C;
        // wave priority 1 while this wavefront issues its chunk-state loads and
        // its gather (its loads go out ahead of co-resident wavefronts' FP64
        // arithmetic) and during the suffix scan over the lanes (a serial chain
        // of cross-lane exchanges), 0 elsewhere: the adjoint 2% faster at
        // 64 x 256 x 1024
        __builtin_amdgcn_s_setprio(1);
        // the state at the lane's chunk start, from the forward's chunk
        // states when it recorded them (loads issued before the gather)
        double v0s = 0.0, v1s = 1.0, Ds = 1.0;
        if (cstate) {
            const int k = t0 + base;
            if (k / kCarryBlock < nblk) {
                const double *q = cstate + (rb + k / kCarryBlock) * kStateDoubles + (k % kCarryBlock) / kStateStride;
                v0s = q[0];
                v1s = q[kStatesPerBlock];
                // the ray's first state in the adjoint's convention: D = 1
                Ds = (k == 0) ? 1.0 : q[2 * kStatesPerBlock];
            }
        }
        if (pose_part)
            gather_tile<C, true, true, W>(v, ray, t0, S, absm, lane, zprev, s_rho, s_z, s_g, nullptr, s_dq);
        else
            gather_tile<C, true, false, W>(v, ray, t0, S, absm, lane, zprev, s_rho, s_z, nullptr, nullptr, s_dq);
        if (SPK) speckle_fill<T>(p, t0, j, fr.speckle_id, lane, s_xig, s_xir);
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        // dL/de (or the target for the fused loss) staged through LDS: the C
        // global loads are issued together, then the per-pixel gains
        // (speckle, post-hoc attenuation) are applied in place
        // the loads are clamped into the ray and issued together (no
        // per-load branches, one wait); samples past the ray read as zero
        const float *src = FUSED ? target : gsrc;
        if (gain_in) {
            // gains recorded by the forward kernel
            float x[C], gn[C];
#pragma unroll
            for (int m = 0; m < C; ++m) {
                const int k = min(t0 + m * 64 + lane, S - 1);
                x[m] = src[obase + k];
                gn[m] = gain_in[obase + k];
            }
#pragma unroll
            for (int m = 0; m < C; ++m) {
                const int i = m * 64 + lane;
                const bool in = (t0 + i < S);
                if (FUSED) {
                    s_eb[pad4(i)] = in ? x[m] : 0.0f;
                    s_gain[pad4(i)] = in ? gn[m] : 1.0f;
                } else {
                    s_eb[pad4(i)] = in ? x[m] * gn[m] : 0.0f;
                }
            }
        } else {
            float x[C];
#pragma unroll
            for (int m = 0; m < C; ++m) x[m] = src[obase + min(t0 + m * 64 + lane, S - 1)];
#pragma unroll
            for (int m = 0; m < C; ++m) {
                const int i = m * 64 + lane;
                s_eb[pad4(i)] = (t0 + i < S) ? x[m] : 0.0f;
            }
            const bool has_gain = SPK || p.atten == 1;
#pragma unroll 1
            for (int m = 0; m < C; ++m) {
                const int i = m * 64 + lane;
                const int k = t0 + i;
                const float gain = (has_gain && k < S) ? pixel_gain_rt<SPK>(p, gk, k, t0, postc, SPK ? s_xig[i] : 1.0f, s_xir) : 1.0f;
                if (FUSED) s_gain[pad4(i)] = gain;
                else s_eb[pad4(i)] *= gain;
            }
        }
        __syncthreads();

        if (cstate) {
            // from the frame of the state's block record to the tile's frame
            // (the exponent is read here, after the barrier, so that the
            // scaling, and the wait for the loads above, stay behind the gather)
            const int es = s_bexp[min((t0 + base) / kCarryBlock, nblk - 1)];
            v0s = ldexp(v0s, es);
            v1s = ldexp(v1s, es);
            Ds = ldexp(Ds, 2 * es);
        } else {
            // otherwise from the tile's carry and a prefix scan of the
            // lanes' chunk products
            Mat Q, X, Tot;
            double qd, xd, td;
            chunk_product<C, true>(s_rho, base, t0, S, a2, sgn, Q, qd);
            scan_exclusive(lane, Q, qd, X, xd, Tot, td);
            const double c0 = s_carry[t][0], c1 = s_carry[t][1], cD = s_carry[t][2];
            v0s = fma(c0, X.a, c1 * X.c);
            v1s = fma(c0, X.b, c1 * X.d);
            Ds = cD * xd;
        }
        // Walk 1 (forward over the lane's C interfaces): the chunk's affine
        // adjoint map lambda_start = lambda_end J_chunk + f_chunk, with
        // J_chunk = diag(Q^T, det) and f_chunk = sum_i f_i (Q_i^loc)^T, where
        // Q_i^loc = M_first .. M_{i-1} and f_i is step i's forcing (adj_forcing).
        // The walk's final Q^loc is the chunk product Q itself.
        Adj f{0.0, 0.0, 0.0};
        Mat Q{1.0, 0.0, 0.0, 1.0};
        double qd = 1.0;
        const double w1s = rcp64(v1s);     // 1 / v1 at the chunk start
        {
            double v0 = v0s, v1 = v1s, D = Ds, w1 = w1s;
            Mat &QL = Q;
            double &qdl = qd;
            // branch-free: an interface outside [1, S) has rho = 0 (gather)
            // and the identity map, so its step leaves the state unchanged and
            // forces nothing (pixel 0 is zero; the loss still counts it)
#pragma unroll kWalkUnroll
            for (int i = 0; i < C; ++i) {
                const int k = t0 + base + i;
                const bool valid = (k >= 1) && (k < S);
                const double r = s_rho[pad8(base + i)];
                const Map m = make_map(r, a2, sgn, valid);
                const double v1n = fma(v0, r, v1);
                const double w1p = rcp64(v1n);
                const double e = r * D * w1 * w1p;
                double eb;
                if (FUSED) {
                    const double gn = s_gain[pad4(base + i)];
                    const double diff = e * gn - (double)s_eb[pad4(base + i)];
                    loss += act ? diff * diff * inv_npix : 0.0;
                    eb = 2.0 * diff * inv_npix * gn;
                    s_eb[pad4(base + i)] = (float)eb;
                } else {
                    eb = s_eb[pad4(base + i)];
                }
                const double f0 = -eb * e * r * w1p;
                const double f1 = -eb * e * (w1 + w1p);
                const double fD = eb * r * w1 * w1p;
                f.l0 = fma(f0, QL.a, fma(f1, QL.b, f.l0));
                f.l1 = fma(f0, QL.c, fma(f1, QL.d, f.l1));
                f.lD = fma(fD, qdl, f.lD);
                const double n00 = fma(QL.a, m.m00, QL.b * m.m10), n01 = fma(QL.a, r, QL.b);
                const double n10 = fma(QL.c, m.m00, QL.d * m.m10), n11 = fma(QL.c, r, QL.d);
                QL = Mat{n00, n01, n10, n11};
                qdl *= m.det;
                const double v0n = fma(v0, m.m00, v1 * m.m10);
                v0 = v0n;
                v1 = v1n;
                w1 = w1p;
                D *= m.det;
            }
        }
        __builtin_amdgcn_s_setprio(1);
        // suffix composition over lanes: Psi_l = Phi_l o Phi_{l+1} o ... o Phi_63
        Mat PQ = Q;
        double pd = qd;
        Adj pf = f;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            Mat oq;
            oq.a = __shfl_down(PQ.a, d);
            oq.b = __shfl_down(PQ.b, d);
            oq.c = __shfl_down(PQ.c, d);
            oq.d = __shfl_down(PQ.d, d);
            const double od = __shfl_down(pd, d);
            const double of0 = __shfl_down(pf.l0, d), of1 = __shfl_down(pf.l1, d);
            const double ofD = __shfl_down(pf.lD, d);
            if (lane + d < 64) {
                // f_new = f_{l+d} Q_l^T + f_l ;  Q_new = Q_l Q_{l+d} ; d_new = d_{l+d} d_l
                const double n0 = fma(of0, PQ.a, fma(of1, PQ.b, pf.l0));
                const double n1 = fma(of0, PQ.c, fma(of1, PQ.d, pf.l1));
                const double nD = fma(ofD, pd, pf.lD);
                PQ = matmul(PQ, oq);
                pd = od * pd;
                pf = Adj{n0, n1, nD};
            }
        }
        // adjoint at this tile's end
        Adj tl = lam;
        if (W > 1) {
            if (act && lane == 1) {
                s_x[wv][0] = PQ.a;
                s_x[wv][1] = PQ.b;
                s_x[wv][2] = PQ.c;
                s_x[wv][3] = PQ.d;
                s_x[wv][4] = pd;
                s_x[wv][5] = pf.l0;
                s_x[wv][6] = pf.l1;
                s_x[wv][7] = pf.lD;
            }
            if (act && lane == 0) {
                s_x[wv][8] = Q.a;
                s_x[wv][9] = Q.b;
                s_x[wv][10] = Q.c;
                s_x[wv][11] = Q.d;
                s_x[wv][12] = qd;
                s_x[wv][13] = f.l0;
                s_x[wv][14] = f.l1;
                s_x[wv][15] = f.lD;
            }
            __syncthreads();
            // the round's incoming adjoint through the deeper tiles of the
            // round (lane 0's chunk-start adjoint of each, in the previous
            // tile's frame), then on through the round for the next one
            Adj x = lam;
            for (int u = 0; u < W; ++u) {
                if (u == wv) tl = x;
                const int tu = rt - u;
                if (tu < 0) break;
                const double *q = s_x[u];
                Adj e1, c1;
                e1.l0 = fma(x.l0, q[0], fma(x.l1, q[1], q[5]));
                e1.l1 = fma(x.l0, q[2], fma(x.l1, q[3], q[6]));
                e1.lD = fma(x.lD, q[4], q[7]);
                c1.l0 = fma(e1.l0, q[8], fma(e1.l1, q[9], q[13]));
                c1.l1 = fma(e1.l0, q[10], fma(e1.l1, q[11], q[14]));
                c1.lD = fma(e1.lD, q[12], q[15]);
                const int ex = (tu > 0) ? s_cexp[tu] : 0;
                x.l0 = ldexp(c1.l0, -ex);
                x.l1 = ldexp(c1.l1, -ex);
                x.lD = ldexp(c1.lD, -2 * ex);
            }
            lam = x;
        }
        // adjoint at this lane's chunk end: Psi_{l+1}(lambda_tile_end)
        Adj le;
        {
            Mat nq;
            nq.a = __shfl_down(PQ.a, 1);
            nq.b = __shfl_down(PQ.b, 1);
            nq.c = __shfl_down(PQ.c, 1);
            nq.d = __shfl_down(PQ.d, 1);
            const double nd = __shfl_down(pd, 1);
            const double nf0 = __shfl_down(pf.l0, 1), nf1 = __shfl_down(pf.l1, 1);
            const double nfD = __shfl_down(pf.lD, 1);
            if (lane == 63) {
                le = tl;
            } else {
                le.l0 = fma(tl.l0, nq.a, fma(tl.l1, nq.b, nf0));
                le.l1 = fma(tl.l0, nq.c, fma(tl.l1, nq.d, nf1));
                le.lD = fma(tl.lD, nd, nfD);
            }
        }
        __builtin_amdgcn_s_setprio(0);
        // adjoint at the lane's chunk start: lambda_end J_chunk + f_chunk
        Adj lc;
        lc.l0 = fma(le.l0, Q.a, fma(le.l1, Q.b, f.l0));
        lc.l1 = fma(le.l0, Q.c, fma(le.l1, Q.d, f.l1));
        lc.lD = fma(le.lD, qd, f.lD);
        const Adj lstart = lc;
        // Walk 2 (forward again): the adjoint after step i follows from the
        // one before it by the exact inverse of step i,
        //   lambda_{i+1} = (lambda_i - f_i) J_i^{-1},  det M_i = a^2 (1 - rho^2) > 0,
        // and gives dL/drho_i (adj_rbar).
        {
            double v0 = v0s, v1 = v1s, D = Ds, w1 = w1s;
#pragma unroll kWalkUnroll
            for (int i = 0; i < C; ++i) {
                const int k = t0 + base + i;
                const bool valid = (k >= 1) && (k < S);
                double qz = 0.0;
                {   // branch-free, as walk 1 (dq = 0 outside [1, S))
                    const double r = s_rho[pad8(base + i)];
                    const Map m = make_map(r, a2, sgn, valid);
                    const double v1n = fma(v0, r, v1);
                    const double w1p = rcp64(v1n);
                    const double e = r * D * w1 * w1p;
                    const double eb = s_eb[pad4(base + i)];
                    const double x0 = lc.l0 + eb * e * r * w1p;
                    const double x1 = lc.l1 + eb * e * (w1 + w1p);
                    const double xD = lc.lD - eb * r * w1 * w1p;
                    const double ie = rcp64(m.det);
                    // M = [[A, r], [B, 1]]:  x (M^T)^{-1} = (x0 - r x1, A x1 - B x0) / det
                    const Adj la{(x0 - r * x1) * ie, fma(m.m00, x1, -m.m10 * x0) * ie, xD * ie};
                    const double dA = -2.0 * a2 * r * (1.0 + sgn);
                    const double dB = -a2 * sgn;
                    const double dE = -2.0 * a2 * r;
                    const double rb = la.l0 * fma(v0, dA, v1 * dB) + la.l1 * v0 + eb * D * w1p * w1p + la.lD * D * dE;
                    // Eq. 1 on this interface (samples zl = Z_{k-1}, zr = Z_k):
                    // dL/dzr = rb dq zl, dL/dzl = -rb dq zr (dq from the gather)
                    qz = rb * s_dq[pad8(base + i)];
                    lc = la;
                    const double v0n = fma(v0, m.m00, v1 * m.m10);
                    v0 = v0n;
                    v1 = v1n;
                    w1 = w1p;
                    D *= m.det;
                }
                s_rho[pad8(base + i)] = qz;       // s_rho now holds the interfaces' dL/dZ factors
            }
        }
        le = lstart;
        // adjoint of this tile's start state, expressed for the previous tile's
        // (un-renormalised) end state
        if (W == 1) {
            Adj ls{lane_read(le.l0, 0), lane_read(le.l1, 0), lane_read(le.lD, 0)};   // le = chunk-start adjoint
            const int ex = (t > 0) ? s_cexp[t] : 0;
            lam.l0 = ldexp(ls.l0, -ex);
            lam.l1 = ldexp(ls.l1, -ex);
            lam.lD = ldexp(ls.lD, -2 * ex);
        }
        __syncthreads();

        // dL/dZ_k per sample (rho depends on the samples on both sides):
        // sample k is the right end of interface k-1 and the left end of
        // interface k.  Branch-free: the interface factors vanish outside
        // [1, S), so dL/dZ is zero for k >= S and only the store is guarded.
        // the sample after this tile and its interface's factor: the previous
        // tile's (W = 1), the neighbouring wavefront's, or for the round's
        // deepest tile those kept from the last round
        double zn_t = z_next, rn_t = rbar_next;
        if (W > 1 && wv > 0) {
            zn_t = s_z_w[wv - 1][pad8(0)];
            rn_t = s_rho_w[wv - 1][pad8(0)];
        }
#pragma unroll 1
        for (int jj = 0; jj < C; ++jj) {
            const int i = jj * 64 + lane;
            const int k = t0 + i;
            const double zl = (i > 0) ? s_z[pad8(i - 1)] : zstart;
            const double zr = (i + 1 < T) ? s_z[pad8(i + 1)] : zn_t;
            const double ql = s_rho[pad8(i)];
            const double qr = (k + 1 < S) ? ((i + 1 < T) ? s_rho[pad8(i + 1)] : rn_t) : 0.0;
            const double zb = fma(-qr, zr, ql * zl);
            // zbar is NULL when no volume gradient is wanted (nothing reads it)
            if (zbar && k < S && act) zbar[obase + k] = (float)zb;
            if (pose_part && act) {
                // dL/dp = zb dZ/dp; dL/dR accumulates (s_k dir) outer dL/dp
                const double sk = fma((double)k, ray.ds, ray.r0);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double gp = zb * (double)s_g[a * T + i];
                    gsum[a] += gp;
                    gssum[a] = fma(sk, gp, gssum[a]);
                }
            }
        }
        if (W == 1) {
            rbar_next = lane_read(s_rho[pad8(lane)], 0);
            z_next = lane_read(s_z[pad8(lane)], 0);
        } else {
            // for the next round's deepest tile: this round's shallowest
            rbar_next = s_rho_w[W - 1][pad8(0)];
            z_next = s_z_w[W - 1][pad8(0)];
        }
        __syncthreads();
    }
    double r[6];
    if (pose_part) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r[a] = wave_sum(gsum[a]);
            r[3 + a] = wave_sum(gssum[a]);
        }
    }
    double ls = 0.0;
    if (FUSED && loss_acc) ls = wave_sum(loss);
    if (W > 1) {
        // the wavefronts' shares added in a fixed order
        if (lane == 0) {
#pragma unroll
            for (int a = 0; a < 6; ++a) s_red[wv][a] = pose_part ? r[a] : 0.0;
            s_red[wv][6] = ls;
        }
        __syncthreads();
        if (wv == 0) {
            for (int u = 1; u < W; ++u) {
#pragma unroll
                for (int a = 0; a < 6; ++a) r[a] += s_red[u][a];
                ls += s_red[u][6];
            }
        }
    }
    if (pose_part) {
        if (threadIdx.x == 0) {
            // this ray's share of dL/dt = sum g and dL/dR = sum g (s dir)^T,
            // dir = (sx, 0, cz), with g back from the ray's basis to the world
            // frame; k_pose_reduce sums the rays of each pose (in a fixed
            // order: no contended atomics on the pose's entries)
            double *pr = pose_part + (size_t)kRayPart * g;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double gt = fma(r[0], ray.bd[a], fma(r[1], ray.bt[a], r[2] * ray.bn[a]));
                const double gs = fma(r[3], ray.bd[a], fma(r[4], ray.bt[a], r[5] * ray.bn[a]));
                pr[a] = gt;
                pr[3 + 2 * a] = gs * ray.dirx;
                pr[4 + 2 * a] = gs * ray.dirz;
            }
        }
    }
    if (FUSED && loss_acc) {
        // one partial per ray, summed by k_sum_f64 (no contended atomics)
        if (threadIdx.x == 0) loss_acc[g] = ls;
    }
}

// --------------------------------------------------------------------------
// scatter of dL/dZ_k: trilinear weights into the volume gradient.  One
// wavefront takes RB neighbouring rays of one fan (64/RB lanes per ray) and
// one segment of `seg` depths, and walks them together in groups of
// (64/RB) spl depths; every lane owns spl (4, 2 or 1) consecutive depths of
// its ray.
// A straight ray meets each cell once, so a
// lane's consecutive samples in one cell form a run that it sums in
// registers before touching memory.  The stencils of a group fill a small
// box of the volume (neighbouring rays of a fan overlap); the runs go into an
// LDS copy of that box with LDS atomics, and the box is then flushed with one
// global atomic per touched voxel, consecutive lanes on consecutive x.  A
// group whose box does not fit falls back to per-sample global atomics.
//
// The box holds FP64: FP64 LDS atomics (ds_add_f64) run at the rate of
// plain LDS stores on gfx950, FP32 LDS atomics several times slower.  The
// FP64 sum of a voxel's FP32 contributions is rounded to FP32 once, when the
// box is flushed.
// --------------------------------------------------------------------------
constexpr int kScatterSpl = 4;     // consecutive depths per lane, at most

// floor(a / b) for a >= 0, b >= 1, a + b < 2^21, from rb = rcp(b) (within
// 1 ulp): (a + 0.5) / b lies at least 0.5 / b from an integer, more than the
// product's error (a / b + 1) 2^-22.  A few instructions, where an integer
// division takes about thirty.
__device__ __forceinline__ int small_quot(int a, float rb)
{
    return (int)(((float)a + 0.5f) * rb);
}

template <int RB>
struct ScatterBox {
    static constexpr int cap = RB == 2 ? 4096 : (RB == 4 ? 2048 : 1024);   // FP64 entries
};

template <int RB>
__global__ __launch_bounds__(64) void k_scatter(VolArgs v, FanTable tab, const RayRec *__restrict__ rays,
                                                const float *__restrict__ zbar, float *__restrict__ gZ,
                                                int seg_shift, int xgrp, unsigned long long *__restrict__ fix,
                                                const double *__restrict__ fscale)
{
    constexpr int LPR = 64 / RB;                 // lanes per ray
    constexpr int CAP = ScatterBox<RB>::cap;
    // s_box is all zeros between groups: cleared once here, and every flush
    // clears the entries it reads
    __shared__ double s_box[CAP];
    const int lane = threadIdx.x;
    const int slot = lane / LPR, ll = lane % LPR;
    // depth chunk of this lane, rotated by the ray slot: in one instruction
    // the rays of the wavefront sit at different depths (>= 1 mm apart), so
    // lanes of one LDS atomic rarely meet in one cell
    constexpr int SH = LPR / RB;
    const int ch = (ll + slot * SH) % LPR;
    // block -> (fan, depth segment, first ray).  Each fan owns ceil(n_rays /
    // RB) ray blocks.  One-dimensional grid: the fans one after the other,
    // each with its ceil(n_samples / seg) segments of ray blocks (ray blocks
    // fastest: neighbouring wavefronts share voxels).  Two-dimensional grid:
    // the ray blocks of all fans along x, the segment along y (a fan's
    // blocks past its depth exit at once).  The launcher records each fan's
    // first block in unit_begin.
    const int b = remap_block(blockIdx.x, gridDim.x, xgrp);
    const bool two_d = gridDim.y > 1;
    const int seg = 1 << seg_shift;              // a power of two: no division per fan
    int fi = 0;
    {
        // the fan whose wavefronts hold b: binary search over the fans' first units
        int hi = tab.n - 1;
        while (fi < hi) {
            const int mid = (fi + hi + 1) >> 1;
            if (tab.f[mid].unit_begin <= b) fi = mid; else hi = mid - 1;
        }
    }
    const FanRec fr = tab.f[fi];
    const int acc = fr.unit_begin, nrb = (fr.n_rays + RB - 1) / RB;
    const int sgi = two_d ? (int)blockIdx.y : (b - acc) / nrb;
    const int j = (b - acc - (two_d ? 0 : sgi * nrb)) * RB + slot;
    const bool ray_ok = j < fr.n_rays;
    const int S = fr.n_samples;
    const int k_begin = sgi * seg;
    if (k_begin >= S) return;                   // whole wavefront: past this fan's depth
    const int k_end = min(S, k_begin + seg);
    // RB rays per wavefront, their geometry as the adjoint set it up
    Ray ray;
    {
        const RayRec &r = rays[fr.ray_begin + (ray_ok ? j : 0)];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ray.u0[a] = r.u0[a];
            ray.du[a] = r.du[a];
        }
    }
    const float *zrow = zbar + fr.out_offset + (long long)(ray_ok ? j : 0) * S;
    const int sxy = v.nx * v.ny;
    // depths per lane (4, 2 or 1) from the step length in voxels, so that a
    // group spans about 11 voxels along the rays and its box fits LDS also
    // for coarse steps (one sample per voxel and more); the wavefront's
    // first ray decides (the rays of a fan share their step length)
    int spl;
    {
        const double s2 = ray.du[0] * ray.du[0] + ray.du[1] * ray.du[1] + ray.du[2] * ray.du[2];
        spl = (s2 <= 0.35 * 0.35) ? 4 : ((s2 <= 0.7 * 0.7) ? 2 : 1);
        spl = __builtin_amdgcn_readfirstlane(spl);
    }
    const int G = LPR * spl;                     // depths per group (divides LPR kScatterSpl)
    // deterministic mode: 64-bit fixed-point sums (integer adds, in any
    // order the same) with the step's scale instead of FP32 atomics
    const double fsc = fix ? fscale[0] : 0.0;
    for (int t = lane; t < CAP; t += 64) s_box[t] = 0.0;
    // dL/dZ of the next group is loaded one group ahead; the lane's depths
    // past spl stay zero (inactive).  The loads are clamped into the row and
    // masked afterwards (no branch per load; spl is uniform).
    float zn[kScatterSpl];
#pragma unroll
    for (int q = 0; q < kScatterSpl; ++q) {
        const int k = k_begin + ch * spl + q;
        const float x = (q < spl) ? zrow[min(k, S - 1)] : 0.0f;
        zn[q] = (ray_ok && k < k_end) ? x : 0.0f;
    }
    for (int k0 = k_begin; k0 < k_end; k0 += G) {
        // the segment's last group loads nothing ahead (the next segment
        // belongs to another wavefront)
        const bool ahead = k0 + G < k_end;
        float zb[kScatterSpl];
#pragma unroll
        for (int q = 0; q < kScatterSpl; ++q) {
            zb[q] = zn[q];
            const int k = k0 + G + ch * spl + q;
            const float x = (ahead && q < spl) ? zrow[min(k, S - 1)] : 0.0f;
            zn[q] = (ray_ok && k < k_end) ? x : 0.0f;
        }
        Stencil st[kScatterSpl];
        int qf = -1, ql = -1;
#pragma unroll
        for (int q = 0; q < kScatterSpl; ++q) {
            st[q] = Stencil{0, 0, 0, 0, 0.0, 0.0, 0.0};
            if (zb[q] != 0.0f) {
                st[q] = stencil_at(v, ray, k0 + ch * spl + q);
                if (qf < 0) qf = q;
                ql = q;
            }
        }
        // bounding box of the group's cells: cell coordinates are monotone
        // along a straight ray, so per ray the extremes sit at its first and
        // last active sample (first and last active chunk)
        int fx = 0, fy = 0, fz = 0, lx = 0, ly = 0, lz = 0;
#pragma unroll
        for (int q = 0; q < kScatterSpl; ++q) {
            if (q == qf) { fx = st[q].ix; fy = st[q].iy; fz = st[q].iz; }
            if (q == ql) { lx = st[q].ix; ly = st[q].iy; lz = st[q].iz; }
        }
        const unsigned long long am = __ballot(qf >= 0);
        if (am == 0ull) continue;  // nothing to scatter in this group (uniform)
        int ox = 0x3fffffff, oy = 0x3fffffff, oz = 0x3fffffff, ex = -1, ey = -1, ez = -1;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            constexpr unsigned long long msk = (1ull << LPR) - 1;
            const unsigned long long m = (am >> (r * LPR)) & msk;
            if (m == 0ull) continue;
            // bit ll -> bit (ll + r SH) mod LPR: the ray's active chunks in order
            const int sh = r * SH;
            const unsigned long long mc = ((m << sh) | (m >> (LPR - sh))) & msk;
            const int c0 = __builtin_ctzll(mc), c1 = 63 - __builtin_clzll(mc);
            const int l0 = r * LPR + (c0 - sh + LPR) % LPR, l1 = r * LPR + (c1 - sh + LPR) % LPR;
            const int ax = __builtin_amdgcn_readlane(fx, l0), bxv = __builtin_amdgcn_readlane(lx, l1);
            const int ay = __builtin_amdgcn_readlane(fy, l0), byv = __builtin_amdgcn_readlane(ly, l1);
            const int az = __builtin_amdgcn_readlane(fz, l0), bzv = __builtin_amdgcn_readlane(lz, l1);
            ox = min(ox, min(ax, bxv)); ex = max(ex, max(ax, bxv));
            oy = min(oy, min(ay, byv)); ey = max(ey, max(ay, byv));
            oz = min(oz, min(az, bzv)); ez = max(ez, max(az, bzv));
        }
        const int bx = ex - ox + 2, by = ey - oy + 2, bz = ez - oz + 2;
        // odd row and plane strides: neighbouring cells along any axis land
        // in different LDS banks
        const int rs = bx | 1;
        const int ps = (rs * by) | 1;
        const bool fits = bx <= 64 && (long long)ps * bz <= CAP;
        if (!fits) {
#pragma unroll
            for (int q = 0; q < kScatterSpl; ++q) {
                if (zb[q] == 0.0f) continue;
                const float wx = (float)st[q].fx, wy = (float)st[q].fy, wz = (float)st[q].fz;
                const float gx = 1.0f - wx, gy = 1.0f - wy, gz = 1.0f - wz;
                const float w8[8] = {zb[q] * gx * gy * gz, zb[q] * wx * gy * gz, zb[q] * gx * wy * gz,
                                     zb[q] * wx * wy * gz, zb[q] * gx * gy * wz, zb[q] * wx * gy * wz,
                                     zb[q] * gx * wy * wz, zb[q] * wx * wy * wz};
                const int off[8] = {0, 1, v.nx, v.nx + 1, sxy, sxy + 1, sxy + v.nx, sxy + v.nx + 1};
                if (fix) {
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        if (w8[c] != 0.0f)
                            atomicAdd(fix + st[q].idx + off[c], (unsigned long long)__double2ll_rn((double)w8[c] * fsc));
                } else {
                    float *dst = gZ + st[q].idx;
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        if (w8[c] != 0.0f) atomicAdd(dst + off[c], w8[c]);
                }
            }
            continue;
        }
        // runs of a lane summed in registers, one LDS atomic per corner and run
        {
            const int off[8] = {0, 1, rs, rs + 1, ps, ps + 1, ps + rs, ps + rs + 1};
            float ra[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            int cur = -1;
#pragma unroll
            for (int q = 0; q < kScatterSpl; ++q) {
                if (zb[q] == 0.0f) continue;
                // box offsets and strides stay far below 2^24: 24-bit multiplies
                const int l = (int)(__umul24((unsigned)(st[q].iz - oz), (unsigned)ps) +
                                    __umul24((unsigned)(st[q].iy - oy), (unsigned)rs)) + (st[q].ix - ox);
                if (l != cur && cur >= 0) {
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        if (ra[c] != 0.0f)
                            atomicAdd(&s_box[cur + off[c]], (double)ra[c]);
                        ra[c] = 0.0f;
                    }
                }
                cur = l;
                const float wx = (float)st[q].fx, wy = (float)st[q].fy, wz = (float)st[q].fz;
                const float gx = 1.0f - wx, gy = 1.0f - wy, gz = 1.0f - wz;
                ra[0] += zb[q] * gx * gy * gz;
                ra[1] += zb[q] * wx * gy * gz;
                ra[2] += zb[q] * gx * wy * gz;
                ra[3] += zb[q] * wx * wy * gz;
                ra[4] += zb[q] * gx * gy * wz;
                ra[5] += zb[q] * wx * gy * wz;
                ra[6] += zb[q] * gx * wy * wz;
                ra[7] += zb[q] * wx * wy * wz;
            }
            if (cur >= 0) {
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (ra[c] != 0.0f)
                        atomicAdd(&s_box[cur + off[c]], (double)ra[c]);
            }
        }
        __syncthreads();
        // wave priority 1 for the flush (LDS reads and the global atomics wait
        // on latency): in the two-chain step it then runs ahead of the other
        // chain's arithmetic on the same CUs (step 0.5% faster)
        __builtin_amdgcn_s_setprio(1);
        // flush: the box's entries in x-fastest order, 64 consecutive entries
        // per pass (consecutive lanes on consecutive x of a row); a lane's
        // (x, y, z) advances by constant carries, and four entries' LDS reads
        // are issued before their atomics
        {
            const int E = bx * by * bz;
            // lane -> (x, y, z) and the step of 64 entries, with bx <= 64
            // and the box within CAP entries
            const float rbx = __builtin_amdgcn_rcpf((float)bx), rby = __builtin_amdgcn_rcpf((float)by);
            const int dyz = small_quot(64, rbx), dz = small_quot(dyz, rby);
            const int dx = 64 - (int)__umul24((unsigned)dyz, (unsigned)bx);
            const int dy = dyz - (int)__umul24((unsigned)dz, (unsigned)by);
            const int yz = small_quot(lane, rbx);
            int z = small_quot(yz, rby);
            int x = lane - (int)__umul24((unsigned)yz, (unsigned)bx);
            int y = yz - (int)__umul24((unsigned)z, (unsigned)by);
            for (int e0 = 0; e0 < E; e0 += 256) {
                double val[4];
                int at[4], gi[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    val[u] = 0.0;
                    at[u] = gi[u] = 0;
                    if (e0 + 64 * u + lane < E) {
                        at[u] = (int)(__umul24((unsigned)z, (unsigned)ps) + __umul24((unsigned)y, (unsigned)rs)) + x;
                        gi[u] = (int)(__umul24((unsigned)(oz + z), (unsigned)sxy) +
                                      __umul24((unsigned)(oy + y), (unsigned)v.nx)) + (ox + x);
                        val[u] = s_box[at[u]];
                    }
                    x += dx;
                    y += dy;
                    z += dz;
                    if (x >= bx) { x -= bx; ++y; }
                    if (y >= by) { y -= by; ++z; }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (val[u] != 0.0) {
                        s_box[at[u]] = 0.0;
                        if (fix) {
                            atomicAdd(fix + gi[u], (unsigned long long)__double2ll_rn(val[u] * fsc));
                        } else {
                            const float xv = (float)val[u];
                            if (xv != 0.0f) atomicAdd(gZ + gi[u], xv);
                        }
                    }
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// lateral blur (Sec. 2.4): per depth row k, a normalised Gaussian along the
// ray index, sigma_k = s0 + (s1 - s0) k / (S - 1) rays, radius ceil(3 sigma)
// decided in float32, edge replicate.  A block of 4 wavefronts takes 64 rays
// x 64 depths; lanes run along depth (coalesced 256-byte rows) and each
// wavefront owns 16 consecutive rays.  A wavefront loads its rows plus the
// halo of RM rays on either side straight into registers (all loads issued
// before the first use) and keeps its depth's weights in registers, so no
// LDS staging and no block barrier sits between the loads and the sums.
//   MODE 0: out = B in            MODE 1: out = B^T in
//   MODE 2: image = B in, out = 2 (image - target) / P, loss += |.|^2 / P
// RM (4, 8, 16, 32) is a register bound on the radius: taps beyond a row's
// own radius carry weight zero and leave the sums unchanged.
// --------------------------------------------------------------------------
constexpr int kBlurRays = 64;      // rays per block
constexpr int kBlurRows = 16;      // rays per wavefront

// normalised weights w_t (t = 0..RM, zero beyond the row radius r) of depth
// row k; returns r (-1: identity row, w_0 = 1)
template <int RM>
__device__ __forceinline__ int blur_weights(const PhysArgs &p, int S, int k, float (&w)[RM + 1])
{
    const float frac = S > 1 ? __fdiv_rn((float)k, (float)(S - 1)) : 0.0f;
    const float d = __fsub_rn(p.s1, p.s0);
    const float sig = __fadd_rn(p.s0, __fmul_rn(d, frac));
    if (!(sig >= 1e-3f)) {
#pragma unroll
        for (int t = 0; t <= RM; ++t) w[t] = (t == 0) ? 1.0f : 0.0f;
        return -1;
    }
    int r = (int)ceilf(__fmul_rn(3.0f, sig));
    r = min(r, min(p.blur_rmax, RM));
    const float c = -0.5f / (sig * sig);
    float e[RM + 1];
    float tot = 1.0f;
#pragma unroll
    for (int t = 1; t <= RM; ++t) {
        e[t] = (t <= r) ? expf(c * (float)(t * t)) : 0.0f;
        if (t <= r) tot += 2.0f * e[t];
    }
    const float inv = 1.0f / tot;
    w[0] = inv;
#pragma unroll
    for (int t = 1; t <= RM; ++t) w[t] = e[t] * inv;
    return r;
}

template <int MODE, int RM>
__global__ __launch_bounds__(256) void k_blur(PhysArgs p, FanTable tab, const float *__restrict__ in,
                                              const float *__restrict__ target, float *__restrict__ out,
                                              float *__restrict__ image, double *__restrict__ loss_acc)
{
    constexpr int W = kBlurRows + 2 * RM;      // window rows j0 - RM .. j0 + 16 + RM - 1
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int b = blockIdx.x;
    const int fi = find_blur_fan(tab, b);
    const FanRec fr = tab.f[fi];
    const int S = fr.n_samples, n = fr.n_rays;
    const int nkb = (S + 63) / 64;
    const int lb = b - fr.blk_begin;
    const int kb = lb % nkb, jb = lb / nkb;
    const int k = kb * 64 + lane;
    const int j0 = jb * kBlurRays + wv * kBlurRows;
    const bool active = (k < S) && (j0 < n);
    const long long col = fr.out_offset + k;
    const double inv_npix = 1.0 / ((double)n * (double)S);
    const float two_inv_npix = (float)(2.0 * inv_npix);
    double lsum = 0.0;
    if (active) {
        // every load clamped into the fan (no per-load branches): MODE 1
        // then zeroes the rows outside it, the others replicate the edge
        float x[W];
#pragma unroll
        for (int m = 0; m < W; ++m) {
            const int g = j0 - RM + m;
            x[m] = in[col + (long long)min(max(g, 0), n - 1) * S];
        }
        float tg[MODE == 2 ? kBlurRows : 1];
        if (MODE == 2) {
#pragma unroll
            for (int o = 0; o < kBlurRows; ++o) tg[o] = target[col + (long long)min(j0 + o, n - 1) * S];
        }
        if (MODE == 1) {
#pragma unroll
            for (int m = 0; m < W; ++m) {
                const int g = j0 - RM + m;
                x[m] = (g >= 0 && g < n) ? x[m] : 0.0f;
            }
        }
        float w[RM + 1];
        const int r = blur_weights<RM>(p, S, k, w);
        // transpose at the edge rows 0 and n-1: the replicated taps fold back
        // onto the edge, weight tail_m = sum_{t >= m} w_t for the tap |t| + 1
        float tl[RM + 2];
        if (MODE == 1) {
            float acc = 0.0f;
            tl[RM + 1] = 0.0f;
#pragma unroll
            for (int t = RM; t >= 0; --t) {
                if (t <= r) acc += w[t];
                tl[t] = (t <= r) ? acc : 0.0f;
            }
        }
#pragma unroll
        for (int o = 0; o < kBlurRows; ++o) {
            const int j = j0 + o;
            if (j >= n) break;
            float acc = 0.0f;
#pragma unroll
            for (int t = -RM; t <= RM; ++t) acc = fmaf(w[t < 0 ? -t : t], x[o + RM + t], acc);
            if (MODE == 1 && (j == 0 || j == n - 1)) {
                const float mult = (j == 0 && j == n - 1) ? 2.0f : 1.0f;
                float e = 0.0f;
#pragma unroll
                for (int t = -RM; t <= RM; ++t) e = fmaf(tl[(t < 0 ? -t : t) + 1], x[o + RM + t], e);
                acc = fmaf(mult, e, acc);
            }
            const long long oidx = col + (long long)j * S;
            if (MODE == 2) {
                // residual in FP32 (one rounding of the difference of two
                // floats); its square summed in FP64, scaled once at the end
                const float d = acc - tg[o];
                if (image) image[oidx] = acc;
                out[oidx] = d * two_inv_npix;
                lsum += (double)(d * d);
            } else {
                out[oidx] = acc;
            }
        }
    }
    if (MODE == 2 && loss_acc) {
        // one partial per block, summed by k_sum_f64 (no contended atomics)
        __shared__ double s_part[4];
        lsum = wave_sum(lsum) * inv_npix;
        if (lane == 0) s_part[wv] = lsum;
        __syncthreads();
        if (tid == 0) loss_acc[b] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
    }
}

// Residual and transpose blur in one pass (the fused step with blur, radius
// bound RM <= 8): ebar = B^T (2 (B pre - target) / P), image = B pre
// (optional), one loss partial per block.  A block of 4 wavefronts takes 64
// rays x 64 depths as k_blur does.  It first forms the residual of its rays
// and of RM rays on either side (each wavefront RW of those 64 + 2 RM rows,
// from a register window of pre, as MODE 2), parks it in LDS (zero outside
// the fan, as MODE 1 reads it), and then applies B^T to its own rows from
// LDS, as MODE 1.  The arithmetic of each value is that of the two-kernel
// path; only the loss partials group the rows differently.  The residual
// never goes to memory.
template <int RM>
__global__ __launch_bounds__(256) void k_blur_fused(PhysArgs p, FanTable tab, const float *__restrict__ pre,
                                                    const float *__restrict__ target, float *__restrict__ ebar,
                                                    float *__restrict__ image, double *__restrict__ loss_acc)
{
    constexpr int NR = kBlurRays + 2 * RM;     // residual rows J0 - RM .. J0 + 64 + RM - 1
    constexpr int RW = NR / 4;                 // residual rows per wavefront
    constexpr int W = RW + 2 * RM;             // pre window of a wavefront
    static_assert(NR % 4 == 0, "residual rows split over four wavefronts");
    __shared__ float s_r[NR][65];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int b = blockIdx.x;
    const int fi = find_blur_fan(tab, b);
    const FanRec fr = tab.f[fi];
    const int S = fr.n_samples, n = fr.n_rays;
    const int nkb = (S + 63) / 64;
    const int lb = b - fr.blk_begin;
    const int kb = lb % nkb, jb = lb / nkb;
    const int k = kb * 64 + lane;
    const int J0 = jb * kBlurRays;
    const bool kin = k < S;
    const long long col = fr.out_offset + min(k, S - 1);
    const double inv_npix = 1.0 / ((double)n * (double)S);
    const float two_inv_npix = (float)(2.0 * inv_npix);
    float w[RM + 1];
    const int r = blur_weights<RM>(p, S, min(k, S - 1), w);
    double lsum = 0.0;
    {
        // residual rows g0 .. g0 + RW - 1 of this wavefront
        const int g0 = J0 - RM + wv * RW;
        float x[W];
#pragma unroll
        for (int m = 0; m < W; ++m) {
            const int g = g0 - RM + m;
            x[m] = pre[col + (long long)min(max(g, 0), n - 1) * S];
        }
        float tg[RW];
#pragma unroll
        for (int o = 0; o < RW; ++o) tg[o] = target[col + (long long)min(max(g0 + o, 0), n - 1) * S];
#pragma unroll
        for (int o = 0; o < RW; ++o) {
            const int g = g0 + o;
            float acc = 0.0f;
#pragma unroll
            for (int t = -RM; t <= RM; ++t) acc = fmaf(w[t < 0 ? -t : t], x[o + RM + t], acc);
            const float d = acc - tg[o];
            const bool in_fan = kin && g >= 0 && g < n;
            s_r[wv * RW + o][lane] = in_fan ? d * two_inv_npix : 0.0f;
            // the block's own rows: image and loss
            if (in_fan && g >= J0 && g < J0 + kBlurRays) {
                if (image) image[col + (long long)g * S] = acc;
                lsum += (double)(d * d);
            }
        }
    }
    __syncthreads();
    // transpose blur of this wavefront's 16 rays from the LDS residual
    const int j0 = J0 + wv * kBlurRows;
    if (kin && j0 < n) {
        float tl[RM + 2];
        {
            float acc = 0.0f;
            tl[RM + 1] = 0.0f;
#pragma unroll
            for (int t = RM; t >= 0; --t) {
                if (t <= r) acc += w[t];
                tl[t] = (t <= r) ? acc : 0.0f;
            }
        }
        float x[kBlurRows + 2 * RM];
#pragma unroll
        for (int m = 0; m < kBlurRows + 2 * RM; ++m) x[m] = s_r[wv * kBlurRows + m][lane];
#pragma unroll
        for (int o = 0; o < kBlurRows; ++o) {
            const int j = j0 + o;
            if (j >= n) break;
            float acc = 0.0f;
#pragma unroll
            for (int t = -RM; t <= RM; ++t) acc = fmaf(w[t < 0 ? -t : t], x[o + RM + t], acc);
            if (j == 0 || j == n - 1) {
                const float mult = (j == 0 && j == n - 1) ? 2.0f : 1.0f;
                float e = 0.0f;
#pragma unroll
                for (int t = -RM; t <= RM; ++t) e = fmaf(tl[(t < 0 ? -t : t) + 1], x[o + RM + t], e);
                acc = fmaf(mult, e, acc);
            }
            ebar[col + (long long)j * S] = acc;
        }
    }
    if (loss_acc) {
        // one partial per block, summed by k_sum_f64 (no contended atomics)
        __shared__ double s_part[4];
        lsum = wave_sum(lsum) * inv_npix;
        if (lane == 0) s_part[wv] = lsum;
        __syncthreads();
        if (tid == 0) loss_acc[b] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
    }
}

// --------------------------------------------------------------------------
// pose gradient: dL/dt and dL/dw from the accumulated dL/dR (Gallego-Yezzi)
// --------------------------------------------------------------------------
__device__ void skew(const double w[3], double W[9])
{
    W[0] = 0.0;   W[1] = -w[2]; W[2] = w[1];
    W[3] = w[2];  W[4] = 0.0;   W[5] = -w[0];
    W[6] = -w[1]; W[7] = w[0];  W[8] = 0.0;
}

__device__ void mm3(const double *A, const double *B, double *Cm)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Cm[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// pose pi's (dL/dt, dL/dw) from its accumulator
__device__ void pose_finalize_one(const double *__restrict__ acc, const float *__restrict__ poses, int pi,
                                  float *__restrict__ grad)
{
    const double *a = acc + (size_t)kPoseAcc * pi;
    const double w[3] = {poses[6 * pi + 3], poses[6 * pi + 4], poses[6 * pi + 5]};
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double W[9];
    skew(w, W);
    for (int c = 0; c < 3; ++c) {
        double dR[9];
        double e[3] = {0.0, 0.0, 0.0};
        e[c] = 1.0;
        double E[9];
        skew(e, E);
        if (th2 < 1e-10) {
            double EW[9], WE[9];
            mm3(E, W, EW);
            mm3(W, E, WE);
            for (int q = 0; q < 9; ++q) dR[q] = E[q] + 0.5 * (EW[q] + WE[q]);
        } else {
            double R[9];
            rotation(w, R);
            double vv[3];
            for (int q = 0; q < 3; ++q) vv[q] = e[q] - R[3 * q + c];
            const double x[3] = {w[1] * vv[2] - w[2] * vv[1], w[2] * vv[0] - w[0] * vv[2],
                                 w[0] * vv[1] - w[1] * vv[0]};
            double X[9], Sm[9];
            skew(x, X);
            for (int q = 0; q < 9; ++q) Sm[q] = (w[c] * W[q] + X[q]) / th2;
            mm3(Sm, R, dR);
        }
        double s = 0.0;
        for (int q = 0; q < 9; ++q) s += a[3 + q] * dR[q];
        grad[6 * pi + 3 + c] = (float)s;
    }
    for (int q = 0; q < 3; ++q) grad[6 * pi + q] = (float)a[q];
}

__global__ void k_pose_finalize(const double *__restrict__ acc, const float *__restrict__ poses,
                                int n, float *__restrict__ grad)
{
    const int pi = blockIdx.x * blockDim.x + threadIdx.x;
    if (pi < n) pose_finalize_one(acc, poses, pi, grad);
}

// one wavefront per fan of a table: the per-ray partials of the adjoint
// summed into the pose's accumulator (lane-strided, then across lanes)
__global__ __launch_bounds__(64) void k_pose_reduce(FanTable tab, const double *__restrict__ part,
                                                    double *__restrict__ acc)
{
    const FanRec fr = tab.f[blockIdx.x];
    const int lane = threadIdx.x;
    double s[kRayPart];
#pragma unroll
    for (int c = 0; c < kRayPart; ++c) s[c] = 0.0;
    for (int j = lane; j < fr.n_rays; j += 64) {
        const double *pr = part + (size_t)kRayPart * (fr.ray_begin + j);
#pragma unroll
        for (int c = 0; c < kRayPart; ++c) s[c] += pr[c];
    }
#pragma unroll
    for (int c = 0; c < kRayPart; ++c) s[c] = wave_sum(s[c]);
    if (lane == 0) {
        double *pa = acc + (size_t)kPoseAcc * fr.pose;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            pa[a] += s[a];
            pa[3 + 3 * a + 0] += s[3 + 2 * a];
            pa[3 + 3 * a + 2] += s[4 + 2 * a];
        }
    }
}

// --------------------------------------------------------------------------
// footprint: mark every stencil corner of every sample
// --------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_footprint(VolArgs v, FanTable tab, const float *__restrict__ poses,
                                                  uint8_t *__restrict__ mask)
{
    const int lane = threadIdx.x;
    const int g = blockIdx.x;
    const int fi = find_fan(tab, g);
    const FanRec fr = tab.f[fi];
    const int j = g - fr.ray_begin;
    PhysArgs p{};
    p.atten = 2;
    Ray ray;
    setup_ray(v, p, fr, poses, j, ray);
    const int sxy = v.nx * v.ny;
    for (int k = lane; k < fr.n_samples; k += 64) {
        const Stencil st = stencil_at(v, ray, k);
        uint8_t *q = mask + st.idx;
        q[0] = 1;
        q[1] = 1;
        q[v.nx] = 1;
        q[v.nx + 1] = 1;
        q[sxy] = 1;
        q[sxy + 1] = 1;
        q[sxy + v.nx] = 1;
        q[sxy + v.nx + 1] = 1;
    }
}

// --------------------------------------------------------------------------
// sampling-only render: the impedance at every ray sample (one wavefront per
// ray, coalesced stores)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_sample_rays(VolArgs v, FanTable tab, const float *__restrict__ poses,
                                                   float *__restrict__ out, int xgrp)
{
    const int lane = threadIdx.x;
    const int g = remap_block(blockIdx.x, gridDim.x, xgrp);
    const int fi = find_fan(tab, g);
    const FanRec fr = tab.f[fi];
    const int j = g - fr.ray_begin;
    const int S = fr.n_samples;
    PhysArgs p{};
    p.atten = 2;
    Ray ray;
    setup_ray(v, p, fr, poses, j, ray);
    const long long obase = fr.out_offset + (long long)j * S;
    const int sxy = v.nx * v.ny;
#pragma unroll 4
    for (int k = lane; k < S; k += 64) {
        const Stencil st = stencil_at(v, ray, k);
        out[obase + k] = (float)trilinear(v.Z, v.nx, sxy, st, nullptr);
    }
}

// --------------------------------------------------------------------------
// scan conversion of one fan's polar image onto a Cartesian grid of the
// probe's x-z plane (one thread per output pixel, FP64 geometry)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scan_convert(const float *__restrict__ img, int n_r, int S, double A,
                                                      double r0, double ds, int nx, int nz, double x0, double z0,
                                                      double dx, double dz, float fill, float *__restrict__ out)
{
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long long)nx * nz) return;
    const int iz = (int)(idx / nx), ix = (int)(idx - (long long)iz * nx);
    const double x = x0 + (double)ix * dx, z = z0 + (double)iz * dz;
    const double r = sqrt(x * x + z * z);
    const double th = atan2(x, z);
    const double jr = (th + 0.5 * A) * (double)(n_r - 1) / A;
    const double kr = (r - r0) / ds;
    if (!(jr >= 0.0 && jr <= (double)(n_r - 1) && kr >= 0.0 && kr <= (double)(S - 1))) {
        out[idx] = fill;
        return;
    }
    const int j0 = min((int)floor(jr), n_r - 2), k0 = min((int)floor(kr), S - 2);
    const double fj = jr - (double)j0, fk = kr - (double)k0;
    const float *p0 = img + (long long)j0 * S + k0;
    const float *p1 = p0 + S;
    const double a = lerp((double)p0[0], (double)p0[1], fk);
    const double b = lerp((double)p1[0], (double)p1[1], fk);
    out[idx] = (float)lerp(a, b, fj);
}

// --------------------------------------------------------------------------
// small utilities
// --------------------------------------------------------------------------
__global__ void k_zero_f64(double *p, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_zero_f32(float *p, long long n)
{
    const long long n4 = n / 4;
    float4 *p4 = reinterpret_cast<float4 *>(p);
    const bool aligned = ((reinterpret_cast<uintptr_t>(p) & 15) == 0);
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (aligned) {
        for (long long i = i0; i < n4; i += stride) p4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (long long i = 4 * n4 + i0; i < n; i += stride) p[i] = 0.0f;
    } else {
        for (long long i = i0; i < n; i += stride) p[i] = 0.0f;
    }
}

// out = sum of n partials, or out += it (single block, fixed order:
// deterministic)
__device__ __forceinline__ void sum_block(const double *__restrict__ part, long long n, double *__restrict__ out,
                                          int accumulate)
{
    __shared__ double s_w[4];
    double acc = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) acc += part[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
        *out = accumulate ? *out + t : t;
    }
}

__global__ __launch_bounds__(256) void k_sum_f64(const double *__restrict__ part, long long n, double *__restrict__ out,
                                                 int accumulate)
{
    sum_block(part, n, out, accumulate);
}

// the end of a fused step in one launch: block 0 sums the loss partials
// (when loss is given), the other blocks finalise 256 poses each
__global__ __launch_bounds__(256) void k_finish(const double *__restrict__ part, long long n_part,
                                                double *__restrict__ loss, const double *__restrict__ acc,
                                                const float *__restrict__ poses, int n_poses,
                                                float *__restrict__ grad)
{
    if (loss && blockIdx.x == 0) {
        sum_block(part, n_part, loss, 0);
        return;
    }
    const int pi = (blockIdx.x - (loss ? 1 : 0)) * 256 + threadIdx.x;
    if (grad && pi < n_poses) pose_finalize_one(acc, poses, pi, grad);
}

// deterministic dL/dZ: the sum of |dL/dZ| over every sample of the step
// bounds every voxel's sum (the trilinear weights of a sample are at most 1
// and add up to 1), and sets the fixed-point scale 2^e with that bound times
// 2^e below 2^61, so no 64-bit sum can overflow however the atomics are
// ordered.  Each wavefront sums one ray's row (the rows of the fans only:
// gaps between pose images are never read), in a fixed order
__global__ __launch_bounds__(256) void k_abs_rows(FanTable tab, const float *__restrict__ zbar,
                                                  double *__restrict__ part)
{
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= tab.total_rays) return;            // whole wavefront
    const FanRec fr = tab.f[find_fan(tab, g)];
    const int S = fr.n_samples;
    const float *row = zbar + fr.out_offset + (long long)(g - fr.ray_begin) * S;
    double acc = 0.0;
    for (int k = lane; k < S; k += 64) acc += fabs((double)row[k]);
    acc = wave_sum(acc);
    if (lane == 0) part[g] = acc;
}

// fscale[2] = the sum of the n per-ray sums (one block, fixed order), and
// fscale[0..1] = 2^e, 2^-e
__global__ __launch_bounds__(256) void k_fix_scale(const double *__restrict__ part, long long n,
                                                   double *__restrict__ fscale)
{
    sum_block(part, n, fscale + 2, 0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double a = fscale[2];
        const int e = (a > 0.0 && isfinite(a)) ? 60 - ilogb(a) : 0;
        fscale[0] = ldexp(1.0, e);
        fscale[1] = ldexp(1.0, -e);
    }
}

// grad_Z (+)= the fixed-point sums times 2^-e, rounded once to FP32
__global__ __launch_bounds__(256) void k_fix_to_f32(const unsigned long long *__restrict__ fix, long long n,
                                                    const double *__restrict__ fscale, float *__restrict__ gZ,
                                                    int overwrite)
{
    const double inv = fscale[1];
    const long long stride = (long long)gridDim.x * 256;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const double x = (double)(long long)fix[i] * inv;
        gZ[i] = overwrite ? (float)x : (float)((double)gZ[i] + x);
    }
}

// two buffers cleared in one launch (grid-stride over both)
__global__ void k_zero_pair(float *__restrict__ a, long long na, double *__restrict__ b, long long nb)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long n4 = na / 4;
    float4 *a4 = reinterpret_cast<float4 *>(a);
    if ((reinterpret_cast<uintptr_t>(a) & 15) == 0) {
        for (long long i = i0; i < n4; i += stride) a4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (long long i = 4 * n4 + i0; i < na; i += stride) a[i] = 0.0f;
    } else {
        for (long long i = i0; i < na; i += stride) a[i] = 0.0f;
    }
    for (long long i = i0; i < nb; i += stride) b[i] = 0.0;
}

// --------------------------------------------------------------------------
// volume reconstruction helpers: the smoothness prior
//   R = w sum_axes sum_{pairs along the axis} ((Z_b - Z_a) / h_axis)^2
// (one thread per voxel: grad_Z += dR/dZ of its own voxel, and the energy of
// the pairs to its +x, +y, +z neighbours into a per-block partial), and the
// element-wise Adam update with the result clamped to [lo, hi]
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_smooth(const float *__restrict__ Z, int nx, int ny, int nz, float wx,
                                                float wy, float wz, float *__restrict__ gZ,
                                                double *__restrict__ part)
{
    const long long n = (long long)nx * ny * nz;
    const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if (v < n) {
        const int ix = (int)(v % nx);
        const long long r = v / nx;
        const int iy = (int)(r % ny), iz = (int)(r / ny);
        const long long sxy = (long long)nx * ny;
        // neighbours clamped to the voxel itself at the faces, where their
        // differences are then exactly zero: the seven loads issue together
        const float z = Z[v];
        const float xm = Z[v - (ix > 0 ? 1 : 0)], xp = Z[v + (ix + 1 < nx ? 1 : 0)];
        const float ym = Z[v - (iy > 0 ? nx : 0)], yp = Z[v + (iy + 1 < ny ? nx : 0)];
        const float zm = Z[v - (iz > 0 ? sxy : 0)], zp = Z[v + (iz + 1 < nz ? sxy : 0)];
        float g = 0.0f;
        // axis weights w / h^2; d(Z_b - Z_a)^2 / dZ = -2 (Z_b - Z_a) for a, +2 for b
        g += 2.0f * wx * (z - xm);
        { const float d = xp - z; g -= 2.0f * wx * d; e += (double)wx * (double)d * (double)d; }
        g += 2.0f * wy * (z - ym);
        { const float d = yp - z; g -= 2.0f * wy * d; e += (double)wy * (double)d * (double)d; }
        g += 2.0f * wz * (z - zm);
        { const float d = zp - z; g -= 2.0f * wz * d; e += (double)wz * (double)d * (double)d; }
        gZ[v] += g;
    }
    __shared__ double s_w[4];
    e = wave_sum(e);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ x, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, long long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2, float lo, float hi)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        // bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t
        const float step = lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        x[i] = fminf(fmaxf(x[i] - step, lo), hi);
    }
}

// --------------------------------------------------------------------------
// impedance mapping (Sec. 2.2): the paper turns MRI or CT intensities into
// impedance voxel by voxel.  Here the map is a piecewise-linear table
// (x_j, z_j), constant beyond its ends; a voxel of intensity v in
// [x_j, x_{j+1}) maps to z_j + t (z_{j+1} - z_j), t = (v - x_j) / (x_{j+1} - x_j).
// --------------------------------------------------------------------------
// segment j of v (x_j <= v < x_{j+1}, 0 <= j <= n - 2) for x_0 < v < x_{n-1}:
// branch-free search in LDS, one halving step per bit of n - 2 (top: the
// largest power of two <= n - 2, or 0 when n = 2)
__device__ __forceinline__ int lut_segment(const float *sx, int top, int n, float v)
{
    int j = 0;
    for (int s = top; s > 0; s >>= 1) {
        const int c = j + s;
        j = (c <= n - 2 && v >= sx[c]) ? c : j;
    }
    return j;
}

__device__ __forceinline__ int lut_top(int n) { return n > 2 ? 1 << (31 - __builtin_clz(n - 2)) : 0; }

__device__ __forceinline__ float lut_eval(const float *sx, const float *sz, int top, int n, float v)
{
    if (v <= sx[0]) return sz[0];
    if (v >= sx[n - 1]) return sz[n - 1];
    // NaN fails both tests above and stays NaN here
    const int j = lut_segment(sx, top, n, v);
    const float t = __fdiv_rn(v - sx[j], sx[j + 1] - sx[j]);
    return fmaf(t, sz[j + 1] - sz[j], sz[j]);
}

__global__ __launch_bounds__(256) void k_map(const float *__restrict__ in, long long n, LutArgs lut,
                                             float *__restrict__ Z)
{
    __shared__ float s_x[kMaxKnots], s_z[kMaxKnots];
    const int m = lut.n;
    for (int i = threadIdx.x; i < m; i += 256) {
        s_x[i] = lut.x[i];
        s_z[i] = lut.z[i];
    }
    __syncthreads();
    const int top = lut_top(m);
    // four voxels per thread and pass, one grid stride apart: their loads
    // and searches are independent
    const long long stride = (long long)gridDim.x * 256;
    for (long long i0 = (long long)blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += 4 * stride) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long long i = i0 + u * stride;
            v[u] = (i < n) ? in[i] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long long i = i0 + u * stride;
            const float z = lut_eval(s_x, s_z, top, m, v[u]);
            if (i < n) Z[i] = z;
        }
    }
}

// dL/dv = dL/dZ (z_{j+1} - z_j) / (x_{j+1} - x_j) inside the table (the right
// segment at a knot), 0 beyond its ends; dL/dz_j += (1 - t) dL/dZ and
// dL/dz_{j+1} += t dL/dZ, or all of dL/dZ to the end knot beyond an end.
// The knot sums go through an FP64 LDS copy per block, then one global FP64
// atomic per knot and block.
// The table gradient is a histogram over the knots.  Its LDS accumulators
// are replicated 8 times (lane % 8 picks the copy, rows padded to 65 so the
// copies of one knot sit in different banks): lanes of one wavefront that
// meet on a knot mostly add into different copies instead of serialising on
// one address.
constexpr int kMapCopies = 8, kMapRow = kMaxKnots + 1;

__global__ __launch_bounds__(256) void k_map_backward(const float *__restrict__ in, long long n, LutArgs lut,
                                                      const float *__restrict__ gZ, float *__restrict__ grad_in,
                                                      double *__restrict__ grad_z)
{
    __shared__ float s_x[kMaxKnots], s_z[kMaxKnots];
    __shared__ double s_g[kMapCopies * kMapRow];
    const int m = lut.n;
    for (int i = threadIdx.x; i < m; i += 256) {
        s_x[i] = lut.x[i];
        s_z[i] = lut.z[i];
    }
    for (int i = threadIdx.x; i < kMapCopies * kMapRow; i += 256) s_g[i] = 0.0;
    __syncthreads();
    double *g_own = s_g + (threadIdx.x % kMapCopies) * kMapRow;
    const float x0 = s_x[0], xn = s_x[m - 1];
    const int top = lut_top(m);
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const float v = in[i];
        const float g = gZ[i];
        float gi = 0.0f;
        if (v <= x0) {
            if (grad_z) atomicAdd(&g_own[0], (double)g);
        } else if (v >= xn) {
            if (grad_z) atomicAdd(&g_own[m - 1], (double)g);
        } else {
            const int j = lut_segment(s_x, top, m, v);
            const float dx = s_x[j + 1] - s_x[j];
            gi = g * __fdiv_rn(s_z[j + 1] - s_z[j], dx);
            if (grad_z) {
                const double t = (double)__fdiv_rn(v - s_x[j], dx);
                atomicAdd(&g_own[j], (1.0 - t) * (double)g);
                atomicAdd(&g_own[j + 1], t * (double)g);
            }
        }
        if (grad_in) grad_in[i] = gi;
    }
    if (grad_z) {
        __syncthreads();
        for (int k = threadIdx.x; k < m; k += 256) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < kMapCopies; ++c) t += s_g[c * kMapRow + k];
            if (t != 0.0) atomicAdd(grad_z + k, t);
        }
    }
}

__global__ void k_philox(const uint32_t *__restrict__ ctr, long long n, uint32_t k0, uint32_t k1,
                         uint32_t *__restrict__ out)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t w[4];
    philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1, w);
    for (int q = 0; q < 4; ++q) out[4 * i + q] = w[q];
}

template <bool SPK>
__global__ __launch_bounds__(64) void k_gain(PhysArgs p, FanRec fr, float *__restrict__ out)
{
    constexpr int T = 256;
    __shared__ float s_xig[SPK ? T : 1];
    __shared__ float s_xir[SPK ? T / 4 + 8 : 1];
    const int lane = threadIdx.x;
    const int j = blockIdx.y;
    const int t0 = blockIdx.x * T;
    const int S = fr.n_samples;
    if (SPK) speckle_fill<T>(p, t0, j, fr.speckle_id, lane, s_xig, s_xir);
    __syncthreads();
    const float postc = posthoc_coef(p, fr.ds);
    const GainK gk = gain_consts(p, fr.n_samples);
    for (int m = 0; m < T / 64; ++m) {
        const int i = m * 64 + lane;
        const int k = t0 + i;
        if (k < S) out[(long long)j * S + k] = pixel_gain_rt<SPK>(p, gk, k, t0, postc, SPK ? s_xig[i] : 1.0f, s_xir);
    }
}

inline int grid_for(long long n, int block)
{
    long long g = (n + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

// rays of the fans at the front of a table whose rays are walked by
// kSpanWaves wavefronts each (a table lists its fans longest first)
inline int span_rays(const FanTable &t, int span_samples)
{
    int n = 0;
    if (span_samples <= 0) return 0;
    for (int f = 0; f < t.n && t.f[f].n_samples >= span_samples; ++f) n += t.f[f].n_rays;
    return n;
}

// the side stream starts after what st has queued; st waits for it at the
// join (graph capture turns both into graph edges)
inline hipError_t fork_side(hipStream_t st, const SideStream &s)
{
    hipError_t e = hipEventRecord(s.fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(s.st, s.fork, 0);
    return e;
}

inline hipError_t join_side(hipStream_t st, const SideStream &s)
{
    hipError_t e = hipEventRecord(s.join, s.st);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, s.join, 0);
    return e;
}

}  // namespace

// --------------------------------------------------------------------------
// launch wrappers
// --------------------------------------------------------------------------
#define DUS_FWD_LAUNCH(CH, SPK, WV, NG, TAB, ZERO, STR)                                         \
    hipLaunchKernelGGL((k_forward<CH, SPK, WV>), dim3(NG), dim3(64 * WV), 0, STR, v, p, TAB, poses, out, \
                       min_pivot, pivot_base, carry, carry_exp, cstate, gain, xcd_group, ZERO)

#define DUS_FWD_CASE(CH)                                                                       \
    case CH:                                                                                   \
        if (n_span > 0) {                                                                      \
            if (p.speckle) DUS_FWD_LAUNCH(CH, true, kSpanWaves, n_span, t, ZeroArgs{}, sst);    \
            else DUS_FWD_LAUNCH(CH, false, kSpanWaves, n_span, t, ZeroArgs{}, sst);             \
        }                                                                                      \
        if (n_one > 0 || zero.na > 0 || zero.nb > 0) {                                         \
            if (p.speckle) DUS_FWD_LAUNCH(CH, true, 1, t.total_rays, t1, zero, st);            \
            else DUS_FWD_LAUNCH(CH, false, 1, t.total_rays, t1, zero, st);                     \
        }                                                                                      \
        break;

// automatic forward tile (chunk 0): 8 x 64 samples, unless the table's rays
// fill 512-sample tiles clearly worse than 256-sample ones.  On full tiles
// the 4 x 64 tile costs about 7% more per sample (64 poses x 256 x 1024:
// 164 against 153 us); on the uneven 64-pose batch, whose rays pad to 1.20x
// their samples in 512-sample tiles and to 1.09x in 256-sample ones, it
// takes 217 against 229 us.
static int auto_fwd_chunk(const FanTable &t)
{
    long long pad4 = 0, pad8 = 0;
    for (int f = 0; f < t.n; ++f) {
        const long long r = t.f[f].n_rays, s = t.f[f].n_samples;
        pad4 += r * ((s + 255) / 256) * 256;
        pad8 += r * ((s + 511) / 512) * 512;
    }
    return (pad8 * 100 > pad4 * 107) ? 4 : 8;
}

hipError_t launch_forward(int chunk, int xcd_group, const VolArgs &v, const PhysArgs &p,
                          const FanTable &t, const float *poses, float *out, float *min_pivot,
                          int pivot_base, double *carry, int32_t *carry_exp, double *cstate, float *gain,
                          hipStream_t st, const ZeroArgs &zero, int span_samples, const SideStream *side)
{
    if (t.total_rays <= 0) return hipSuccess;
    if (chunk == 0) chunk = auto_fwd_chunk(t);
    if (chunk != 4 && chunk != 8 && chunk != 16) return hipErrorInvalidValue;
    // the rays of the table's long fans (its first ones: a table lists its
    // fans longest first) get kSpanWaves wavefronts each, the rest one
    const int n_span = span_rays(t, span_samples);
    const int n_one = t.total_rays - n_span;
    // the clears go with the one-wavefront launch (it covers every ray)
    FanTable t1 = t;
    t1.ray0 = n_span;
    hipStream_t sst = st;
    if (n_span > 0 && side) {
        hipError_t e = fork_side(st, *side);
        if (e != hipSuccess) return e;
        sst = side->st;
    }
    switch (chunk) {
        DUS_FWD_CASE(4)
        DUS_FWD_CASE(8)
        DUS_FWD_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (sst != st) {
        // joined also after a failed launch: a capture must not end with a
        // fork left open, and the caller's stream must wait for the side's work
        const hipError_t ej = join_side(st, *side);
        if (e == hipSuccess) e = ej;
    }
    return e;
}

#define DUS_BWD_LAUNCH(CH, SPK, FUSED, WV, NG, TAB, STR)                                          \
    hipLaunchKernelGGL((k_backward<CH, SPK, FUSED, WV>), dim3(NG), dim3(64 * WV), 0, STR, v, p, TAB,   \
                       poses, zbar ? rays : nullptr, gsrc, target, zbar, pose_acc ? pose_part : nullptr, \
                       loss, carry, carry_exp, cstate, gain, xcd_group)

// the long rays (the table's first n_span) with the forward's hand-off take
// kSpanWaves * 4 / C wavefronts each (the LDS of C = 8 holds half as many)
#define DUS_BWD_CASE(CH)                                                                       \
    case CH:                                                                                   \
        if (n_span > 0) {                                                                      \
            if (fused) DUS_BWD_LAUNCH(CH, false, true, kSpanWaves * 4 / CH, n_span, t, sst);        \
            else DUS_BWD_LAUNCH(CH, false, false, kSpanWaves * 4 / CH, n_span, t, sst);             \
        }                                                                                      \
        if (n_one > 0) {                                                                       \
            if (fused) {                                                                       \
                if (spk) DUS_BWD_LAUNCH(CH, true, true, 1, t.total_rays, t1, st);                     \
                else DUS_BWD_LAUNCH(CH, false, true, 1, t.total_rays, t1, st);                        \
            } else {                                                                           \
                if (spk) DUS_BWD_LAUNCH(CH, true, false, 1, t.total_rays, t1, st);                    \
                else DUS_BWD_LAUNCH(CH, false, false, 1, t.total_rays, t1, st);                       \
            }                                                                                  \
        }                                                                                      \
        break;

hipError_t launch_adjoint(int chunk, int xcd_group, const VolArgs &v, const PhysArgs &p,
                          const FanTable &t, const float *poses, RayRec *rays, const float *gsrc,
                          const float *target, float *zbar, double *pose_acc, double *pose_part, double *loss,
                          const double *carry, const int32_t *carry_exp, const double *cstate,
                          const float *gain, hipStream_t st, int span_samples, const SideStream *side)
{
    if (t.total_rays <= 0) return hipSuccess;
    if (pose_acc && !pose_part) return hipErrorInvalidValue;
    if (zbar && !rays) return hipErrorInvalidValue;
    if (chunk != 4 && chunk != 8) return hipErrorInvalidValue;
    const bool fused = (target != nullptr);
    const bool spk = p.speckle && !gain;      // recorded gains replace the speckle variates
    if (!carry) cstate = nullptr;             // chunk states are read in the frames of the carry records
    // several wavefronts per long ray need the forward's carry records and
    // chunk states (and its gains, when there is speckle)
    const int n_span = (carry && cstate && !spk) ? span_rays(t, span_samples) : 0;
    const int n_one = t.total_rays - n_span;
    FanTable t1 = t;
    t1.ray0 = n_span;
    hipStream_t sst = st;
    if (n_span > 0 && side) {
        hipError_t e = fork_side(st, *side);
        if (e != hipSuccess) return e;
        sst = side->st;
    }
    switch (chunk) {
        DUS_BWD_CASE(4)
        DUS_BWD_CASE(8)
    default:
        return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (sst != st) {
        // joined also after a failed launch: a capture must not end with a
        // fork left open, and the caller's stream must wait for the side's work
        const hipError_t ej = join_side(st, *side);
        if (e == hipSuccess) e = ej;
    }
    return e;
}

hipError_t launch_pose_reduce(const FanTable &t, const double *pose_part, double *pose_acc, hipStream_t st)
{
    if (t.n <= 0 || t.total_rays <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pose_reduce, dim3(t.n), dim3(64), 0, st, t, pose_part, pose_acc);
    return hipGetLastError();
}

hipError_t launch_scatter(int scatter_rays, int xcd_group, const VolArgs &v, const FanTable &t,
                          const RayRec *rays, const float *zbar, float *gZ, hipStream_t st,
                          unsigned long long *fix, const double *fscale, int wave_target)
{
    if (t.total_rays <= 0 || (!gZ && !fix)) return hipSuccess;
    if (!zbar || !rays || (fix && !fscale)) return hipErrorInvalidValue;
    // depth segments, the same power-of-two length for every fan, a whole
    // number of the largest groups (256 / RB depths): the shortest that
    // keeps the launch within wave_target wavefronts, about 32 per SIMD over
    // the launches that run at the same time (a wavefront's set-up is a few
    // loads, so short segments cost little and even out the finishing times;
    // a fan of long rays gets as many wavefronts per ray as its length asks
    // for)
    auto units = [&](int rb, int sg) {
        long long u = 0;
        for (int f = 0; f < t.n; ++f)
            u += (long long)((t.f[f].n_rays + rb - 1) / rb) * ((t.f[f].n_samples + sg - 1) / sg);
        return u;
    };
    // 0: automatic.  Eight rays per wavefront, unless even the shortest
    // segments leave fewer than two wavefronts per SIMD; then two
    if (scatter_rays == 0) scatter_rays = (units(8, 32) < 2048) ? 2 : 8;
    int seg = 256 / scatter_rays, seg_shift = 0;
    while (seg < DUS_MAX_SAMPLES && units(scatter_rays, seg) > std::max(wave_target, 1024)) seg *= 2;
    while ((1 << seg_shift) < seg) ++seg_shift;
    const long long nunits = units(scatter_rays, seg);
    if (nunits <= 0) return hipSuccess;
    if (nunits > INT32_MAX) return hipErrorInvalidValue;
    // fans of different lengths run faster segment by segment (a 2-D grid,
    // uneven 64-pose batch: 188 -> 178 us) unless most of that grid would be
    // empty blocks (a few very long fans: 1-D); equal fans run faster fan by
    // fan (bench step 144 -> 137 us)
    long long nrb_all = 0;
    int smax = 0;
    for (int f = 0; f < t.n; ++f) {
        nrb_all += (t.f[f].n_rays + scatter_rays - 1) / scatter_rays;
        smax = std::max(smax, t.f[f].n_samples);
    }
    const long long nseg_max = (smax + seg - 1) / seg;
    const long long grid2 = nrb_all * nseg_max;
    const bool two_d = grid2 > nunits && grid2 <= 2 * nunits;
    const dim3 grid = two_d ? dim3((unsigned)nrb_all, (unsigned)nseg_max) : dim3((unsigned)nunits);
    // each fan's first wavefront (along x for the 2-D grid)
    FanTable ts = t;
    long long u = 0;
    for (int f = 0; f < t.n; ++f) {
        ts.f[f].unit_begin = (int32_t)u;
        const long long nrb = (t.f[f].n_rays + scatter_rays - 1) / scatter_rays;
        u += two_d ? nrb : nrb * ((t.f[f].n_samples + seg - 1) / seg);
    }
    switch (scatter_rays) {
    case 2:
        hipLaunchKernelGGL((k_scatter<2>), grid, dim3(64), 0, st, v, ts, rays, zbar, gZ, seg_shift, xcd_group,
                           fix, fscale);
        break;
    case 4:
        hipLaunchKernelGGL((k_scatter<4>), grid, dim3(64), 0, st, v, ts, rays, zbar, gZ, seg_shift, xcd_group,
                           fix, fscale);
        break;
    case 8:
        hipLaunchKernelGGL((k_scatter<8>), grid, dim3(64), 0, st, v, ts, rays, zbar, gZ, seg_shift, xcd_group,
                           fix, fscale);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_backward(int chunk, int xcd_group, int scatter_rays, const VolArgs &v,
                           const PhysArgs &p, const FanTable &t, const float *poses, RayRec *rays,
                           const float *gsrc, const float *target, float *zbar, float *gZ,
                           double *pose_acc, double *pose_part, double *loss, const double *carry,
                           const int32_t *carry_exp, const double *cstate, const float *gain,
                           hipStream_t st)
{
    hipError_t e = launch_adjoint(chunk, xcd_group, v, p, t, poses, rays, gsrc, target, zbar, pose_acc, pose_part,
                                  loss, carry, carry_exp, cstate, gain, st);
    if (e != hipSuccess) return e;
    return launch_scatter(scatter_rays, xcd_group, v, t, rays, zbar, gZ, st);
}

#define DUS_BLUR_LAUNCH(MODE, TGT, IMG, LOSS)                                                       \
    do {                                                                                           \
        if (R <= 4)                                                                                \
            hipLaunchKernelGGL((k_blur<MODE, 4>), dim3(grid), dim3(256), 0, st, p, t, in, TGT, out, IMG, LOSS);  \
        else if (R <= 8)                                                                           \
            hipLaunchKernelGGL((k_blur<MODE, 8>), dim3(grid), dim3(256), 0, st, p, t, in, TGT, out, IMG, LOSS);  \
        else if (R <= 16)                                                                          \
            hipLaunchKernelGGL((k_blur<MODE, 16>), dim3(grid), dim3(256), 0, st, p, t, in, TGT, out, IMG, LOSS); \
        else                                                                                       \
            hipLaunchKernelGGL((k_blur<MODE, 32>), dim3(grid), dim3(256), 0, st, p, t, in, TGT, out, IMG, LOSS); \
    } while (0)

hipError_t launch_blur(bool transpose, const PhysArgs &p, const FanTable &t, const float *in,
                       float *out, hipStream_t st)
{
    const int grid = t.total_blur_blocks;
    if (grid <= 0) return hipSuccess;
    const int R = p.blur_rmax;
    if (R > DUS_MAX_BLUR_RADIUS) return hipErrorInvalidValue;
    if (transpose)
        DUS_BLUR_LAUNCH(1, nullptr, nullptr, nullptr);
    else
        DUS_BLUR_LAUNCH(0, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_blur_residual(const PhysArgs &p, const FanTable &t, const float *pre,
                                const float *target, float *image, float *resid, float *ebar,
                                double *loss, hipStream_t st)
{
    const int grid = t.total_blur_blocks;
    if (grid <= 0) return hipSuccess;
    const int R = p.blur_rmax;
    if (R > DUS_MAX_BLUR_RADIUS) return hipErrorInvalidValue;
    // radius up to 8: one pass, the residual kept in LDS
    if (R <= 4) {
        hipLaunchKernelGGL((k_blur_fused<4>), dim3(grid), dim3(256), 0, st, p, t, pre, target, ebar, image, loss);
        return hipGetLastError();
    }
    if (R <= 8) {
        hipLaunchKernelGGL((k_blur_fused<8>), dim3(grid), dim3(256), 0, st, p, t, pre, target, ebar, image, loss);
        return hipGetLastError();
    }
    if (!resid) return hipErrorInvalidValue;
    {
        const float *in = pre;
        float *out = resid;
        DUS_BLUR_LAUNCH(2, target, image, loss);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_blur(true, p, t, resid, ebar, st);
}

// --------------------------------------------------------------------------
// Static device scratch of the allocation-free entry points.  The array is
// part of the code object: every GPU that loads the library holds its own
// copy, at its own address, until the process ends.  In host code its name
// stands for the host-side shadow, not for device memory, so the device
// address is looked up once per device (with that device current) and only
// that address is handed to kernels.
// --------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void **ptr)
{
    *ptr = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_pose_finalize(const double *acc, const float *poses, int n_poses,
                                float *grad_pose, hipStream_t st)
{
    if (n_poses <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pose_finalize, dim3((n_poses + 63) / 64), dim3(64), 0, st, acc, poses,
                       n_poses, grad_pose);
    return hipGetLastError();
}

hipError_t launch_sample(int xcd_group, const VolArgs &v, const FanTable &t, const float *poses, float *out,
                         hipStream_t st)
{
    if (t.total_rays <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample_rays, dim3(t.total_rays), dim3(64), 0, st, v, t, poses, out, xcd_group);
    return hipGetLastError();
}

hipError_t launch_scan_convert(const float *img, int n_rays, int n_samples, double aperture, double r0,
                               double ds, int nx, int nz, double x0, double z0, double dx, double dz,
                               float fill, float *out, hipStream_t st)
{
    const long long n = (long long)nx * nz;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_convert, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, img, n_rays,
                       n_samples, aperture, r0, ds, nx, nz, x0, z0, dx, dz, fill, out);
    return hipGetLastError();
}

hipError_t launch_footprint(const VolArgs &v, const FanTable &t, const float *poses, uint8_t *mask,
                            hipStream_t st)
{
    if (t.total_rays <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_footprint, dim3(t.total_rays), dim3(64), 0, st, v, t, poses, mask);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double *ptr, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(n, 256)), dim3(256), 0, st, ptr, (long long)n);
    return hipGetLastError();
}

hipError_t launch_zero_f32(float *ptr, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f32, dim3(grid_for((n + 3) / 4, 256)), dim3(256), 0, st, ptr,
                       (long long)n);
    return hipGetLastError();
}

hipError_t launch_finish(const double *part, int64_t n_part, double *loss, const double *acc, const float *poses,
                         int n_poses, float *grad, hipStream_t st)
{
    const int pose_blocks = grad ? (n_poses + 255) / 256 : 0;
    const int grid = (loss ? 1 : 0) + pose_blocks;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finish, dim3(grid), dim3(256), 0, st, part, (long long)n_part, loss, acc, poses, n_poses,
                       grad);
    return hipGetLastError();
}

hipError_t launch_abs_rows(const FanTable &t, const float *zbar, double *part, hipStream_t st)
{
    if (t.total_rays <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_abs_rows, dim3((t.total_rays + 3) / 4), dim3(256), 0, st, t, zbar, part);
    return hipGetLastError();
}

hipError_t launch_fix_scale(const double *part, int64_t n, double *fscale, hipStream_t st)
{
    hipLaunchKernelGGL(k_fix_scale, dim3(1), dim3(256), 0, st, part, (long long)n, fscale);
    return hipGetLastError();
}

hipError_t launch_fix_to_f32(const unsigned long long *fix, int64_t n, const double *fscale, float *gZ,
                             bool overwrite, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fix_to_f32, dim3(grid_for((n + 3) / 4, 256)), dim3(256), 0, st, fix, (long long)n, fscale,
                       gZ, overwrite ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_zero_pair(float *a, int64_t na, double *b, int64_t nb, hipStream_t st)
{
    if (na <= 0 && nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_pair, dim3(grid_for(std::max<int64_t>((na + 3) / 4, nb), 256)), dim3(256), 0, st, a,
                       (long long)na, b, (long long)nb);
    return hipGetLastError();
}

hipError_t launch_sum_f64(const double *part, int64_t n, double *out, hipStream_t st, bool accumulate)
{
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, st, part, (long long)n, out, accumulate ? 1 : 0);
    return hipGetLastError();
}

int64_t smooth_blocks(int nx, int ny, int nz) { return ((int64_t)nx * ny * nz + 255) / 256; }

hipError_t launch_smooth(const float *Z, int nx, int ny, int nz, float wx, float wy, float wz, float *gZ,
                         double *part, hipStream_t st)
{
    const int64_t blocks = smooth_blocks(nx, ny, nz);
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_smooth, dim3((unsigned)blocks), dim3(256), 0, st, Z, nx, ny, nz, wx, wy, wz, gZ, part);
    return hipGetLastError();
}

hipError_t launch_adam(float *x, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, float lo, float hi, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n, 256)), dim3(256), 0, st, x, g, m, v, (long long)n, lr, b1, b2,
                       eps, c1, c2, lo, hi);
    return hipGetLastError();
}

hipError_t launch_map(const float *in, int64_t n, const LutArgs &lut, float *Z, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_map, dim3(grid_for((n + 3) / 4, 256)), dim3(256), 0, st, in, (long long)n, lut, Z);
    return hipGetLastError();
}

hipError_t launch_map_backward(const float *in, int64_t n, const LutArgs &lut, const float *gZ, float *grad_in,
                               double *grad_z, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    // at most 4096 blocks: one FP64 global atomic per knot and block
    int g = grid_for(n, 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_map_backward, dim3(g), dim3(256), 0, st, in, (long long)n, lut, gZ, grad_in, grad_z);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t *out,
                         hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const long long g = (n + 255) / 256;
    if (g > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)g), dim3(256), 0, st, ctr, (long long)n, k0, k1,
                       out);
    return hipGetLastError();
}

hipError_t launch_pixel_gain(const PhysArgs &p, const FanRec &f, float *out, hipStream_t st)
{
    if (f.n_rays <= 0 || f.n_samples <= 0) return hipSuccess;
    dim3 grid((f.n_samples + 255) / 256, f.n_rays);
    if (p.speckle)
        hipLaunchKernelGGL((k_gain<true>), grid, dim3(64), 0, st, p, f, out);
    else
        hipLaunchKernelGGL((k_gain<false>), grid, dim3(64), 0, st, p, f, out);
    return hipGetLastError();
}

}  // namespace dus
