/*
 * diffus_oracle.c -- plain FP64 CPU oracle of the DiffUS fan-beam renderer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP kernels are
 * checked against.  Only tests/, __graft_entry__.smoke() and the cpu_baseline
 * leg of bench.py may load it.  It shares no code, header, table or helper
 * with the GPU library: every formula below is written out again from the
 * paper (arXiv 2508.06768, "DiffUS: Differentiable Ultrasound Rendering from
 * Volumetric Imaging").
 *
 * What it computes, in the paper's order:
 *   Sec. 2.1, Eq. 1       reflection / transmission coefficients of an interface
 *   Sec. 2.1 assumptions  straight rays, uniform attenuation
 *   Sec. 2.3, Eq. 2-4     the coupled forward/backward amplitude system A x = b
 *   Sec. 2.4              progressive solves at depths k = 1..N, echo d_0^(k),
 *                         pixel = first difference along depth, fan geometry,
 *                         multiplicative depth-dependent speckle, depth-dependent
 *                         lateral Gaussian blur
 * plus the exact derivative of all of it (the paper's stated purpose,
 * gradient-based registration and reconstruction, Sec. 1 / abstract).
 *
 * Readings of the paper where it is silent:
 *   - sampling: trilinear at a fixed step ds along each ray, clamp-to-edge
 *     outside the volume, voxel centres at integer index;
 *   - attenuation "in system": every interface step carries a one-way
 *     amplitude factor a = 10^(-alpha f ds_cm / 20) on the wave that crosses
 *     the step; "post hoc": Eq. 4 untouched and the pixel at depth s_k is
 *     multiplied by 10^(-2 alpha f (s_k - r0)_cm / 20);
 *   - the depth-k system uses samples Z_0..Z_k, terminated with d_k = 0;
 *   - pixel e_k = d_0^(k) - d_0^(k-1), e_0 = 0, raw and signed;
 *   - speckle: unit-mean Rayleigh multipliers drawn with Philox4x32-10
 *     (Salmon et al., SC'11) from a fixed counter, a radial term interpolated
 *     from cells along depth plus a granular per-pixel term;
 *   - blur: lateral (across rays) Gaussian per depth row, sigma linear in depth,
 *     radius ceil(3 sigma) decided in float32, edge replicate.
 *
 * Built with -ffp-contract=off so that the float32 decisions (blur radius)
 * are the plain IEEE operations written here.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Plain argument records (the oracle's own; ctypes mirrors them).          */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double *V;     /* impedance, [nz][ny][nx], x fastest, MRayl */
    int32_t nx, ny, nz;
    int32_t pad_;
    double h[3];         /* voxel spacing (mm) along x, y, z */
    double o[3];         /* world position (mm) of the centre of voxel (0,0,0) */
} orc_volume;

typedef struct {
    int32_t n_rays, n_samples;
    double aperture;     /* full fan angle (rad) */
    double ds;           /* depth step along a ray (mm) */
    double r0;           /* distance of the first sample from the apex (mm) */
    int32_t speckle_id;  /* stream id of this fan in the speckle counter */
    int32_t pad_;
} orc_fan;

typedef struct {
    double alpha;        /* dB / cm / MHz */
    double freq;         /* MHz */
    int32_t refl_mode;   /* 0: |.| as printed in Eq. 1;  1: signed coefficient */
    int32_t atten_mode;  /* 0: in the system;  1: post hoc;  2: off */
    int32_t speckle_on;
    int32_t spk_cell;    /* radial cell length in samples */
    double Ar, gam, Ag0, Ag1;
    int32_t blur_on;
    float sigma0, sigma1;    /* blur width at first / last depth, in rays */
    int32_t pad_;
    uint64_t seed;
} orc_physics;

/* ------------------------------------------------------------------------ */
/* Rotation of the probe: rotation vector w, R = exp([w]x) (Rodrigues).     */
/* The fan is shot "from the virtual transducer position" (Sec. 2.4); the   */
/* pose maps probe coordinates q to world p = t + R q.                      */
/* ------------------------------------------------------------------------ */
static void skew(const double w[3], double W[9])
{
    W[0] = 0.0;   W[1] = -w[2]; W[2] = w[1];
    W[3] = w[2];  W[4] = 0.0;   W[5] = -w[0];
    W[6] = -w[1]; W[7] = w[0];  W[8] = 0.0;
}

static void matmul3(const double A[9], const double B[9], double C[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

void orc_rotation(const double w[3], double R[9])
{
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2);
    double A, B;
    if (th < 1e-4) {            /* Taylor series of sin(t)/t and (1-cos t)/t^2 */
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
    }
    double W[9], W2[9];
    skew(w, W);
    matmul3(W, W, W2);
    for (int i = 0; i < 9; ++i) R[i] = A * W[i] + B * W2[i];
    R[0] += 1.0; R[4] += 1.0; R[8] += 1.0;
}

/* dR/dw_c for c = 0,1,2, stored dR[9*c + 3*a + b].  Closed form of Gallego
 * and Yezzi (J. Math. Imaging Vis. 2015):
 *   dR/dw_c = (w_c [w]x + [w x ((I - R) e_c)]x) R / |w|^2,
 * and its first-order expansion E_c + (E_c W + W E_c)/2 near w = 0. */
void orc_rotation_grad(const double w[3], double dR[27])
{
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double W[9];
    skew(w, W);
    if (th2 < 1e-10) {
        for (int c = 0; c < 3; ++c) {
            double e[3] = {0, 0, 0}, E[9], EW[9], WE[9];
            e[c] = 1.0;
            skew(e, E);
            matmul3(E, W, EW);
            matmul3(W, E, WE);
            for (int i = 0; i < 9; ++i) dR[9 * c + i] = E[i] + 0.5 * (EW[i] + WE[i]);
        }
        return;
    }
    double R[9];
    orc_rotation(w, R);
    for (int c = 0; c < 3; ++c) {
        double v[3];                       /* (I - R) e_c */
        for (int a = 0; a < 3; ++a) v[a] = (a == c ? 1.0 : 0.0) - R[3 * a + c];
        double x[3] = {w[1] * v[2] - w[2] * v[1],
                       w[2] * v[0] - w[0] * v[2],
                       w[0] * v[1] - w[1] * v[0]};
        double X[9], S[9], out[9];
        skew(x, X);
        for (int i = 0; i < 9; ++i) S[i] = (w[c] * W[i] + X[i]) / th2;
        matmul3(S, R, out);
        memcpy(dR + 9 * c, out, sizeof(out));
    }
}

/* ------------------------------------------------------------------------ */
/* Trilinear sample of Z at voxel coordinate u (clamp-to-edge), with its     */
/* derivative dZ/du (zero along an axis where u lies outside the volume).    */
/* "Each acoustic beam traverses a linear sequence of voxels" (Sec. 2.3).    */
/* ------------------------------------------------------------------------ */
static void axis_cell(double u, int n, int *i0, double *f, int *inside)
{
    double uc = u;
    *inside = (u >= 0.0 && u <= (double)(n - 1));
    if (uc < 0.0) uc = 0.0;
    if (uc > (double)(n - 1)) uc = (double)(n - 1);
    int i = (int)floor(uc);
    if (i > n - 2) i = n - 2;
    *i0 = i;
    *f = uc - (double)i;
}

static double lerp(double a, double b, double t) { return a + t * (b - a); }

/* returns Z(u); grad (nullable) receives dZ/du; idx/wt (nullable) receive
 * the 8 corner indices and their trilinear weights */
double orc_sample(const orc_volume *vol, const double u[3], double grad[3],
                  int64_t idx[8], double wt[8])
{
    int x0, y0, z0, inx, iny, inz;
    double fx, fy, fz;
    axis_cell(u[0], vol->nx, &x0, &fx, &inx);
    axis_cell(u[1], vol->ny, &y0, &fy, &iny);
    axis_cell(u[2], vol->nz, &z0, &fz, &inz);
    const int64_t sx = 1, sy = vol->nx, sz = (int64_t)vol->nx * vol->ny;
    const int64_t b = (int64_t)z0 * sz + (int64_t)y0 * sy + x0;
    const double *V = vol->V;
    double c000 = V[b], c100 = V[b + sx];
    double c010 = V[b + sy], c110 = V[b + sy + sx];
    double c001 = V[b + sz], c101 = V[b + sz + sx];
    double c011 = V[b + sz + sy], c111 = V[b + sz + sy + sx];
    /* lerp along x, then y, then z */
    double a00 = lerp(c000, c100, fx), a10 = lerp(c010, c110, fx);
    double a01 = lerp(c001, c101, fx), a11 = lerp(c011, c111, fx);
    double b0 = lerp(a00, a10, fy), b1 = lerp(a01, a11, fy);
    double z = lerp(b0, b1, fz);
    if (grad) {
        double dx00 = c100 - c000, dx10 = c110 - c010, dx01 = c101 - c001, dx11 = c111 - c011;
        double gx = lerp(lerp(dx00, dx10, fy), lerp(dx01, dx11, fy), fz);
        double gy = lerp(a10 - a00, a11 - a01, fz);
        double gz = b1 - b0;
        grad[0] = inx ? gx : 0.0;
        grad[1] = iny ? gy : 0.0;
        grad[2] = inz ? gz : 0.0;
    }
    if (idx) {
        for (int c = 0; c < 8; ++c) {
            int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
            idx[c] = b + cz * sz + cy * sy + cx * sx;
            wt[c] = (cx ? fx : 1.0 - fx) * (cy ? fy : 1.0 - fy) * (cz ? fz : 1.0 - fz);
        }
    }
    return z;
}

/* ------------------------------------------------------------------------ */
/* Fan geometry (Sec. 2.4): ray j of n_rays leaves the apex at angle        */
/* theta_j = -A/2 + j A/(n_rays-1) in the probe x-z plane, beam along +z.   */
/* Sample k sits at distance s_k = r0 + k ds.                              */
/* ------------------------------------------------------------------------ */
static void ray_dir(const orc_fan *fan, int j, double dir[3])
{
    double th = 0.0;
    if (fan->n_rays > 1)
        th = -0.5 * fan->aperture + (double)j * fan->aperture / (double)(fan->n_rays - 1);
    dir[0] = sin(th);
    dir[1] = 0.0;
    dir[2] = cos(th);
}

/* Z along ray j, optionally dZ/dp (world, per mm) and the probe-frame points */
void orc_ray_samples(const orc_volume *vol, const double pose[6], const orc_fan *fan, int j,
                     double *Zs, double *gradp, double *q)
{
    double R[9], dir[3];
    orc_rotation(pose + 3, R);
    ray_dir(fan, j, dir);
    for (int k = 0; k < fan->n_samples; ++k) {
        double s = fan->r0 + (double)k * fan->ds;
        double qk[3] = {s * dir[0], s * dir[1], s * dir[2]};
        double u[3], g[3];
        for (int a = 0; a < 3; ++a) {
            double p = pose[a] + R[3 * a] * qk[0] + R[3 * a + 1] * qk[1] + R[3 * a + 2] * qk[2];
            u[a] = (p - vol->o[a]) / vol->h[a];
        }
        Zs[k] = orc_sample(vol, u, gradp ? g : NULL, NULL, NULL);
        if (gradp)
            for (int a = 0; a < 3; ++a) gradp[3 * k + a] = g[a] / vol->h[a];
        if (q)
            for (int a = 0; a < 3; ++a) q[3 * k + a] = qk[a];
    }
}

/* ------------------------------------------------------------------------ */
/* Eq. 1: coefficients of the interface between sample i (Z1) and i+1 (Z2). */
/*   R_{1->2} = |Z2-Z1|/(Z1+Z2),  T_{1->2} = 2 Z2/(Z1+Z2)                   */
/*   R_{2->1} = |Z1-Z2|/(Z1+Z2),  T_{2->1} = 2 Z1/(Z1+Z2)                   */
/* refl_mode 1 drops the |.| (the signed pressure coefficient).             */
/* ------------------------------------------------------------------------ */
typedef struct { double R, Rb, T, Tb; } iface;   /* R_{i->i+1}, R_{i+1->i}, T_{i->i+1}, T_{i+1->i} */

static iface coeffs(double Z1, double Z2, int mode)
{
    iface c;
    double s = Z1 + Z2;
    if (mode == 0) {
        c.R = fabs(Z2 - Z1) / s;
        c.Rb = fabs(Z1 - Z2) / s;
    } else {
        c.R = (Z2 - Z1) / s;
        c.Rb = (Z1 - Z2) / s;
    }
    c.T = 2.0 * Z2 / s;
    c.Tb = 2.0 * Z1 / s;
    return c;
}

void orc_coeffs(double Z1, double Z2, int mode, double out[4])
{
    iface c = coeffs(Z1, Z2, mode);
    out[0] = c.R; out[1] = c.Rb; out[2] = c.T; out[3] = c.Tb;
}

/* one-way amplitude factor over one depth step (attenuation in the system) */
double orc_step_amplitude(const orc_physics *ph, double ds_mm)
{
    if (ph->atten_mode != 0) return 1.0;
    return pow(10.0, -ph->alpha * ph->freq * (ds_mm / 10.0) / 20.0);
}

/* ------------------------------------------------------------------------ */
/* Progressive solve, Sec. 2.4, literal O(S^2) form: for every truncation   */
/* depth k the system of Eq. 2-4 over samples 0..k with g_0 = 1, d_k = 0 is  */
/* solved by banded back-substitution of the reflectance Gamma_i = d_i/g_i:  */
/*   Gamma_k = 0,                                                           */
/*   g_{i+1} = a T_{i->i+1} g_i + a^2 R_{i+1->i} d_{i+1}                    */
/*   d_i     = R_{i->i+1} g_i + a T_{i+1->i} d_{i+1}                        */
/*   => Gamma_i = R_i + a^2 T_i T'_i Gamma_{i+1} / (1 - a^2 R'_i Gamma_{i+1})*/
/* and d_0^(k) = Gamma_0 (g_0 = 1).  d0[0] = 0 (no interface yet).          */
/* Returns the smallest |pivot| met over all k (nullable).                  */
/* ------------------------------------------------------------------------ */
void orc_echo_banded(const double *Zs, int S, double a, int mode, double *d0, double *min_pivot)
{
    double a2 = a * a, mp = INFINITY;
    if (S > 0) d0[0] = 0.0;
    for (int k = 1; k < S; ++k) {
        double G = 0.0;
        for (int i = k - 1; i >= 0; --i) {
            iface c = coeffs(Zs[i], Zs[i + 1], mode);
            double piv = 1.0 - a2 * c.Rb * G;
            if (fabs(piv) < mp) mp = fabs(piv);
            G = c.R + a2 * c.T * c.Tb * G / piv;
        }
        d0[k] = G;
    }
    if (min_pivot) *min_pivot = mp;
}

/* ------------------------------------------------------------------------ */
/* Same echoes in O(S): composing the Moebius maps of the back-substitution  */
/* above.  Gamma_i = (m00 Gamma_{i+1} + m01) / (m10 Gamma_{i+1} + m11) with  */
/*   M_i = [[a^2 (T T' - R R'), R], [-a^2 R', 1]],                           */
/* so with P_0 = I, P_{k+1} = P_k M_k the depth-k echo is                    */
/*   d_0^(k) = P_k[0][1] / P_k[1][1].                                        */
/* e (nullable) receives the first differences; d0 (nullable) the echoes.    */
/* min_pivot receives min_k |P_{k+1}[1][1] / P_k[1][1]|: the pivots of the   */
/* top-down elimination of the same banded systems.                         */
/* ------------------------------------------------------------------------ */
void orc_echo_transfer(const double *Zs, int S, double a, int mode,
                       double *e, double *d0, double *min_pivot)
{
    double a2 = a * a, mp = INFINITY;
    double P00 = 1.0, P01 = 0.0, P10 = 0.0, P11 = 1.0, prev = 0.0;
    if (S > 0) {
        if (e) e[0] = 0.0;
        if (d0) d0[0] = 0.0;
    }
    for (int k = 0; k + 1 < S; ++k) {
        iface c = coeffs(Zs[k], Zs[k + 1], mode);
        double m00 = a2 * (c.T * c.Tb - c.R * c.Rb), m01 = c.R, m10 = -a2 * c.Rb, m11 = 1.0;
        double n00 = P00 * m00 + P01 * m10, n01 = P00 * m01 + P01 * m11;
        double n10 = P10 * m00 + P11 * m10, n11 = P10 * m01 + P11 * m11;
        double piv = fabs(n11 / P11);
        if (piv < mp) mp = piv;
        P00 = n00; P01 = n01; P10 = n10; P11 = n11;
        double G = P01 / P11;
        if (d0) d0[k + 1] = G;
        if (e) e[k + 1] = G - prev;
        prev = G;
    }
    if (min_pivot) *min_pivot = mp;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,       */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Ten rounds of    */
/* the multiply-xor bijection with multipliers 0xD2511F53 and 0xCD9E8D57,   */
/* key bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85.              */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
    memcpy(out, c, sizeof(c));
}

void orc_philox_batch(const uint32_t *ctrs, int64_t n, const uint32_t key[2], uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctrs + 4 * i, key, out + 4 * i);
}

/* unit-mean Rayleigh variate from a 32-bit word: u in (0,1] from the top 24
 * bits, xi = sqrt(-2 ln u) / sqrt(pi/2) */
static double rayleigh(uint32_t x)
{
    double u = ((double)(x >> 8) + 1.0) * (1.0 / 16777216.0);
    return sqrt(-2.0 * log(u)) * sqrt(2.0 / M_PI);
}

/* the same map, exported for its pins */
double orc_rayleigh(uint32_t x) { return rayleigh(x); }

static uint32_t philox_word(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed, int w)
{
    uint32_t ctr[4] = {c0, c1, c2, c3}, key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)}, out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[w];
}

/* Speckle multiplier of ray j (Sec. 2.4): multiplicative, depth dependent,
 *   m_k = 1 + Ar zeta^gam (xi_r - 1) + (Ag0 + Ag1 zeta)(xi_g - 1),
 * zeta = k/(S-1); xi_g granular per pixel from counter (k>>2, j, id, 0)
 * word k&3; xi_r radial, linear between cell values taken every spk_cell
 * samples from counter (c>>2, j, id, 1) word c&3. */
void orc_speckle_ray(const orc_fan *fan, const orc_physics *ph, int j, double *m)
{
    int S = fan->n_samples;
    uint32_t id = (uint32_t)fan->speckle_id;
    for (int k = 0; k < S; ++k) {
        double zeta = S > 1 ? (double)k / (double)(S - 1) : 0.0;
        double xg = rayleigh(philox_word((uint32_t)k >> 2, (uint32_t)j, id, 0u, ph->seed, k & 3));
        int cell = ph->spk_cell;
        int c0 = k / cell;
        double fr = (double)(k - c0 * cell) / (double)cell;
        double r0 = rayleigh(philox_word((uint32_t)c0 >> 2, (uint32_t)j, id, 1u, ph->seed, c0 & 3));
        double r1 = rayleigh(philox_word((uint32_t)(c0 + 1) >> 2, (uint32_t)j, id, 1u, ph->seed, (c0 + 1) & 3));
        double xr = (1.0 - fr) * r0 + fr * r1;
        m[k] = 1.0 + ph->Ar * pow(zeta, ph->gam) * (xr - 1.0) + (ph->Ag0 + ph->Ag1 * zeta) * (xg - 1.0);
    }
}

/* per-pixel multiplier applied to the raw echo: post-hoc attenuation and
 * speckle (both optional) */
static void pixel_gain(const orc_fan *fan, const orc_physics *ph, int j, double *gain)
{
    int S = fan->n_samples;
    for (int k = 0; k < S; ++k) gain[k] = 1.0;
    if (ph->atten_mode == 1)
        for (int k = 0; k < S; ++k)
            gain[k] = pow(10.0, -2.0 * ph->alpha * ph->freq * ((double)k * fan->ds / 10.0) / 20.0);
    if (ph->speckle_on) {
        double *m = (double *)malloc(sizeof(double) * (size_t)(S > 0 ? S : 1));
        orc_speckle_ray(fan, ph, j, m);
        for (int k = 0; k < S; ++k) gain[k] *= m[k];
        free(m);
    }
}

/* ------------------------------------------------------------------------ */
/* Depth-dependent lateral blur (Sec. 2.4): at depth row k a normalised      */
/* Gaussian along the ray index with sigma_k = s0 + (s1 - s0) k/(S-1) rays,  */
/* radius ceil(3 sigma_k); sigma and radius are decided in float32; edge     */
/* replicate; sigma below 1e-3 leaves the row unchanged.                     */
/* ------------------------------------------------------------------------ */
static int blur_row(const orc_physics *ph, int S, int k, double *w /* [2*r+1] */, int maxr)
{
    float frac = S > 1 ? (float)k / (float)(S - 1) : 0.0f;
    float d = ph->sigma1 - ph->sigma0;
    float md = d * frac;
    float sig = ph->sigma0 + md;
    if (!(sig >= 1e-3f)) return -1;
    float r3 = 3.0f * sig;
    int r = (int)ceilf(r3);
    if (r > maxr) r = maxr;
    double sd = (double)sig, tot = 0.0;
    for (int t = -r; t <= r; ++t) {
        w[t + r] = exp(-(double)(t * t) / (2.0 * sd * sd));
        tot += w[t + r];
    }
    for (int t = -r; t <= r; ++t) w[t + r] /= tot;
    return r;
}

#define ORC_MAXR 64

void orc_blur(const orc_fan *fan, const orc_physics *ph, const double *in, double *out)
{
    int n = fan->n_rays, S = fan->n_samples;
    double w[2 * ORC_MAXR + 1];
    for (int k = 0; k < S; ++k) {
        int r = blur_row(ph, S, k, w, ORC_MAXR);
        for (int j = 0; j < n; ++j) {
            if (r < 0) { out[(int64_t)j * S + k] = in[(int64_t)j * S + k]; continue; }
            double acc = 0.0;
            for (int t = -r; t <= r; ++t) {
                int jj = j + t;
                if (jj < 0) jj = 0;
                if (jj > n - 1) jj = n - 1;
                acc += w[t + r] * in[(int64_t)jj * S + k];
            }
            out[(int64_t)j * S + k] = acc;
        }
    }
}

/* transpose of orc_blur: out = B^T in */
void orc_blur_T(const orc_fan *fan, const orc_physics *ph, const double *in, double *out)
{
    int n = fan->n_rays, S = fan->n_samples;
    double w[2 * ORC_MAXR + 1];
    for (int64_t i = 0; i < (int64_t)n * S; ++i) out[i] = 0.0;
    for (int k = 0; k < S; ++k) {
        int r = blur_row(ph, S, k, w, ORC_MAXR);
        for (int j = 0; j < n; ++j) {
            double g = in[(int64_t)j * S + k];
            if (r < 0) { out[(int64_t)j * S + k] += g; continue; }
            for (int t = -r; t <= r; ++t) {
                int jj = j + t;
                if (jj < 0) jj = 0;
                if (jj > n - 1) jj = n - 1;
                out[(int64_t)jj * S + k] += w[t + r] * g;
            }
        }
    }
}

/* radius of depth row k as decided in float32 (-1: identity row) */
int orc_blur_radius(const orc_physics *ph, int S, int k)
{
    double w[2 * ORC_MAXR + 1];
    return blur_row(ph, S, k, w, ORC_MAXR);
}

/* ------------------------------------------------------------------------ */
/* Display: scan conversion of one fan's polar image (rows = rays at angles */
/* -A/2 .. A/2, columns = depths r0 + k ds) onto a Cartesian grid of the    */
/* probe's x-z plane, as in the fan images of Fig. 3.  Pixel (iz, ix) sits  */
/* at x = x0 + ix dx, z = z0 + iz dz; its polar indices are                 */
/*   j = (atan2(x, z) + A/2)(n_r - 1)/A,   k = (|(x, z)| - r0)/ds,          */
/* and its value is the bilinear interpolation of the image (along depth,   */
/* then along the rays) inside 0 <= j <= n_r-1, 0 <= k <= S-1, else fill.   */
/* ------------------------------------------------------------------------ */
void orc_scan_convert(const double *img, int n_r, int S, double A, double r0, double ds,
                      int nx, int nz, double x0, double z0, double dx, double dz, double fill,
                      double *out)
{
    for (int iz = 0; iz < nz; ++iz)
        for (int ix = 0; ix < nx; ++ix) {
            const double x = x0 + ix * dx, z = z0 + iz * dz;
            const double r = sqrt(x * x + z * z), th = atan2(x, z);
            const double j = (th + 0.5 * A) * (n_r - 1) / A, k = (r - r0) / ds;
            double v = fill;
            if (j >= 0.0 && j <= n_r - 1 && k >= 0.0 && k <= S - 1) {
                int j0 = (int)floor(j), k0 = (int)floor(k);
                if (j0 > n_r - 2) j0 = n_r - 2;
                if (k0 > S - 2) k0 = S - 2;
                const double fj = j - j0, fk = k - k0;
                const double *p0 = img + (size_t)j0 * S + k0, *p1 = p0 + S;
                const double a = p0[0] + fk * (p0[1] - p0[0]);
                const double b = p1[0] + fk * (p1[1] - p1[0]);
                v = a + fj * (b - a);
            }
            out[(size_t)iz * nx + ix] = v;
        }
}

/* ------------------------------------------------------------------------ */
/* Whole fan: raw echoes, gains, blur.                                      */
/*   solver 0: O(S) transfer form;  1: literal O(S^2) progressive solve.     */
/* img [n_rays][S]; raw (nullable) receives the pre-effect echoes e;         */
/* min_pivot (nullable) per ray.  Returns 0 on success.                      */
/* ------------------------------------------------------------------------ */
int orc_render(const orc_volume *vol, const double pose[6], const orc_fan *fan,
               const orc_physics *ph, int solver, double *img, double *raw, double *min_pivot)
{
    int n = fan->n_rays, S = fan->n_samples;
    if (n <= 0 || S <= 0) return 0;
    double a = orc_step_amplitude(ph, fan->ds);
    double *pre = (double *)malloc(sizeof(double) * (size_t)n * S);
    if (!pre) return -1;
    int err = 0;
#pragma omp parallel
    {
        double *Zs = (double *)malloc(sizeof(double) * S);
        double *d0 = (double *)malloc(sizeof(double) * S);
        double *gain = (double *)malloc(sizeof(double) * S);
#pragma omp for schedule(dynamic)
        for (int j = 0; j < n; ++j) {
            double *e = pre + (int64_t)j * S;
            double mp;
            orc_ray_samples(vol, pose, fan, j, Zs, NULL, NULL);
            if (solver == 1) {
                orc_echo_banded(Zs, S, a, ph->refl_mode, d0, NULL);
                orc_echo_transfer(Zs, S, a, ph->refl_mode, NULL, NULL, &mp);
                e[0] = 0.0;
                for (int k = 1; k < S; ++k) e[k] = d0[k] - d0[k - 1];
            } else {
                orc_echo_transfer(Zs, S, a, ph->refl_mode, e, NULL, &mp);
            }
            if (min_pivot) min_pivot[j] = mp;
            if (raw) memcpy(raw + (int64_t)j * S, e, sizeof(double) * S);
            pixel_gain(fan, ph, j, gain);
            for (int k = 0; k < S; ++k) e[k] *= gain[k];
        }
        free(Zs); free(d0); free(gain);
    }
    if (ph->blur_on)
        orc_blur(fan, ph, pre, img);
    else
        memcpy(img, pre, sizeof(double) * (size_t)n * S);
    free(pre);
    return err;
}

/* ------------------------------------------------------------------------ */
/* Exact derivative of orc_render (transfer form) for a given dL/dimg.       */
/* Reverse mode, written out in the order of the forward:                   */
/*   img = blur(gain * e),  e_k = G_k - G_{k-1},  G_k = P_k[0][1]/P_k[1][1], */
/*   P_{k+1} = P_k M_k(R, R', T, T'),  coefficients(Z_k, Z_{k+1}) per Eq. 1, */
/*   Z_k = trilinear(V, (t + R(w) q_k - o)/h).                              */
/* grad_V (nullable) is accumulated (+=); grad_pose (nullable) receives      */
/* dL/d(t_x, t_y, t_z, w_x, w_y, w_z).                                       */
/* ------------------------------------------------------------------------ */
int orc_backward(const orc_volume *vol, const double pose[6], const orc_fan *fan,
                 const orc_physics *ph, const double *grad_img, double *grad_V, double *grad_pose)
{
    int n = fan->n_rays, S = fan->n_samples;
    double gt[3] = {0, 0, 0}, GR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (grad_pose) for (int i = 0; i < 6; ++i) grad_pose[i] = 0.0;
    if (n <= 0 || S <= 0) return 0;
    double a = orc_step_amplitude(ph, fan->ds), a2 = a * a;
    double *ebar_all = (double *)malloc(sizeof(double) * (size_t)n * S);
    if (ph->blur_on)
        orc_blur_T(fan, ph, grad_img, ebar_all);
    else
        memcpy(ebar_all, grad_img, sizeof(double) * (size_t)n * S);
#pragma omp parallel
    {
        double *Zs = (double *)malloc(sizeof(double) * S);
        double *gp = (double *)malloc(sizeof(double) * 3 * S);
        double *q = (double *)malloc(sizeof(double) * 3 * S);
        double *gain = (double *)malloc(sizeof(double) * S);
        double *P = (double *)malloc(sizeof(double) * 4 * S);
        double *Zbar = (double *)malloc(sizeof(double) * S);
        double lgt[3] = {0, 0, 0}, lGR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma omp for schedule(dynamic)
        for (int j = 0; j < n; ++j) {
            double *eb = ebar_all + (int64_t)j * S;
            orc_ray_samples(vol, pose, fan, j, Zs, gp, q);
            pixel_gain(fan, ph, j, gain);
            /* forward: all prefix products */
            P[0] = 1.0; P[1] = 0.0; P[2] = 0.0; P[3] = 1.0;
            for (int k = 0; k + 1 < S; ++k) {
                iface c = coeffs(Zs[k], Zs[k + 1], ph->refl_mode);
                double m00 = a2 * (c.T * c.Tb - c.R * c.Rb), m01 = c.R, m10 = -a2 * c.Rb, m11 = 1.0;
                const double *p = P + 4 * k;
                double *o = P + 4 * (k + 1);
                o[0] = p[0] * m00 + p[1] * m10; o[1] = p[0] * m01 + p[1] * m11;
                o[2] = p[2] * m00 + p[3] * m10; o[3] = p[2] * m01 + p[3] * m11;
            }
            for (int k = 0; k < S; ++k) Zbar[k] = 0.0;
            /* reverse */
            double B00 = 0, B01 = 0, B10 = 0, B11 = 0;   /* dL/dP_k */
            for (int k = S - 1; k >= 1; --k) {
                double ebk = eb[k] * gain[k];
                double ebk1 = (k + 1 < S) ? eb[k + 1] * gain[k + 1] : 0.0;
                double Gbar = ebk - ebk1;                  /* e_k = G_k - G_{k-1} */
                const double *p = P + 4 * k;
                double G = p[1] / p[3];
                B01 += Gbar / p[3];
                B11 += -Gbar * G / p[3];
                /* P_k = P_{k-1} M_{k-1} */
                const double *pm = P + 4 * (k - 1);
                iface c = coeffs(Zs[k - 1], Zs[k], ph->refl_mode);
                double m00 = a2 * (c.T * c.Tb - c.R * c.Rb), m01 = c.R, m10 = -a2 * c.Rb, m11 = 1.0;
                /* Mbar = P_{k-1}^T Pbar */
                double M00 = pm[0] * B00 + pm[2] * B10;
                double M01 = pm[0] * B01 + pm[2] * B11;
                double M10 = pm[1] * B00 + pm[3] * B10;
                /* Pbar_{k-1} = Pbar M^T */
                double n00 = B00 * m00 + B01 * m01, n01 = B00 * m10 + B01 * m11;
                double n10 = B10 * m00 + B11 * m01, n11 = B10 * m10 + B11 * m11;
                B00 = n00; B01 = n01; B10 = n10; B11 = n11;
                /* coefficient adjoints */
                double Rbar = M00 * (-a2 * c.Rb) + M01;
                double Rbbar = M00 * (-a2 * c.R) + M10 * (-a2);
                double Tbar = M00 * a2 * c.Tb;
                double Tbbar = M00 * a2 * c.T;
                double Z1 = Zs[k - 1], Z2 = Zs[k], s = Z1 + Z2, s2 = s * s, d = Z2 - Z1;
                double dR1, dR2, dRb1, dRb2;
                if (ph->refl_mode == 0) {
                    double sg = (d > 0) ? 1.0 : ((d < 0) ? -1.0 : 0.0);
                    dR1 = (-sg * s - fabs(d)) / s2;
                    dR2 = (sg * s - fabs(d)) / s2;
                    dRb1 = dR1; dRb2 = dR2;          /* |Z1-Z2| = |Z2-Z1| */
                } else {
                    dR1 = -2.0 * Z2 / s2; dR2 = 2.0 * Z1 / s2;
                    dRb1 = -dR1; dRb2 = -dR2;
                }
                double dT1 = -2.0 * Z2 / s2, dT2 = 2.0 * Z1 / s2;
                double dTb1 = 2.0 * Z2 / s2, dTb2 = -2.0 * Z1 / s2;
                Zbar[k - 1] += Rbar * dR1 + Rbbar * dRb1 + Tbar * dT1 + Tbbar * dTb1;
                Zbar[k] += Rbar * dR2 + Rbbar * dRb2 + Tbar * dT2 + Tbbar * dTb2;
            }
            /* Z_k = trilinear(V, u_k) */
            double R[9], dir[3];
            orc_rotation(pose + 3, R);
            ray_dir(fan, j, dir);
            for (int k = 0; k < S; ++k) {
                double zb = Zbar[k];
                if (zb == 0.0) continue;
                if (grad_V) {
                    double u[3];
                    for (int ax = 0; ax < 3; ++ax) {
                        double p = pose[ax] + R[3 * ax] * q[3 * k] + R[3 * ax + 1] * q[3 * k + 1] +
                                   R[3 * ax + 2] * q[3 * k + 2];
                        u[ax] = (p - vol->o[ax]) / vol->h[ax];
                    }
                    int64_t idx[8];
                    double wt[8];
                    orc_sample(vol, u, NULL, idx, wt);
                    for (int c = 0; c < 8; ++c) {
#pragma omp atomic
                        grad_V[idx[c]] += zb * wt[c];
                    }
                }
                for (int ax = 0; ax < 3; ++ax) {
                    double g = zb * gp[3 * k + ax];
                    lgt[ax] += g;
                    for (int b = 0; b < 3; ++b) lGR[3 * ax + b] += g * q[3 * k + b];
                }
            }
        }
#pragma omp critical
        {
            for (int i = 0; i < 3; ++i) gt[i] += lgt[i];
            for (int i = 0; i < 9; ++i) GR[i] += lGR[i];
        }
        free(Zs); free(gp); free(q); free(gain); free(P); free(Zbar);
    }
    free(ebar_all);
    if (grad_pose) {
        double dR[27];
        orc_rotation_grad(pose + 3, dR);
        for (int i = 0; i < 3; ++i) grad_pose[i] = gt[i];
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int i = 0; i < 9; ++i) s += GR[i] * dR[9 * c + i];
            grad_pose[3 + c] = s;
        }
    }
    return 0;
}

/* Threads the parallel loops above run on (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the thread count of the parallel loops (no effect without OpenMP). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
