/*
 * Runs the FP64 oracle's entry points on small seeded inputs (a volume with
 * samples inside and outside it, both reflection conventions, the three
 * attenuation modes, speckle and blur on and off, edge sizes S = 1, 2 and a
 * one-ray fan), built with -fsanitize=address,undefined: any out-of-bounds
 * access, leak or undefined operation in the oracle stops the run.
 */
#include "../../oracle/diffus_oracle.c"

#include <stdio.h>

static uint64_t lcg = 88172645463325252ull;

static double uni(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

int main(void)
{
    const int nx = 13, ny = 11, nz = 17;
    double *V = (double *)malloc(sizeof(double) * nx * ny * nz);
    for (int i = 0; i < nx * ny * nz; ++i) V[i] = 1.4 + 0.4 * uni();
    orc_volume vol = {V, nx, ny, nz, 0, {1.0, 0.9, 1.1}, {0.0, -0.5, 0.2}};
    double *G = (double *)calloc((size_t)nx * ny * nz, sizeof(double));
    const int shapes[][2] = {{5, 40}, {1, 33}, {3, 1}, {4, 2}, {2, 0}, {0, 7}};
    for (int sh = 0; sh < 6; ++sh)
        for (int refl = 0; refl < 2; ++refl)
            for (int att = 0; att < 3; ++att)
                for (int fx = 0; fx < 2; ++fx) {
                    orc_fan fan = {shapes[sh][0], shapes[sh][1], 1.2, 0.7, 0.5, 3, 0};
                    orc_physics ph;
                    memset(&ph, 0, sizeof(ph));
                    ph.alpha = 0.5;
                    ph.freq = 5.0;
                    ph.refl_mode = refl;
                    ph.atten_mode = att;
                    ph.speckle_on = fx;
                    ph.spk_cell = 8;
                    ph.Ar = 0.3;
                    ph.gam = 1.5;
                    ph.Ag0 = 0.2;
                    ph.Ag1 = 0.3;
                    ph.blur_on = fx;
                    ph.sigma0 = 0.5f;
                    ph.sigma1 = 2.5f;
                    ph.seed = 99;
                    /* apex outside the volume on one side: clamped samples */
                    const double pose[6] = {6.0, 4.0, -2.0, 0.1, -0.2, 0.3};
                    const int n = fan.n_rays * fan.n_samples;
                    double *img = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
                    double *raw = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
                    double *piv = (double *)malloc(sizeof(double) * (fan.n_rays > 0 ? fan.n_rays : 1));
                    double *g = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
                    for (int s = 0; s < 2; ++s)
                        if (orc_render(&vol, pose, &fan, &ph, s, img, raw, piv) != 0) return 1;
                    for (int i = 0; i < n; ++i) g[i] = uni() - 0.5;
                    double gp[6];
                    if (orc_backward(&vol, pose, &fan, &ph, g, G, gp) != 0) return 1;
                    if (orc_backward(&vol, pose, &fan, &ph, g, NULL, gp) != 0) return 1;
                    if (fan.n_rays > 0 && fan.n_samples > 0) {
                        double *m = (double *)malloc(sizeof(double) * fan.n_samples);
                        orc_speckle_ray(&fan, &ph, fan.n_rays - 1, m);
                        free(m);
                        orc_blur(&fan, &ph, img, raw);
                        orc_blur_T(&fan, &ph, img, raw);
                        double *sc = (double *)malloc(sizeof(double) * 9 * 7);
                        if (fan.n_rays >= 2 && fan.n_samples >= 2)
                            orc_scan_convert(img, fan.n_rays, fan.n_samples, fan.aperture, fan.r0, fan.ds, 9, 7,
                                             -10.0, -1.0, 2.5, 5.0, -1.0, sc);
                        free(sc);
                    }
                    free(img);
                    free(raw);
                    free(piv);
                    free(g);
                }
    /* per-ray pieces */
    double Zs[9], d0[9], e[9], mp;
    for (int i = 0; i < 9; ++i) Zs[i] = 1.3 + 6.5 * (i == 4) + 0.1 * uni();
    for (int mode = 0; mode < 2; ++mode) {
        orc_echo_banded(Zs, 9, 0.97, mode, d0, &mp);
        orc_echo_transfer(Zs, 9, 0.97, mode, e, d0, &mp);
    }
    double w[3] = {1e-6, 2e-6, -1e-6}, R[9], dR[27];
    orc_rotation(w, R);
    orc_rotation_grad(w, dR);
    w[0] = 2.0;
    orc_rotation(w, R);
    orc_rotation_grad(w, dR);
    const double u[3] = {-3.0, 5.5, 40.0};
    double gr[3], wt[8];
    int64_t idx[8];
    (void)orc_sample(&vol, u, gr, idx, wt);
    uint32_t ctr[8] = {0, 1, 2, 3, 0xffffffffu, 0, 7, 9}, key[2] = {5, 6}, out[8];
    orc_philox_batch(ctr, 2, key, out);
    (void)orc_rayleigh(0u);
    (void)orc_rayleigh(0xffffffffu);
    free(V);
    free(G);
    printf("oracle driver: ok\n");
    return 0;
}
