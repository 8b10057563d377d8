/* The oracle (oracle/xro.c) built with AddressSanitizer and
 * UndefinedBehaviorSanitizer and driven through every entry point on small
 * shots: off-axis sources, two domains, two spindle steps, sub-pixels,
 * layers, a table that some terms miss (F_default), both lattice shapes, and
 * the gradient.  Memory errors or undefined behaviour abort the run; the
 * values are checked to be finite and, for fluence x 2, exactly doubled. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/xro.h"

#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            exit(1);                                                             \
        }                                                                        \
    } while (0)

int main(void)
{
    static double F[5 * 6 * 7];
    for (int i = 0; i < 5 * 6 * 7; ++i) F[i] = 1.0 + (double)((i * 37) % 11);
    const double dir[2][3] = {{0.0, 0.0, 1.0}, {0.001, -0.002, 0.9999975}};
    double d1 = sqrt(dir[1][0] * dir[1][0] + dir[1][1] * dir[1][1] + dir[1][2] * dir[1][2]);
    double src_dir[6] = {dir[0][0], dir[0][1], dir[0][2], dir[1][0] / d1, dir[1][1] / d1, dir[1][2] / d1};
    double lam[2] = {1.3, 1.31}, w[2] = {0.6, 0.4};
    double umats[18] = {1, 0, 0, 0, 1, 0, 0, 0, 1,  /* identity, then 0.01 rad about x */
                        1, 0, 0, 0, cos(0.01), -sin(0.01), 0, sin(0.01), cos(0.01)};
    xro_shot s;
    memset(&s, 0, sizeof s);
    s.n_fast = 6;
    s.n_slow = 5;
    s.pixel = 2e-3;
    s.distance = 0.05;
    s.beam_f = 4e-3;
    s.beam_s = 5e-3;
    s.fdet[0] = 1.0;
    s.sdet[1] = 1.0;
    s.odet[2] = 1.0;
    s.oversample = 2;
    s.n_layers = 2;
    s.layer_dt = 1e-4;
    s.atten_len = 1.2e-4;
    s.n_src = 2;
    s.src_dir = src_dir;
    s.src_lambda = lam;
    s.src_weight = w;
    s.fluence = 1e24;
    s.kahn = 0.6;
    s.evec[0] = 1.0;
    const double cell[9] = {20, 0, 0, 0, 22, 0, 3, 0, 25};
    memcpy(s.cell, cell, sizeof cell);
    s.U[0] = s.U[4] = s.U[8] = 1.0;
    s.n_mos = 2;
    s.umats = umats;
    s.n_phi = 2;
    s.phi0 = 0.0;
    s.dphi = 0.02;
    s.spindle[1] = 1.0;
    s.N[0] = 4;
    s.N[1] = 5;
    s.N[2] = 6;
    s.gauss_c = 0.63;
    s.scale = 1.0;
    s.hkl_min[0] = -2;
    s.hkl_min[1] = -3;
    s.hkl_min[2] = -3;
    s.hkl_count[0] = 5;
    s.hkl_count[1] = 6;
    s.hkl_count[2] = 7;
    s.F = F;
    s.F_default = 2.5;

    int32_t pix[2 * 30];
    for (int k = 0; k < 30; ++k) {
        pix[2 * k] = k % 6;
        pix[2 * k + 1] = k / 6;
    }
    double a[30], b[30], mats[9 * 4], S[3 * 8], h[3 * 8], g[13], dl[30];
    for (int shape = XRO_SINCG; shape <= XRO_GAUSS; ++shape) {
        s.shape = shape;
        s.fluence = 1e24;
        CHECK(xro_simulate(&s, 30, pix, a, 2) == 0);
        s.fluence = 2e24;
        CHECK(xro_simulate(&s, 30, pix, b, 1) == 0);
        for (int k = 0; k < 30; ++k) CHECK(isfinite(a[k]) && a[k] >= 0.0 && b[k] == 2.0 * a[k]);
    }
    CHECK(xro_cell_mats(&s, mats) == 0);
    for (int k = 0; k < 36; ++k) CHECK(isfinite(mats[k]));
    int32_t idx[6 * 8];
    for (int q = 0; q < 8; ++q) {
        int32_t e[6] = {q % 6, q % 5, q % 4, q % 2, q % 2, q % 4};
        memcpy(idx + 6 * q, e, sizeof e);
    }
    CHECK(xro_trace(&s, 8, idx, S, h) == 0);
    for (int k = 0; k < 24; ++k) CHECK(isfinite(S[k]) && isfinite(h[k]));
    for (int k = 0; k < 30; ++k) dl[k] = (k % 3) - 1.0;
    s.shape = XRO_GAUSS;
    s.fluence = 1e24;
    CHECK(xro_gradient(&s, 30, pix, dl, g, 2) == 0);
    for (int k = 0; k < 13; ++k) CHECK(isfinite(g[k]));
    CHECK(isfinite(xro_lattice_sq(0.0, 5.0, XRO_SINCG, 0.63)) && xro_lattice_sq(0.0, 5.0, XRO_SINCG, 0.63) == 25.0);
    const double d[3] = {0.0, 0.6, 0.8}, inc[3] = {0.0, 0.0, 1.0}, e[3] = {1.0, 0.0, 0.0};
    CHECK(isfinite(xro_polarization(d, inc, e, 0.5)));
    CHECK(isfinite(xro_capture(1, 1e-4, 1.2e-4, 0.8)));
    /* background: every branch of the curve (below, inside, at a knot, above) */
    const double ks[4] = {0.0, 0.05, 0.1, 0.3}, kF[4] = {2.0, 2.6, 1.8, 1.1};
    xro_bg bg = {4, ks, kF, 1e10};
    CHECK(xro_bg_curve(&bg, -1.0) == 2.0 && xro_bg_curve(&bg, 0.05) == 2.6 && xro_bg_curve(&bg, 7.0) == 1.1);
    CHECK(isfinite(xro_bg_curve(&bg, 0.07)));
    double c[30];
    CHECK(xro_background(&s, &bg, 30, pix, c, 2) == 0);
    for (int k = 0; k < 30; ++k) CHECK(isfinite(c[k]) && c[k] > 0.0);
    printf("oracle checks passed under the sanitizers\n");
    return 0;
}
