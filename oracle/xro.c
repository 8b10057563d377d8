/*
 * xro.c -- plain FP64 CPU oracle of the per-pixel X-ray tracing sum.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg are the only callers.  It shares no code with the HIP
 * library: no headers, helpers, tables or constants.
 *
 * What is computed (paper, section II "Scientific background" and section III,
 * the description of the spots kernel): the photon count of every detector
 * pixel is simulated from a physical model of the crystal.  The count depends
 * on the crystal orientation, on its composition from smaller crystals (mosaic
 * domains), on the photon energy spectrum, and on one real structure factor
 * per Bragg spot.  Pixels are computed independently (section III).  The paper
 * prints no equation, so the physics below is the textbook kinematic model:
 *
 *   I(pixel) = r_e^2 * fluence * scale / (O^2 * n_phi * n_mos)
 *            * sum_{sub-pixel, layer}  dOmega * capture
 *              * sum_{source j}  w_j * P_j
 *                * sum_{phi k, domain m}  F(h0)^2 * L^2(h - h0)
 *
 * with h = M_{k,m} S the fractional Miller indices, S = (d - i_j)/lambda_j the
 * scattering vector, h0 the nearest integer triple, F the structure factor,
 * L^2 the squared lattice (shape) transform of an Na x Nb x Nc crystal,
 * P_j the Kahn polarization factor, dOmega the solid angle of the sample point
 * and capture the Beer-Lambert fraction absorbed in the sensor layer.
 *
 * Every sum is Neumaier-compensated (Neumaier 1974).  The background of an
 * amorphous scatterer (air, water) is at the end of the file.
 *
 * Evaluation contract.  A lattice factor near a zero of sin(pi N f) is
 * ill-conditioned in h, so S and h are computed with one fixed operation
 * sequence, without contraction (build with -ffp-contract=off):
 *   Fp   = ((double)i_f + ((double)v + 0.5) / O) * p - beam_f  (Sp likewise)
 *   r_i  = (Fp*fdet_i + Sp*sdet_i) + (distance + t*dt)*odet_i
 *   R    = sqrt((r_0*r_0 + r_1*r_1) + r_2*r_2)
 *   d_i  = r_i / R
 *   S_i  = (d_i - inc_i) / lambda
 *   h_i  = fma(M_i2, S_2, M_i0*S_0 + M_i1*S_1)
 *   M rows  a'_i = umat_m (R_k (U a_i)),  each product y_r = (Q_r0 x_0 + Q_r1 x_1) + Q_r2 x_2
 *   R_k  (Rodrigues) entries  (((1-c) u_r) u_c + [r==c] c) + s K_rc,
 *        K the cross-product matrix of the spindle u, c = cos, s = sin of
 *        phi0 + k*dphi.
 */
#include "xro.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double XRO_PI = 3.14159265358979323846264338327950288;
/* classical electron radius, metres (CODATA 2018) */
static const double XRO_RE = 2.8179403262e-15;

/* ---- compensated summation (Neumaier 1974) ----------------------------- */
typedef struct { double s, c; } ksum;

static void ksum_add(ksum *k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x))
        k->c += (k->s - t) + x;
    else
        k->c += (x - t) + k->s;
    k->s = t;
}

static double ksum_get(const ksum *k) { return k->s + k->c; }

/* ---- small vector helpers ----------------------------------------------- */
static void matvec(const double *Q, const double *x, double *y)
{
    for (int r = 0; r < 3; ++r)
        y[r] = (Q[3 * r + 0] * x[0] + Q[3 * r + 1] * x[1]) + Q[3 * r + 2] * x[2];
}

static double dot3(const double *a, const double *b)
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Rotation by angle phi about the unit axis u (Rodrigues' formula). */
static void rodrigues(const double *u, double phi, double *R)
{
    double c = cos(phi), s = sin(phi);
    double K[9] = {0.0, -u[2], u[1], u[2], 0.0, -u[0], -u[1], u[0], 0.0};
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q)
            R[3 * r + q] = (((1.0 - c) * u[r]) * u[q] + (r == q ? c : 0.0)) + s * K[3 * r + q];
}

/* Lab-frame cell vectors for spindle step k and mosaic domain m: the crystal
 * is turned by its orientation U, then by the spindle, then by the domain's
 * small rotation (paper section II: orientation and mosaic composition). */
static void cell_mat(const xro_shot *s, int k, int m, double *M)
{
    double Rk[9];
    rodrigues(s->spindle, s->phi0 + (double)k * s->dphi, Rk);
    const double *Um = s->umats + 9 * (size_t)m;
    for (int i = 0; i < 3; ++i) {
        double v1[3], v2[3];
        matvec(s->U, s->cell + 3 * i, v1);
        matvec(Rk, v1, v2);
        matvec(Um, v2, M + 3 * i);
    }
}

/* ---- physics pieces ------------------------------------------------------ */

/* Squared lattice transform along one axis at fractional index h.
 * SINCG: the interference function of N unit cells, sin^2(pi N h)/sin^2(pi h).
 * It is 1-periodic in h for integer N, so it is evaluated at the reduced
 * arguments f = h - rint(h) and g = N f - rint(N f), which equal the original
 * ones modulo integers; at f = 0 it takes its limit N^2.
 * GAUSS: N^2 exp(-2 N^2 f^2 / c), the squared Gaussian stand-in of width c. */
double xro_lattice_sq(double h, double N, int32_t shape, double c)
{
    double f = h - rint(h);
    if (shape == XRO_GAUSS)
        return N * N * exp(-2.0 * N * N * f * f / c);
    if (f == 0.0)
        return N * N;
    double g = N * f - rint(N * f);
    double q = sin(XRO_PI * g) / sin(XRO_PI * f);
    return q * q;
}

/* Kahn et al. (1982) polarization factor
 *   P = (1 + cos^2 2theta - K cos 2psi sin^2 2theta) / 2,
 * 2theta the scattering angle between d and the source direction inc, psi the
 * azimuth of d about inc measured from the polarization direction (the part
 * of e perpendicular to inc). */
double xro_polarization(const double *d, const double *inc, const double *e, double K)
{
    double ep[3], b[3];
    double ei = dot3(e, inc);
    for (int i = 0; i < 3; ++i) ep[i] = e[i] - ei * inc[i];
    double n = sqrt(dot3(ep, ep));
    for (int i = 0; i < 3; ++i) ep[i] /= n;
    cross3(inc, ep, b);
    double c2 = dot3(d, inc);
    double psi = atan2(dot3(d, b), dot3(d, ep));
    return 0.5 * (1.0 + c2 * c2 - K * cos(2.0 * psi) * (1.0 - c2 * c2));
}

/* Beer-Lambert: the fraction of photons travelling at angle rho to the sensor
 * normal absorbed between depths t*dt and (t+1)*dt, attenuation length mu.
 * dt == 0 means a sensor without thickness modelling (everything counts). */
double xro_capture(int32_t t, double dt, double mu, double cosrho)
{
    if (dt == 0.0)
        return 1.0;
    double l = mu * cosrho;
    return exp(-(double)t * dt / l) - exp(-(double)(t + 1) * dt / l);
}

/* Structure factor at the integer triple h0 (paper section II: one real
 * structure factor per Bragg spot); outside the tabulated box the default. */
static double fhkl(const xro_shot *s, const double *h0)
{
    int64_t idx = 0;
    for (int i = 0; i < 3; ++i) {
        double lo = (double)s->hkl_min[i];
        double hi = lo + (double)(s->hkl_count[i] - 1);
        if (!(h0[i] >= lo && h0[i] <= hi))
            return s->F_default;
        idx = idx * s->hkl_count[i] + (int64_t)(h0[i] - lo);
    }
    return s->F[idx];
}

/* Position of a sample point and the quantities that depend on it only. */
typedef struct { double d[3], R, cosrho, domega, capture; } sample_pt;

static void sample_point(const xro_shot *s, int i_f, int i_s, int u, int v, int t,
                         sample_pt *sp)
{
    const double O = (double)s->oversample;
    double Fp = ((double)i_f + ((double)v + 0.5) / O) * s->pixel - s->beam_f;
    double Sp = ((double)i_s + ((double)u + 0.5) / O) * s->pixel - s->beam_s;
    double L = s->distance + (double)t * s->layer_dt;
    double r[3];
    for (int i = 0; i < 3; ++i)
        r[i] = (Fp * s->fdet[i] + Sp * s->sdet[i]) + L * s->odet[i];
    sp->R = sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
    for (int i = 0; i < 3; ++i) sp->d[i] = r[i] / sp->R;
    sp->cosrho = dot3(sp->d, s->odet);
    /* solid angle of the full pixel area seen from this sample point; the
     * 1/O^2 of the final normalisation averages the sub-pixels */
    sp->domega = s->pixel * s->pixel * sp->cosrho / (sp->R * sp->R);
    sp->capture = xro_capture(t, s->layer_dt, s->atten_len, sp->cosrho);
}

static void scatter_vec(const xro_shot *s, const sample_pt *sp, int j, double *S)
{
    const double *inc = s->src_dir + 3 * (size_t)j;
    for (int i = 0; i < 3; ++i) S[i] = (sp->d[i] - inc[i]) / s->src_lambda[j];
}

static void miller(const double *M, const double *S, double *h)
{
    for (int i = 0; i < 3; ++i)
        h[i] = fma(M[3 * i + 2], S[2], M[3 * i + 0] * S[0] + M[3 * i + 1] * S[1]);
}

static double norm_factor(const xro_shot *s)
{
    double O = (double)s->oversample;
    return XRO_RE * XRO_RE * s->fluence * s->scale / (O * O * (double)s->n_phi * (double)s->n_mos);
}

static double pixel_value(const xro_shot *s, const double *mats, int i_f, int i_s)
{
    const int O = s->oversample;
    const int nrot = s->n_phi * s->n_mos;
    ksum acc = {0.0, 0.0};
    for (int u = 0; u < O; ++u)
        for (int v = 0; v < O; ++v)
            for (int t = 0; t < s->n_layers; ++t) {
                sample_pt sp;
                sample_point(s, i_f, i_s, u, v, t, &sp);
                for (int j = 0; j < s->n_src; ++j) {
                    double S[3];
                    scatter_vec(s, &sp, j, S);
                    double P = xro_polarization(sp.d, s->src_dir + 3 * (size_t)j, s->evec, s->kahn);
                    ksum sub = {0.0, 0.0};
                    for (int r = 0; r < nrot; ++r) {
                        double h[3], h0[3];
                        miller(mats + 9 * (size_t)r, S, h);
                        double L2 = 1.0;
                        for (int i = 0; i < 3; ++i) {
                            h0[i] = rint(h[i]);
                            L2 *= xro_lattice_sq(h[i], s->N[i], s->shape, s->gauss_c);
                        }
                        double F = fhkl(s, h0);
                        ksum_add(&sub, F * F * L2);
                    }
                    ksum_add(&acc, s->src_weight[j] * P * sp.domega * sp.capture * ksum_get(&sub));
                }
            }
    return norm_factor(s) * ksum_get(&acc);
}

static double *all_mats(const xro_shot *s)
{
    double *mats = (double *)malloc(sizeof(double) * 9 * (size_t)s->n_phi * (size_t)s->n_mos);
    if (!mats) return NULL;
    for (int k = 0; k < s->n_phi; ++k)
        for (int m = 0; m < s->n_mos; ++m)
            cell_mat(s, k, m, mats + 9 * ((size_t)k * s->n_mos + m));
    return mats;
}

int xro_cell_mats(const xro_shot *s, double *out)
{
    double *mats = all_mats(s);
    if (!mats) return -1;
    memcpy(out, mats, sizeof(double) * 9 * (size_t)s->n_phi * (size_t)s->n_mos);
    free(mats);
    return 0;
}

int xro_simulate(const xro_shot *s, int64_t n, const int32_t *pix, double *out, int nthreads)
{
    double *mats = all_mats(s);
    if (!mats) return -1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < n; ++p)
        out[p] = pixel_value(s, mats, pix[2 * p], pix[2 * p + 1]);
    free(mats);
    return 0;
}

int xro_trace(const xro_shot *s, int64_t n, const int32_t *idx, double *S_out, double *h_out)
{
    double *mats = all_mats(s);
    if (!mats) return -1;
    for (int64_t q = 0; q < n; ++q) {
        const int32_t *e = idx + 6 * q;
        int O = s->oversample;
        sample_pt sp;
        sample_point(s, e[0], e[1], e[2] / O, e[2] % O, e[3], &sp);
        scatter_vec(s, &sp, e[4], S_out + 3 * q);
        miller(mats + 9 * (size_t)e[5], S_out + 3 * q, h_out + 3 * q);
    }
    free(mats);
    return 0;
}

/* ---- gradient of a pixel functional, Gaussian shape ----------------------
 * For L = sum_p g_p I_p (g_p = dL/dI_p of any loss), with
 *   L2 = prod_i N_i^2 exp(-2 N_i^2 f_i^2 / c),  f_i = h_i - rint(h_i),
 *   dL2/dh_i = L2 * (-4 N_i^2 f_i / c)            (F is piecewise constant)
 *   dL2/dN_i = L2 * (2/N_i - 4 N_i f_i^2 / c)
 *   h_i = a'_i . S with a'_i = Q_{k,m} (U a_i), so dh_i/d(U a_i) = Q^T S,
 * the gradient with respect to the rows of M0 = U x cell is
 *   sum_terms K g_p w P dOmega C F^2 dL2/dh_i (Q_{k,m}^T S),
 * and dL/dscale = sum_p g_p I_p / scale. */
static void pixel_grad(const xro_shot *s, const double *mats, const double *qmats,
                       int i_f, int i_s, double gp, double *g13)
{
    const int O = s->oversample;
    const int nrot = s->n_phi * s->n_mos;
    const double K = norm_factor(s);
    ksum acc[13];
    memset(acc, 0, sizeof(acc));
    for (int u = 0; u < O; ++u)
        for (int v = 0; v < O; ++v)
            for (int t = 0; t < s->n_layers; ++t) {
                sample_pt sp;
                sample_point(s, i_f, i_s, u, v, t, &sp);
                for (int j = 0; j < s->n_src; ++j) {
                    double S[3];
                    scatter_vec(s, &sp, j, S);
                    double P = xro_polarization(sp.d, s->src_dir + 3 * (size_t)j, s->evec, s->kahn);
                    double wgt = gp * K * s->src_weight[j] * P * sp.domega * sp.capture;
                    for (int r = 0; r < nrot; ++r) {
                        double h[3], h0[3], f[3];
                        miller(mats + 9 * (size_t)r, S, h);
                        double L2 = 1.0;
                        for (int i = 0; i < 3; ++i) {
                            h0[i] = rint(h[i]);
                            f[i] = h[i] - h0[i];
                            L2 *= xro_lattice_sq(h[i], s->N[i], XRO_GAUSS, s->gauss_c);
                        }
                        double F = fhkl(s, h0);
                        double base = wgt * F * F * L2;
                        /* S' = Q^T S */
                        const double *Q = qmats + 9 * (size_t)r;
                        double Sp[3];
                        for (int c = 0; c < 3; ++c)
                            Sp[c] = Q[c] * S[0] + Q[3 + c] * S[1] + Q[6 + c] * S[2];
                        for (int i = 0; i < 3; ++i) {
                            double N = s->N[i];
                            double dh = base * (-4.0 * N * N * f[i] / s->gauss_c);
                            for (int c = 0; c < 3; ++c) ksum_add(&acc[3 * i + c], dh * Sp[c]);
                            ksum_add(&acc[9 + i], base * (2.0 / N - 4.0 * N * f[i] * f[i] / s->gauss_c));
                        }
                        ksum_add(&acc[12], base / s->scale);
                    }
                }
            }
    for (int i = 0; i < 13; ++i) g13[i] = ksum_get(&acc[i]);
}

int xro_gradient(const xro_shot *s, int64_t n, const int32_t *pix, const double *dLdI,
                 double *grad13, int nthreads)
{
    double *mats = all_mats(s);
    size_t nrot = (size_t)s->n_phi * (size_t)s->n_mos;
    double *qmats = (double *)malloc(sizeof(double) * 9 * nrot);
    double *part = (double *)malloc(sizeof(double) * 13 * (size_t)(n > 0 ? n : 1));
    if (!mats || !qmats || !part) { free(mats); free(qmats); free(part); return -1; }
    /* Q_{k,m} = umat_m R_k, the rotation applied after U */
    for (int k = 0; k < s->n_phi; ++k) {
        double Rk[9];
        rodrigues(s->spindle, s->phi0 + (double)k * s->dphi, Rk);
        for (int m = 0; m < s->n_mos; ++m) {
            const double *Um = s->umats + 9 * (size_t)m;
            double *Q = qmats + 9 * ((size_t)k * s->n_mos + m);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    Q[3 * r + c] = Um[3 * r + 0] * Rk[c] + Um[3 * r + 1] * Rk[3 + c] + Um[3 * r + 2] * Rk[6 + c];
        }
    }
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < n; ++p)
        pixel_grad(s, mats, qmats, pix[2 * p], pix[2 * p + 1], dLdI[p], part + 13 * p);
    for (int i = 0; i < 13; ++i) {
        ksum k = {0.0, 0.0};
        for (int64_t p = 0; p < n; ++p) ksum_add(&k, part[13 * p + i]);
        grad13[i] = ksum_get(&k);
    }
    free(mats); free(qmats); free(part);
    return 0;
}

/* ---- background of an amorphous scatterer --------------------------------
 * Section III lists, beside the spots kernel, a kernel that adds the
 * background scattered by the air and the water around the crystal; the
 * paper gives no formula for it.  An amorphous scatterer has no lattice: the
 * molecules scatter independently, and what one molecule scatters depends on
 * the scattering angle only, through sin(theta)/lambda = |S|/2, by its
 * scattering curve F_bg.  With the sample points, S, P, dOmega and capture of
 * the spots sum:
 *
 *   I_bg(pixel) = r_e^2 * fluence * molecules / O^2
 *               * sum_{sub-pixel, layer}  dOmega * capture
 *                 * sum_{source j}  w_j * P_j * F_bg(|S_j| / 2)^2
 *
 * No spindle or mosaic average: the scatterer has no orientation. */
double xro_bg_curve(const xro_bg *bg, double x)
{
    const int n = bg->n_knots;
    const double *s = bg->stol, *F = bg->F;
    if (x <= s[0]) return F[0];
    if (x >= s[n - 1]) return F[n - 1];
    int k = 0;
    while (s[k + 1] <= x) ++k; /* s[k] <= x < s[k+1] */
    double t = (x - s[k]) / (s[k + 1] - s[k]);
    return F[k] + t * (F[k + 1] - F[k]);
}

static double bg_pixel(const xro_shot *s, const xro_bg *bg, int i_f, int i_s)
{
    const int O = s->oversample;
    ksum acc = {0.0, 0.0};
    for (int u = 0; u < O; ++u)
        for (int v = 0; v < O; ++v)
            for (int t = 0; t < s->n_layers; ++t) {
                sample_pt sp;
                sample_point(s, i_f, i_s, u, v, t, &sp);
                for (int j = 0; j < s->n_src; ++j) {
                    double S[3];
                    scatter_vec(s, &sp, j, S);
                    double F = xro_bg_curve(bg, 0.5 * sqrt(dot3(S, S)));
                    double P = xro_polarization(sp.d, s->src_dir + 3 * (size_t)j, s->evec, s->kahn);
                    ksum_add(&acc, s->src_weight[j] * P * sp.domega * sp.capture * F * F);
                }
            }
    double Od = (double)O;
    return XRO_RE * XRO_RE * s->fluence * bg->molecules / (Od * Od) * ksum_get(&acc);
}

int xro_background(const xro_shot *s, const xro_bg *bg, int64_t n, const int32_t *pix,
                   double *out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < n; ++p)
        out[p] = bg_pixel(s, bg, pix[2 * p], pix[2 * p + 1]);
    return 0;
}
