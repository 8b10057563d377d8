/*
 * xro.h -- interface of the plain FP64 CPU oracle of the per-pixel X-ray
 * tracing sum.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  The product path never does, and
 * this header shares nothing with the product's headers.
 *
 * Units: metres (detector), angstrom (wavelength, cell), radians.
 * Lab frame: beam along +z.  Arrays are row-major, C order.
 */
#ifndef XRO_H
#define XRO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { XRO_SINCG = 0, XRO_GAUSS = 1 };

typedef struct xro_shot {
    /* detector */
    int32_t n_fast, n_slow;
    double pixel, distance, beam_f, beam_s;
    double fdet[3], sdet[3], odet[3];
    int32_t oversample, n_layers;
    double layer_dt, atten_len;
    /* beam */
    int32_t n_src;
    const double *src_dir;     /* [n_src][3] */
    const double *src_lambda;  /* [n_src]    */
    const double *src_weight;  /* [n_src]    */
    double fluence, kahn, evec[3];
    /* crystal */
    double cell[9];            /* rows a, b, c (crystal frame) */
    double U[9];
    int32_t n_mos;
    const double *umats;       /* [n_mos][3][3] */
    int32_t n_phi;
    double phi0, dphi, spindle[3];
    double N[3];
    int32_t shape;
    double gauss_c, scale;
    /* structure factors, dense, l fastest */
    int32_t hkl_min[3], hkl_count[3];
    const double *F;
    double F_default;
} xro_shot;

/* Image values of n pixels given as (i_fast, i_slow) pairs. */
int xro_simulate(const xro_shot *s, int64_t n, const int32_t *pix, double *out,
                 int nthreads);

/* Per-term intermediates for n terms given as (i_fast, i_slow, sub, layer,
 * src, rot) sextuples, where sub = u*O + v and rot = k*n_mos + m: the
 * scattering vector S and the fractional Miller indices h. */
int xro_trace(const xro_shot *s, int64_t n, const int32_t *idx, double *S_out,
              double *h_out);

/* The n_phi*n_mos lab-frame cell matrices, rows a', b', c'. */
int xro_cell_mats(const xro_shot *s, double *out);

/* Single-axis lattice factor squared at fractional index h. */
double xro_lattice_sq(double h, double N, int32_t shape, double c);

/* Kahn polarization factor for direction d, source direction inc and beam
 * polarization vector e. */
double xro_polarization(const double *d, const double *inc, const double *e,
                        double K);

/* Fraction of photons captured in layer t of thickness dt. */
double xro_capture(int32_t t, double dt, double mu, double cosrho);

/* Analytic gradient of L = sum_p g_p * I_p over a pixel list for the Gaussian
 * shape, with g_p = dL/dI_p given.  Writes 13 values: dL/dM0 (9, row-major,
 * M0 = U x cell rows), dL/dN (3), dL/dscale (1). */
int xro_gradient(const xro_shot *s, int64_t n, const int32_t *pix,
                 const double *dLdI, double *grad13, int nthreads);

/* An amorphous scatterer around the crystal (air, water): a scattering curve
 * F_bg(stol) given by n_knots (stol_k, F_k) pairs, stol = sin(theta)/lambda
 * strictly increasing, and the number of molecules in the beam. */
typedef struct xro_bg {
    int32_t n_knots;
    const double *stol;
    const double *F;
    double molecules;
} xro_bg;

/* F_bg at one stol: the piecewise-linear interpolant of the knots, constant
 * beyond the first and the last knot. */
double xro_bg_curve(const xro_bg *bg, double stol);

/* Background of n pixels given as (i_fast, i_slow) pairs; the crystal fields
 * of the shot are not used. */
int xro_background(const xro_shot *s, const xro_bg *bg, int64_t n, const int32_t *pix,
                   double *out, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
