// xrt_api.cpp -- host side of libxrt: the C ABI of include/xrt.h.
//
// Validates every argument, builds the per-shot tables (lab-frame cell
// matrices, sources with their polarization basis) in binary64, uploads them
// stream-ordered and launches the kernels.  Compiled with -ffp-contract=off:
// the cell matrices follow the fixed operation sequence documented at
// build_cell_mats so that h is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <climits>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/xrt.h"
#include "xrt_host.h"
#include "xrt_internal.h"

namespace {
thread_local std::string g_err;
}

namespace xrt {
namespace host {

xrt_status fail(xrt_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

xrt_status hip_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory)
        return fail(XRT_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(XRT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace host
}  // namespace xrt

namespace {

using xrt::host::fail;
using xrt::host::hip_fail;

#define HIP_TRY(call, what)                      \
    do {                                         \
        hipError_t e_ = (call);                  \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr double R_E = 2.8179403262e-15;  // classical electron radius, m (CODATA 2018)
constexpr double UNIT_TOL = 1e-12;
constexpr int32_t MAX_LOOP = 1 << 20;

bool is_fin(double x) { return std::isfinite(x); }
bool is_fin_n(const double *x, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}
double dot3(const double *a, const double *b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }
bool unit3(const double *a) { return is_fin_n(a, 3) && std::fabs(std::sqrt(dot3(a, a)) - 1.0) <= UNIT_TOL; }

xrt_status check_detector(const xrt_detector *d)
{
    if (!d) return fail(XRT_EINVAL, "detector is NULL");
    if (d->struct_size != sizeof(xrt_detector))
        return fail(XRT_EVERSION, "xrt_detector.struct_size %u, library expects %zu", d->struct_size,
                    sizeof(xrt_detector));
    if (d->n_fast < 1 || d->n_slow < 1) return fail(XRT_EINVAL, "detector size must be >= 1");
    if ((int64_t)d->n_fast * d->n_slow >= (int64_t)1 << 31)
        return fail(XRT_ERANGE, "detector has 2^31 or more pixels");
    if (!is_fin(d->pixel) || d->pixel <= 0) return fail(XRT_EINVAL, "pixel must be finite and > 0");
    if (!is_fin(d->distance) || d->distance <= 0) return fail(XRT_EINVAL, "distance must be finite and > 0");
    if (!is_fin(d->beam_f) || !is_fin(d->beam_s)) return fail(XRT_EINVAL, "beam centre must be finite");
    if (!unit3(d->fdet) || !unit3(d->sdet) || !unit3(d->odet))
        return fail(XRT_EINVAL, "fdet, sdet and odet must be unit vectors");
    if (d->oversample < 1 || d->oversample > 64) return fail(XRT_ERANGE, "oversample must be in [1, 64]");
    if (d->n_layers < 1 || d->n_layers > 64) return fail(XRT_ERANGE, "n_layers must be in [1, 64]");
    if (!is_fin(d->layer_dt) || d->layer_dt < 0) return fail(XRT_EINVAL, "layer_dt must be finite and >= 0");
    if (d->layer_dt == 0 && d->n_layers != 1)
        return fail(XRT_EINVAL, "layer_dt == 0 (no thickness model) requires n_layers == 1");
    if (!is_fin(d->atten_len) || d->atten_len <= 0) return fail(XRT_EINVAL, "atten_len must be finite and > 0");
    return XRT_OK;
}

xrt_status check_roi(const xrt_detector *d, int64_t f0, int64_t f1, int64_t s0, int64_t s1, int64_t k)
{
    if (f0 < 0 || f1 > d->n_fast || f0 >= f1 || s0 < 0 || s1 > d->n_slow || s0 >= s1)
        return fail(XRT_EINVAL, "ROI %lld: [%lld,%lld)x[%lld,%lld) is empty or outside the %dx%d detector",
                    (long long)k, (long long)f0, (long long)f1, (long long)s0, (long long)s1, d->n_fast,
                    d->n_slow);
    return XRT_OK;
}

xrt_status check_beam(const xrt_beam *b)
{
    if (!b) return fail(XRT_EINVAL, "beam is NULL");
    if (b->struct_size != sizeof(xrt_beam))
        return fail(XRT_EVERSION, "xrt_beam.struct_size %u, library expects %zu", b->struct_size,
                    sizeof(xrt_beam));
    if (b->n_src < 1 || b->n_src > MAX_LOOP) return fail(XRT_ERANGE, "n_src must be in [1, 2^20]");
    if (!b->dir || !b->lambda || !b->weight) return fail(XRT_EINVAL, "source arrays must not be NULL");
    if (!is_fin(b->fluence) || !is_fin(b->kahn)) return fail(XRT_EINVAL, "fluence and kahn must be finite");
    if (!unit3(b->evec)) return fail(XRT_EINVAL, "evec must be a unit vector");
    for (int j = 0; j < b->n_src; ++j) {
        const double *d = b->dir + 3 * j;
        if (!unit3(d)) return fail(XRT_EINVAL, "source %d: direction is not a unit vector", j);
        if (!is_fin(b->lambda[j]) || b->lambda[j] <= 0)
            return fail(XRT_EINVAL, "source %d: lambda must be finite and > 0", j);
        if (!is_fin(b->weight[j])) return fail(XRT_EINVAL, "source %d: weight must be finite", j);
        if (std::fabs(dot3(d, b->evec)) > 1.0 - 1e-6)
            return fail(XRT_EINVAL, "source %d: evec is parallel to the source direction", j);
    }
    return XRT_OK;
}

xrt_status check_background(const xrt_background *g)
{
    if (!g) return fail(XRT_EINVAL, "background is NULL");
    if (g->struct_size != sizeof(xrt_background))
        return fail(XRT_EVERSION, "xrt_background.struct_size %u, library expects %zu", g->struct_size,
                    sizeof(xrt_background));
    if (g->n_knots < 2 || g->n_knots > xrt::BG_MAX_KNOTS)
        return fail(XRT_ERANGE, "n_knots must be in [2, %d]", xrt::BG_MAX_KNOTS);
    if (!g->stol || !g->F) return fail(XRT_EINVAL, "curve arrays must not be NULL");
    if (!is_fin(g->molecules) || g->molecules < 0) return fail(XRT_EINVAL, "molecules must be finite and >= 0");
    for (int k = 0; k < g->n_knots; ++k) {
        if (!is_fin(g->stol[k]) || !is_fin(g->F[k])) return fail(XRT_EINVAL, "knot %d is not finite", k);
        if (k > 0 && !(g->stol[k] > g->stol[k - 1]))
            return fail(XRT_EINVAL, "knot %d: stol must increase strictly", k);
        if (k > 0 && !is_fin((float)((g->F[k] - g->F[k - 1]) / (g->stol[k] - g->stol[k - 1]))))
            return fail(XRT_EINVAL, "knots %d and %d: the slope is not finite in binary32", k - 1, k);
        if (!is_fin((float)g->stol[k]) || !is_fin((float)g->F[k]))
            return fail(XRT_ERANGE, "knot %d does not fit binary32", k);
    }
    return XRT_OK;
}

xrt_status check_crystal(const xrt_crystal *x)
{
    if (!x) return fail(XRT_EINVAL, "crystal is NULL");
    if (x->struct_size != sizeof(xrt_crystal))
        return fail(XRT_EVERSION, "xrt_crystal.struct_size %u, library expects %zu", x->struct_size,
                    sizeof(xrt_crystal));
    if (!is_fin_n(x->cell, 9) || !is_fin_n(x->U, 9)) return fail(XRT_EINVAL, "cell and U must be finite");
    if (x->n_mos < 1 || x->n_phi < 1) return fail(XRT_EINVAL, "n_mos and n_phi must be >= 1");
    if ((int64_t)x->n_mos * x->n_phi > MAX_LOOP) return fail(XRT_ERANGE, "n_phi * n_mos exceeds 2^20");
    if (!x->umats) return fail(XRT_EINVAL, "umats must not be NULL");
    if (!is_fin_n(x->umats, 9 * (size_t)x->n_mos)) return fail(XRT_EINVAL, "umats must be finite");
    if (!is_fin(x->phi0) || !is_fin(x->dphi)) return fail(XRT_EINVAL, "phi0 and dphi must be finite");
    if (!unit3(x->spindle)) return fail(XRT_EINVAL, "spindle must be a unit vector");
    if (x->shape != XRT_SHAPE_SINCG && x->shape != XRT_SHAPE_GAUSS)
        return fail(XRT_EINVAL, "unknown shape %d", x->shape);
    for (int i = 0; i < 3; ++i) {
        const double N = x->N[i];
        if (!is_fin(N) || N <= 0 || N > 1000) return fail(XRT_ERANGE, "N[%d] must be in (0, 1000]", i);
        if (x->shape == XRT_SHAPE_SINCG && N != std::floor(N))
            return fail(XRT_EINVAL, "N[%d] = %g: the sincg shape needs whole unit cells", i, N);
    }
    if (!is_fin(x->gauss_c) || x->gauss_c <= 0) return fail(XRT_EINVAL, "gauss_c must be finite and > 0");
    if (!is_fin(x->scale)) return fail(XRT_EINVAL, "scale must be finite");
    return XRT_OK;
}

void matvec(const double *Q, const double *x, double *y)
{
    for (int r = 0; r < 3; ++r) y[r] = (Q[3 * r + 0] * x[0] + Q[3 * r + 1] * x[1]) + Q[3 * r + 2] * x[2];
}

// Rotation by phi about the unit axis u (Rodrigues), entry by entry as
// (((1 - c) u_r) u_q + [r == q] c) + s K_rq with K the cross-product matrix.
void rodrigues(const double *u, double phi, double *R)
{
    const double c = std::cos(phi), s = std::sin(phi);
    const double K[9] = {0.0, -u[2], u[1], u[2], 0.0, -u[0], -u[1], u[0], 0.0};
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q)
            R[3 * r + q] = (((1.0 - c) * u[r]) * u[q] + (r == q ? c : 0.0)) + s * K[3 * r + q];
}

// Lab-frame cell matrices M_{k,m}, rows a'_i = umat_m (R_k (U a_i)), each
// product y_r = (Q_r0 x_0 + Q_r1 x_1) + Q_r2 x_2 (paper section II: the
// crystal orientation and its mosaic domains).
void build_cell_mats(const xrt_crystal *x, double *out)
{
    for (int k = 0; k < x->n_phi; ++k) {
        double Rk[9];
        rodrigues(x->spindle, x->phi0 + (double)k * x->dphi, Rk);
        for (int m = 0; m < x->n_mos; ++m) {
            double *M = out + 9 * ((size_t)k * x->n_mos + m);
            for (int i = 0; i < 3; ++i) {
                double v1[3], v2[3];
                matvec(x->U, x->cell + 3 * i, v1);
                matvec(Rk, v1, v2);
                matvec(x->umats + 9 * (size_t)m, v2, M + 3 * i);
            }
        }
    }
}

// Rotations Q_{k,m} = umat_m R_k applied after U (for the adjoint:
// h_i = (U a_i) . (Q^T S)).
void build_rotations(const xrt_crystal *x, double *out)
{
    for (int k = 0; k < x->n_phi; ++k) {
        double Rk[9];
        rodrigues(x->spindle, x->phi0 + (double)k * x->dphi, Rk);
        for (int m = 0; m < x->n_mos; ++m) {
            const double *Um = x->umats + 9 * (size_t)m;
            double *Q = out + 9 * ((size_t)k * x->n_mos + m);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    Q[3 * r + c] = (Um[3 * r] * Rk[c] + Um[3 * r + 1] * Rk[3 + c]) + Um[3 * r + 2] * Rk[6 + c];
        }
    }
}

// Source rows: direction, wavelength, weight, the polarization basis
// e_perp = unit(evec - (evec . dir) dir), b = dir x e_perp, and 1/(2 lambda).
void build_sources(const xrt_beam *b, double *out)
{
    for (int j = 0; j < b->n_src; ++j) {
        double *row = out + xrt::SRC_STRIDE * (size_t)j;
        const double *d = b->dir + 3 * j;
        std::memset(row, 0, sizeof(double) * xrt::SRC_STRIDE);
        for (int i = 0; i < 3; ++i) row[xrt::SRC_DIR + i] = d[i];
        row[xrt::SRC_LAMBDA] = b->lambda[j];
        row[xrt::SRC_WEIGHT] = b->weight[j];
        row[xrt::SRC_HIL] = 0.5 / b->lambda[j];
        const double ed = dot3(b->evec, d);
        double e[3];
        for (int i = 0; i < 3; ++i) e[i] = b->evec[i] - ed * d[i];
        const double n = std::sqrt(dot3(e, e));
        for (int i = 0; i < 3; ++i) e[i] /= n;
        row[xrt::SRC_E + 0] = e[0];
        row[xrt::SRC_E + 1] = e[1];
        row[xrt::SRC_E + 2] = e[2];
        row[xrt::SRC_B + 0] = d[1] * e[2] - d[2] * e[1];
        row[xrt::SRC_B + 1] = d[2] * e[0] - d[0] * e[2];
        row[xrt::SRC_B + 2] = d[0] * e[1] - d[1] * e[0];
    }
}

// Detector and beam fields of the kernel parameters.
void fill_geometry(const xrt_detector *d, const xrt_beam *b, xrt::Params &p)
{
    std::memset(&p, 0, sizeof p);
    p.pixel = d->pixel;
    p.distance = d->distance;
    p.beam_f = d->beam_f;
    p.beam_s = d->beam_s;
    for (int i = 0; i < 3; ++i) {
        p.fdet[i] = d->fdet[i];
        p.sdet[i] = d->sdet[i];
        p.odet[i] = d->odet[i];
    }
    p.layer_dt = d->layer_dt;
    p.atten_len = d->atten_len;
    p.O = d->oversample;
    p.T = d->n_layers;
    p.n_src = b->n_src;
    p.kahn = b->kahn;
}

// Geometry and lattice fields of the kernel parameters (everything except
// tables and output).
void fill_params(const xrt_detector *d, const xrt_beam *b, const xrt_crystal *x, xrt::Params &p)
{
    fill_geometry(d, b, p);
    p.n_rot = x->n_phi * x->n_mos;
    p.shape = x->shape;
    double ln = 0.0;
    for (int i = 0; i < 3; ++i) {
        p.N[i] = x->N[i];
        p.gk[i] = 2.0 * x->N[i] * x->N[i] / x->gauss_c;
        p.m2gk[i] = -2.0 * p.gk[i];
        p.inv2N[i] = 2.0 / x->N[i];
        ln += 2.0 * std::log(x->N[i]);
    }
    p.ln_n2 = ln;
    const double O = (double)d->oversample;
    p.norm = R_E * R_E * b->fluence * x->scale / (O * O * (double)x->n_phi * (double)x->n_mos);
}

}  // namespace

struct xrt_fhkl {
    int device;
    int32_t lo[3], hi[3];  // padded box of integer h (hkl_min - PAD .. hkl_max + PAD)
    int32_t sa, sb;        // element strides of the h and k axes in the padded box
    double *F2_64;
    float *F2_32;
    uint32_t bytes64, bytes32;
};

namespace {

// bias plus the element index of h = (0, 0, 0) in the padded table (an exact
// binary64 integer; see table_offset in the kernels): 2^49 for the binary64
// table, 2^50 for the binary32 one.
double biased_zero_index(const xrt_fhkl *t, double bias)
{
    const int64_t o = -((int64_t)t->lo[0] * t->sa + (int64_t)t->lo[1] * t->sb + t->lo[2]);
    return bias + (double)o;
}

// True when every rint(h) of the shot provably lies in the padded box, so the
// kernels may skip the clamp.  |h_i| = |a'_i . S| <= |a'_i| max|S|, and
// |S| = |d - dir_j| / lambda_j = 2 sin(angle(d, dir_j)/2) / lambda_j.  The
// sample points fill a box (detector rectangle x layer depths); if every
// vertex is within 90 degrees of dir_j, the cone of directions within the
// largest vertex angle is convex and holds the whole box, so the vertices
// bound the angle; otherwise |d - dir_j| <= 2.
bool h_inside(const xrt_detector *d, const int64_t box[4], const xrt_beam *b, const double *mats,
              size_t n_rot, const xrt_fhkl *t)
{
    double Fr[2] = {box[0] * d->pixel - d->beam_f, box[1] * d->pixel - d->beam_f};
    double Sr[2] = {box[2] * d->pixel - d->beam_s, box[3] * d->pixel - d->beam_s};
    double Lr[2] = {d->distance, d->distance + (double)(d->n_layers - 1) * d->layer_dt};
    double smax = 0.0;
    for (int j = 0; j < b->n_src; ++j) {
        const double *inc = b->dir + 3 * j;
        double cmin = 1.0;
        for (int a = 0; a < 8; ++a) {
            double r[3];
            for (int i = 0; i < 3; ++i)
                r[i] = Fr[a & 1] * d->fdet[i] + Sr[(a >> 1) & 1] * d->sdet[i] + Lr[a >> 2] * d->odet[i];
            const double n = std::sqrt(dot3(r, r));
            cmin = std::fmin(cmin, dot3(r, inc) / n);
        }
        const double chord = cmin > 1e-6 ? std::sqrt(2.0 - 2.0 * cmin) : 2.0;
        smax = std::fmax(smax, chord / b->lambda[j]);
    }
    smax = smax * (1.0 + 1e-9) + 1e-12;
    for (int i = 0; i < 3; ++i) {
        double rmax = 0.0;
        for (size_t r = 0; r < n_rot; ++r) {
            const double *row = mats + 9 * r + 3 * i;
            rmax = std::fmax(rmax, std::sqrt(dot3(row, row)));
        }
        const double bound = std::ceil(rmax * smax * (1.0 + 1e-9) + 1e-9) + 1.0;
        if (!(bound < 1e9) || -bound < t->lo[i] || bound > t->hi[i]) return false;
    }
    return true;
}

}  // namespace

extern "C" {

xrt_status xrt_version(int32_t *major, int32_t *minor)
{
    if (!major || !minor) return fail(XRT_EINVAL, "NULL output pointer");
    *major = XRT_VERSION_MAJOR;
    *minor = XRT_VERSION_MINOR;
    return XRT_OK;
}

const char *xrt_last_error(void) { return g_err.c_str(); }

xrt_status xrt_fhkl_create(const xrt_fhkl_desc *desc, const void *dev_F, void *stream, xrt_fhkl **out)
{
    if (!desc || !dev_F || !out) return fail(XRT_EINVAL, "NULL argument");
    *out = nullptr;
    if (desc->struct_size != sizeof(xrt_fhkl_desc))
        return fail(XRT_EVERSION, "xrt_fhkl_desc.struct_size %u, library expects %zu", desc->struct_size,
                    sizeof(xrt_fhkl_desc));
    if (desc->dtype != XRT_F32 && desc->dtype != XRT_F64) return fail(XRT_EINVAL, "dtype must be XRT_F32 or XRT_F64");
    if (!is_fin(desc->F_default)) return fail(XRT_EINVAL, "F_default must be finite");
    const int P = xrt::FHKL_PAD;
    int64_t n[3], padded = 1;
    for (int i = 0; i < 3; ++i) {
        if (desc->hkl_count[i] < 1) return fail(XRT_EINVAL, "hkl_count[%d] must be >= 1", i);
        if (desc->hkl_min[i] < -(1 << 20) || desc->hkl_min[i] > (1 << 20) ||
            (int64_t)desc->hkl_min[i] + desc->hkl_count[i] > (1 << 20))
            return fail(XRT_ERANGE, "axis %d: table must lie within |h| <= 2^20", i);
        n[i] = (int64_t)desc->hkl_count[i] + 2 * P;
        padded *= n[i];
    }
    if (padded >= (int64_t)1 << 28) return fail(XRT_ERANGE, "padded table has 2^28 or more entries");

    xrt_fhkl *t = new (std::nothrow) xrt_fhkl();
    if (!t) return fail(XRT_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&t->device);
    if (e == hipSuccess) e = hipMalloc((void **)&t->F2_64, sizeof(double) * padded);
    if (e == hipSuccess) e = hipMalloc((void **)&t->F2_32, sizeof(float) * padded);
    hipStream_t s = (hipStream_t)stream;
    if (e == hipSuccess)
        e = xrt::launch_pad_table(dev_F, desc->dtype == XRT_F64, desc->hkl_count[0], desc->hkl_count[1],
                                  desc->hkl_count[2], P, desc->F_default, t->F2_64, t->F2_32, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(t->F2_64);
        (void)hipFree(t->F2_32);
        delete t;
        return hip_fail(e, "xrt_fhkl_create");
    }
    for (int i = 0; i < 3; ++i) {
        t->lo[i] = desc->hkl_min[i] - P;
        t->hi[i] = desc->hkl_min[i] + desc->hkl_count[i] - 1 + P;
    }
    t->sb = (int32_t)n[2];
    t->sa = (int32_t)(n[1] * n[2]);
    t->bytes64 = (uint32_t)(sizeof(double) * padded);
    t->bytes32 = (uint32_t)(sizeof(float) * padded);
    *out = t;
    return XRT_OK;
}

xrt_status xrt_fhkl_destroy(xrt_fhkl *t)
{
    if (!t) return XRT_OK;
    hipError_t e1 = hipFree(t->F2_64);
    hipError_t e2 = hipFree(t->F2_32);
    delete t;
    if (e1 != hipSuccess) return hip_fail(e1, "xrt_fhkl_destroy");
    if (e2 != hipSuccess) return hip_fail(e2, "xrt_fhkl_destroy");
    return XRT_OK;
}

xrt_status xrt_cell_mats(const xrt_crystal *xtal, double *host_out)
{
    xrt_status st = check_crystal(xtal);
    if (st) return st;
    if (!host_out) return fail(XRT_EINVAL, "NULL output pointer");
    build_cell_mats(xtal, host_out);
    return XRT_OK;
}

}  // extern "C"

// The static device memory of xrt_simulate_noalloc (its layout and size are
// described there); host code reaches it only through the per-device address
// that hipGetSymbolAddress returns.
static __device__ __align__(256) char scratch[XRT_NOALLOC_SCRATCH_BYTES];

namespace {

// Everything a launch over a list of equal-size regions of interest needs:
// kernel parameters and the per-shot tables in one host buffer
// [cell matrices | sources | ROI origins (int32 pairs) | rotations Q].
struct Plan {
    xrt::Params p;
    std::vector<double> host;
    size_t n_rot = 0, o_src = 0, o_orig = 0, o_q = 0;
    bool clamp = true;
};

// Split factor of the per-pixel sums: a region list of fewer than
// SPLIT_TARGET tiles has each pixel's outer iterations (sub-pixel, layer,
// source) cut into K parts so that about SPLIT_TARGET workgroups share the
// work, each part keeping at least SPLIT_MIN_TERMS terms per pixel.  K
// depends on the shot alone (tile count and loop extents), never on the
// device or on other work, so a shot's bits are the same in every path.
constexpr int64_t SPLIT_TARGET = 2048;
constexpr int64_t SPLIT_MIN_TERMS = 1024;

int32_t split_factor(int64_t n_tiles, int64_t n_outer, int64_t terms_per_pixel)
{
    if (n_tiles >= SPLIT_TARGET) return 1;
    int64_t k = (SPLIT_TARGET + n_tiles - 1) / n_tiles;
    k = std::min<int64_t>({k, n_outer, terms_per_pixel / SPLIT_MIN_TERMS, (int64_t)xrt::SERVE_MAX_SPLIT});
    return (int32_t)std::max<int64_t>(k, 1);
}

xrt_status make_plan(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal,
                     const xrt_fhkl *fhkl, int64_t n_roi, const int32_t *origins, int32_t roi_nf,
                     int32_t roi_ns, bool with_q, Plan &pl)
{
    xrt_status st;
    if ((st = check_detector(det)) || (st = check_beam(beam)) || (st = check_crystal(xtal))) return st;
    if (!fhkl) return fail(XRT_EINVAL, "fhkl is NULL");
    if (n_roi < 1 || n_roi > (1 << 22)) return fail(XRT_ERANGE, "n_roi must be in [1, 2^22]");
    if (!origins) return fail(XRT_EINVAL, "ROI origins are NULL");
    if (roi_nf < 1 || roi_ns < 1) return fail(XRT_EINVAL, "ROI size must be >= 1");
    int64_t box[4] = {INT64_MAX, INT64_MIN, INT64_MAX, INT64_MIN};
    for (int64_t k = 0; k < n_roi; ++k) {
        const int64_t f0 = origins[2 * k], s0 = origins[2 * k + 1];
        if ((st = check_roi(det, f0, f0 + roi_nf, s0, s0 + roi_ns, k))) return st;
        box[0] = std::min(box[0], f0);
        box[1] = std::max(box[1], f0 + roi_nf);
        box[2] = std::min(box[2], s0);
        box[3] = std::max(box[3], s0 + roi_ns);
    }
    const int64_t tiles_f = (roi_nf + 15) / 16, tiles_per = tiles_f * ((roi_ns + 15) / 16);
    if (tiles_per * n_roi >= ((int64_t)1 << 31)) return fail(XRT_ERANGE, "too many tiles");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != fhkl->device)
        return fail(XRT_EINVAL, "fhkl lives on device %d, current device is %d", fhkl->device, dev);

    pl.n_rot = (size_t)xtal->n_phi * xtal->n_mos;
    pl.o_src = 9 * pl.n_rot;
    pl.o_orig = pl.o_src + xrt::SRC_STRIDE * (size_t)beam->n_src;
    pl.o_q = pl.o_orig + (size_t)n_roi;  // one double slot holds one int32 pair
    // adjoint: Q in binary64, then in binary32 (10 floats, 5 double slots, per rotation)
    pl.host.assign(pl.o_q + (with_q ? 14 * pl.n_rot : 0), 0.0);
    build_cell_mats(xtal, pl.host.data());
    build_sources(beam, pl.host.data() + pl.o_src);
    std::memcpy(pl.host.data() + pl.o_orig, origins, sizeof(int32_t) * 2 * (size_t)n_roi);
    if (with_q) {
        build_rotations(xtal, pl.host.data() + pl.o_q);
        float *q32 = reinterpret_cast<float *>(pl.host.data() + pl.o_q + 9 * pl.n_rot);
        for (size_t r = 0; r < pl.n_rot; ++r)
            for (int i = 0; i < 9; ++i) q32[10 * r + i] = (float)pl.host[pl.o_q + 9 * r + i];
    }

    xrt::Params &p = pl.p;
    fill_params(det, beam, xtal, p);
    p.roi_nf = roi_nf;
    p.roi_ns = roi_ns;
    p.tiles_f = (int32_t)tiles_f;
    p.tiles_per_roi = (int32_t)tiles_per;
    p.n_roi = (int32_t)n_roi;
    p.n_tiles = (int32_t)(tiles_per * n_roi);
    p.F2_64 = fhkl->F2_64;
    p.F2_32 = fhkl->F2_32;
    p.bytes64 = fhkl->bytes64;
    p.bytes32 = fhkl->bytes32;
    for (int i = 0; i < 3; ++i) {
        p.lo_d[i] = fhkl->lo[i];
        p.hi_d[i] = fhkl->hi[i];
    }
    p.sa = (double)fhkl->sa;
    p.sb = (double)fhkl->sb;
    p.off64 = biased_zero_index(fhkl, 562949953421312.0);   // 2^49
    p.off32 = biased_zero_index(fhkl, 1125899906842624.0);  // 2^50
    pl.clamp = !h_inside(det, box, beam, pl.host.data(), pl.n_rot, fhkl);
    const int64_t n_outer = (int64_t)p.O * p.O * p.T * p.n_src;
    p.split = split_factor(p.n_tiles, n_outer, n_outer * p.n_rot);
    p.partial = nullptr;
    return XRT_OK;
}

// Points the parameters at the uploaded copy of the tables.
void bind_tables(Plan &pl, double *dev)
{
    pl.p.mats = dev;
    pl.p.src = dev + pl.o_src;
    pl.p.origins = reinterpret_cast<const int32_t *>(dev + pl.o_orig);
    pl.p.qmats = pl.host.size() > pl.o_q ? dev + pl.o_q : nullptr;
    pl.p.qmats32 = pl.host.size() > pl.o_q ? reinterpret_cast<const float *>(dev + pl.o_q + 9 * pl.n_rot) : nullptr;
}

xrt_status check_call(int32_t precision, int32_t dtype, const void *ptr, const char *what)
{
    if (precision != XRT_FP64 && precision != XRT_MIXED) return fail(XRT_EINVAL, "unknown precision %d", precision);
    if (dtype != XRT_F32 && dtype != XRT_F64) return fail(XRT_EINVAL, "unknown dtype %d", dtype);
    if (!ptr) return fail(XRT_EINVAL, "%s is NULL", what);
    return XRT_OK;
}

// Bytes of the split sums' partial sums [tile][part][lane] of a plan (0
// when its sums are not split).
size_t partial_bytes(const Plan &pl)
{
    return pl.p.split > 1 ? sizeof(double) * (size_t)pl.p.n_tiles * pl.p.split * 256 : 0;
}

// Uploads the plan's tables and launches the spots kernel (and the reduce
// kernel of split sums).  Device memory for the tables and the partial sums:
// `work` (tables at its start, partial sums at part_at bytes) when given,
// else one stream-ordered allocation freed stream-ordered after the launch.
xrt_status run_spots(Plan &pl, int32_t precision, void *dev_image, int32_t out_dtype, int32_t accumulate,
                     hipStream_t s, const char *who, char *work = nullptr, size_t part_at = 0)
{
    pl.p.image = dev_image;
    pl.p.out_f64 = out_dtype == XRT_F64;
    pl.p.accumulate = accumulate;
    const size_t bytes = sizeof(double) * pl.host.size();
    const size_t part_bytes = partial_bytes(pl);
    double *tables = reinterpret_cast<double *>(work);
    double *part = reinterpret_cast<double *>(work + part_at);
    if (!work) {
        HIP_TRY(hipMallocAsync((void **)&tables, bytes + part_bytes, s), "hipMallocAsync");
        part = tables + pl.host.size();
    }
    hipError_t e = hipMemcpyAsync(tables, pl.host.data(), bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        bind_tables(pl, tables);
        pl.p.partial = part_bytes ? part : nullptr;
        e = xrt::launch_spots(pl.p, precision, pl.clamp, s);
    }
    hipError_t e2 = work ? hipSuccess : hipFreeAsync(tables, s);
    if (e != hipSuccess) return hip_fail(e, who);
    if (e2 != hipSuccess) return hip_fail(e2, who);
    return XRT_OK;
}

// Device memory of xrt_simulate_noalloc: the shot's tables in the first
// NOALLOC_TABLE_BYTES, the split sums' partial sums after them.  A split
// sum has fewer than 2 * SPLIT_TARGET (tile, part) units of 256 lanes, so
// its partial sums fit in NOALLOC_PART_BYTES.  Each device holds its own
// copy from the library's load until the process ends.
constexpr size_t NOALLOC_TABLE_BYTES = (size_t)1 << 20;
constexpr size_t NOALLOC_PART_BYTES = (size_t)2 * SPLIT_TARGET * 256 * sizeof(double);
constexpr size_t NOALLOC_BYTES = NOALLOC_TABLE_BYTES + NOALLOC_PART_BYTES;
static_assert(NOALLOC_BYTES == XRT_NOALLOC_SCRATCH_BYTES, "scratch size of include/xrt.h");

// The device address of `scratch` on each device, looked up once per device
// with that device current (host code never uses the symbol itself).
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch[NOALLOC_MAX_DEVICES] = {};

xrt_status scratch_of_device(int dev, char **out)
{
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(XRT_ERANGE, "device %d beyond the %d devices of the static scratch table", dev,
                    NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(XRT_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = static_cast<char *>(ptr);
    }
    *out = g_scratch[dev];
    return XRT_OK;
}

}  // namespace

namespace xrt {
namespace host {

xrt_status check_shot(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal)
{
    xrt_status st;
    if ((st = check_detector(det)) || (st = check_beam(beam)) || (st = check_crystal(xtal))) return st;
    return check_roi(det, det->roi_f0, det->roi_f1, det->roi_s0, det->roi_s1, 0);
}

xrt_status served_descriptor(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal,
                             const xrt_fhkl *fhkl, int32_t out_dtype, ShotDesc *d, std::vector<double> &tables)
{
    const int32_t origin[2] = {det->roi_f0, det->roi_s0};
    Plan pl;
    xrt_status st = make_plan(det, beam, xtal, fhkl, 1, origin, det->roi_f1 - det->roi_f0,
                              det->roi_s1 - det->roi_s0, false, pl);
    if (st) return st;
    std::memset(d, 0, sizeof *d);
    d->p = pl.p;
    d->p.out_f64 = out_dtype == XRT_F64;
    d->roi_f0 = det->roi_f0;
    d->roi_s0 = det->roi_s0;
    d->clamp = pl.clamp ? 1 : 0;
    tables.assign(pl.host.begin(), pl.host.begin() + (ptrdiff_t)pl.o_orig);
    return XRT_OK;
}

xrt_status check_background_desc(const xrt_background *bg) { return check_background(bg); }

void background_rows(const xrt_background *bg, double *k64, float *k32)
{
    const int n = bg->n_knots;
    for (int k = 0; k < n; ++k) {
        k64[3 * k] = bg->stol[k];
        k64[3 * k + 1] = bg->F[k];
        k64[3 * k + 2] = k + 1 < n ? (bg->F[k + 1] - bg->F[k]) / (bg->stol[k + 1] - bg->stol[k]) : 0.0;
        for (int c = 0; c < 3; ++c) k32[3 * k + c] = (float)k64[3 * k + c];
    }
}

double background_norm(const xrt_detector *det, const xrt_beam *beam, double molecules)
{
    const double O = (double)det->oversample;
    return R_E * R_E * beam->fluence * molecules / (O * O);
}

int32_t split_of(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal)
{
    const int64_t nf = det->roi_f1 - det->roi_f0, ns = det->roi_s1 - det->roi_s0;
    const int64_t n_tiles = ((nf + 15) / 16) * ((ns + 15) / 16);
    const int64_t n_outer = (int64_t)det->oversample * det->oversample * det->n_layers * beam->n_src;
    return split_factor(n_tiles, n_outer, n_outer * xtal->n_phi * xtal->n_mos);
}

void fhkl_tables(const xrt_fhkl *t, const double **F2_64, const float **F2_32, uint32_t *bytes64, uint32_t *bytes32)
{
    *F2_64 = t->F2_64;
    *F2_32 = t->F2_32;
    *bytes64 = t->bytes64;
    *bytes32 = t->bytes32;
}

}  // namespace host
}  // namespace xrt

extern "C" {

xrt_status xrt_simulate(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal,
                        const xrt_fhkl *fhkl, int32_t precision, void *dev_image, int32_t out_dtype,
                        int32_t accumulate, void *stream)
{
    xrt_status st;
    if ((st = check_call(precision, out_dtype, dev_image, "dev_image"))) return st;
    if (accumulate != 0 && accumulate != 1) return fail(XRT_EINVAL, "accumulate must be 0 or 1");
    if (!det) return fail(XRT_EINVAL, "detector is NULL");
    if ((st = check_detector(det))) return st;
    if ((st = check_roi(det, det->roi_f0, det->roi_f1, det->roi_s0, det->roi_s1, 0))) return st;
    const int32_t origin[2] = {det->roi_f0, det->roi_s0};
    Plan pl;
    if ((st = make_plan(det, beam, xtal, fhkl, 1, origin, det->roi_f1 - det->roi_f0, det->roi_s1 - det->roi_s0,
                        false, pl)))
        return st;
    return run_spots(pl, precision, dev_image, out_dtype, accumulate, (hipStream_t)stream, "xrt_simulate");
}

xrt_status xrt_simulate_noalloc(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal,
                                const xrt_fhkl *fhkl, int32_t precision, void *dev_image, int32_t out_dtype,
                                int32_t accumulate, void *stream)
{
    xrt_status st;
    if ((st = check_call(precision, out_dtype, dev_image, "dev_image"))) return st;
    if (accumulate != 0 && accumulate != 1) return fail(XRT_EINVAL, "accumulate must be 0 or 1");
    if (!det) return fail(XRT_EINVAL, "detector is NULL");
    if ((st = check_detector(det))) return st;
    if ((st = check_roi(det, det->roi_f0, det->roi_f1, det->roi_s0, det->roi_s1, 0))) return st;
    const int32_t origin[2] = {det->roi_f0, det->roi_s0};
    Plan pl;
    if ((st = make_plan(det, beam, xtal, fhkl, 1, origin, det->roi_f1 - det->roi_f0, det->roi_s1 - det->roi_s0,
                        false, pl)))
        return st;
    const size_t tb = sizeof(double) * pl.host.size(), pb = partial_bytes(pl);
    if (tb > NOALLOC_TABLE_BYTES)
        return fail(XRT_ERANGE, "xrt_simulate_noalloc: the shot's tables take %zu bytes, above the %zu of the "
                    "static scratch (9 n_phi n_mos + 12 n_src + 1 doubles)", tb, NOALLOC_TABLE_BYTES);
    if (pb > NOALLOC_PART_BYTES)
        return fail(XRT_ERANGE, "xrt_simulate_noalloc: partial sums of %zu bytes above the %zu of the static "
                    "scratch", pb, NOALLOC_PART_BYTES);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    char *work = nullptr;
    if ((st = scratch_of_device(dev, &work))) return st;
    return run_spots(pl, precision, dev_image, out_dtype, accumulate, (hipStream_t)stream, "xrt_simulate_noalloc",
                     work, NOALLOC_TABLE_BYTES);
}

xrt_status xrt_simulate_rois(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal,
                             const xrt_fhkl *fhkl, int32_t precision, int64_t n_roi,
                             const int32_t *host_origins, int32_t roi_nf, int32_t roi_ns, void *dev_images,
                             int32_t out_dtype, void *stream)
{
    xrt_status st;
    if ((st = check_call(precision, out_dtype, dev_images, "dev_images"))) return st;
    Plan pl;
    if ((st = make_plan(det, beam, xtal, fhkl, n_roi, host_origins, roi_nf, roi_ns, false, pl))) return st;
    return run_spots(pl, precision, dev_images, out_dtype, 0, (hipStream_t)stream, "xrt_simulate_rois");
}

xrt_status xrt_backward_rois(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal,
                             const xrt_fhkl *fhkl, int32_t precision, int64_t n_roi,
                             const int32_t *host_origins, int32_t roi_nf, int32_t roi_ns,
                             const void *dev_dLdI, int32_t dLdI_dtype, double *dev_grad13, void *stream)
{
    xrt_status st;
    if ((st = check_call(precision, dLdI_dtype, dev_dLdI, "dev_dLdI"))) return st;
    if (!dev_grad13) return fail(XRT_EINVAL, "dev_grad13 is NULL");
    if (xtal && xtal->struct_size == sizeof(xrt_crystal) && xtal->shape != XRT_SHAPE_GAUSS)
        return fail(XRT_EINVAL, "the adjoint is defined for the Gaussian shape only");
    Plan pl;
    if ((st = make_plan(det, beam, xtal, fhkl, n_roi, host_origins, roi_nf, roi_ns, true, pl))) return st;
    pl.p.split = 1;  // the adjoint reduces per workgroup; its sums are never split
    if (xtal->scale == 0.0) return fail(XRT_EINVAL, "scale must be nonzero for its gradient");
    for (int i = 0; i < 9; ++i) pl.p.m0[i] = 0.0;
    for (int i = 0; i < 3; ++i) {
        double v[3];
        matvec(xtal->U, xtal->cell + 3 * i, v);
        for (int c = 0; c < 3; ++c) pl.p.m0[3 * i + c] = v[c];
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t tb = sizeof(double) * pl.host.size();
    const size_t pb = sizeof(double) * 13 * (size_t)pl.p.n_tiles;
    double *tables = nullptr, *partial = nullptr;
    HIP_TRY(hipMallocAsync((void **)&tables, tb, s), "hipMallocAsync");
    hipError_t e = hipMallocAsync((void **)&partial, pb, s);
    if (e == hipSuccess) e = hipMemcpyAsync(tables, pl.host.data(), tb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        bind_tables(pl, tables);
        e = xrt::launch_grad(pl.p, precision, pl.clamp, dev_dLdI, dLdI_dtype == XRT_F64, partial, dev_grad13,
                             1.0 / xtal->scale, s);
    }
    hipError_t e2 = hipFreeAsync(tables, s);
    hipError_t e3 = partial ? hipFreeAsync(partial, s) : hipSuccess;
    if (e != hipSuccess) return hip_fail(e, "xrt_backward_rois");
    if (e2 != hipSuccess) return hip_fail(e2, "xrt_backward_rois");
    if (e3 != hipSuccess) return hip_fail(e3, "xrt_backward_rois");
    return XRT_OK;
}

xrt_status xrt_simulate_background(const xrt_detector *det, const xrt_beam *beam, const xrt_background *bg,
                                   int32_t precision, void *dev_image, int32_t out_dtype, int32_t accumulate,
                                   void *stream)
{
    xrt_status st;
    if ((st = check_call(precision, out_dtype, dev_image, "dev_image"))) return st;
    if (accumulate != 0 && accumulate != 1) return fail(XRT_EINVAL, "accumulate must be 0 or 1");
    if ((st = check_detector(det)) || (st = check_beam(beam)) || (st = check_background(bg))) return st;
    if ((st = check_roi(det, det->roi_f0, det->roi_f1, det->roi_s0, det->roi_s1, 0))) return st;
    const int32_t nf = det->roi_f1 - det->roi_f0, ns = det->roi_s1 - det->roi_s0;
    const int n = bg->n_knots, n_src = beam->n_src;

    // one upload: [sources | origin | knots | sources (binary32, with the low
    // parts of the directions) | knots (binary32)]
    const size_t o_orig = xrt::SRC_STRIDE * (size_t)n_src, o_k64 = o_orig + 1, o_s32 = o_k64 + 3 * (size_t)n;
    const size_t o_k32 = o_s32 + xrt::SRC32_STRIDE * (size_t)n_src / 2;
    std::vector<double> host(o_k32 + (3 * (size_t)n + 1) / 2, 0.0);
    build_sources(beam, host.data());
    const int32_t origin[2] = {det->roi_f0, det->roi_s0};
    std::memcpy(host.data() + o_orig, origin, sizeof origin);
    double *k64 = host.data() + o_k64;
    float *s32 = reinterpret_cast<float *>(host.data() + o_s32);
    float *k32 = reinterpret_cast<float *>(host.data() + o_k32);
    xrt::host::background_rows(bg, k64, k32);
    for (int j = 0; j < n_src; ++j) {
        const double *row = host.data() + xrt::SRC_STRIDE * (size_t)j;
        float *r32 = s32 + xrt::SRC32_STRIDE * (size_t)j;
        for (int i = 0; i < xrt::SRC_STRIDE; ++i) r32[i] = (float)row[i];
        for (int i = 0; i < 3; ++i)  // dir = r32[i] + r32[LO + i] to about 2^-48
            r32[xrt::SRC32_DIR_LO + i] = (float)(row[xrt::SRC_DIR + i] - (double)r32[xrt::SRC_DIR + i]);
    }

    xrt::BgParams b;
    std::memset(&b, 0, sizeof b);
    xrt::Params &p = b.p;
    fill_geometry(det, beam, p);
    p.roi_nf = nf;
    p.roi_ns = ns;
    p.tiles_f = (nf + 15) / 16;
    p.tiles_per_roi = p.tiles_f * ((ns + 15) / 16);
    p.n_roi = 1;
    p.n_tiles = p.tiles_per_roi;
    p.split = 1;
    p.norm = xrt::host::background_norm(det, beam, bg->molecules);
    p.image = dev_image;
    p.out_f64 = out_dtype == XRT_F64;
    p.accumulate = accumulate;
    b.n_knots = n;

    hipStream_t s = (hipStream_t)stream;
    double *tables = nullptr;
    HIP_TRY(hipMallocAsync((void **)&tables, sizeof(double) * host.size(), s), "hipMallocAsync");
    hipError_t e = hipMemcpyAsync(tables, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        p.src = tables;
        p.origins = reinterpret_cast<const int32_t *>(tables + o_orig);
        b.knots64 = tables + o_k64;
        b.src32 = reinterpret_cast<const float *>(tables + o_s32);
        b.knots32 = reinterpret_cast<const float *>(tables + o_k32);
        e = xrt::launch_background(b, precision, s);
    }
    hipError_t e2 = hipFreeAsync(tables, s);
    if (e != hipSuccess) return hip_fail(e, "xrt_simulate_background");
    if (e2 != hipSuccess) return hip_fail(e2, "xrt_simulate_background");
    return XRT_OK;
}

xrt_status xrt_add_image(double *dev_acc, int32_t acc_nf, int32_t acc_ns, const void *dev_img, int32_t img_dtype,
                         int32_t img_nf, int32_t img_ns, int32_t f0, int32_t s0, void *stream)
{
    if (!dev_acc || !dev_img) return fail(XRT_EINVAL, "NULL image");
    if (img_dtype != XRT_F32 && img_dtype != XRT_F64) return fail(XRT_EINVAL, "unknown dtype %d", img_dtype);
    if (acc_nf < 1 || acc_ns < 1 || img_nf < 1 || img_ns < 1) return fail(XRT_EINVAL, "image sizes must be >= 1");
    if ((int64_t)acc_nf * acc_ns >= ((int64_t)1 << 40)) return fail(XRT_ERANGE, "accumulator has 2^40 or more pixels");
    if (f0 < 0 || s0 < 0 || (int64_t)f0 + img_nf > acc_nf || (int64_t)s0 + img_ns > acc_ns)
        return fail(XRT_EINVAL, "image [%d,%lld)x[%d,%lld) is outside the %dx%d accumulator", f0,
                    (long long)f0 + img_nf, s0, (long long)s0 + img_ns, acc_nf, acc_ns);
    const hipError_t e = xrt::launch_add_image(dev_acc, acc_nf, dev_img, img_dtype == XRT_F64, img_nf, img_ns, f0, s0,
                                               (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "xrt_add_image");
    return XRT_OK;
}

xrt_status xrt_add_images(double *dev_acc, int32_t acc_nf, int32_t acc_ns, const void *const *host_dev_imgs,
                          int32_t img_dtype, int64_t n_img, void *stream)
{
    if (!dev_acc) return fail(XRT_EINVAL, "NULL accumulator");
    if (img_dtype != XRT_F32 && img_dtype != XRT_F64) return fail(XRT_EINVAL, "unknown dtype %d", img_dtype);
    if (acc_nf < 1 || acc_ns < 1) return fail(XRT_EINVAL, "accumulator sizes must be >= 1");
    if ((int64_t)acc_nf * acc_ns >= ((int64_t)1 << 40)) return fail(XRT_ERANGE, "accumulator has 2^40 or more pixels");
    if (n_img < 0 || n_img > ((int64_t)1 << 24)) return fail(XRT_ERANGE, "n_img must be in [0, 2^24]");
    if (n_img == 0) return XRT_OK;
    if (!host_dev_imgs) return fail(XRT_EINVAL, "NULL image list");
    for (int64_t k = 0; k < n_img; ++k)
        if (!host_dev_imgs[k]) return fail(XRT_EINVAL, "image %lld is NULL", (long long)k);
    const int64_t n_pix = (int64_t)acc_nf * acc_ns;
    for (int64_t k0 = 0; k0 < n_img; k0 += xrt::ADD_BATCH) {
        xrt::AddBatch b;
        std::memset(&b, 0, sizeof b);
        const int n = (int)std::min<int64_t>(xrt::ADD_BATCH, n_img - k0);
        for (int k = 0; k < n; ++k) b.img[k] = host_dev_imgs[k0 + k];
        const hipError_t e = xrt::launch_add_images(dev_acc, n_pix, b, n, img_dtype == XRT_F64, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "xrt_add_images");
    }
    return XRT_OK;
}

xrt_status xrt_trace_terms(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal,
                           int64_t n, const int32_t *host_idx, double *host_S, double *host_h)
{
    xrt_status st;
    if ((st = check_detector(det)) || (st = check_beam(beam)) || (st = check_crystal(xtal))) return st;
    if (n < 0 || n > (1 << 24)) return fail(XRT_ERANGE, "n must be in [0, 2^24]");
    if (n == 0) return XRT_OK;
    if (!host_idx || !host_S || !host_h) return fail(XRT_EINVAL, "NULL array");
    const int O = det->oversample, nrot = xtal->n_phi * xtal->n_mos;
    for (int64_t q = 0; q < n; ++q) {
        const int32_t *e = host_idx + 6 * q;
        if (e[0] < 0 || e[0] >= det->n_fast || e[1] < 0 || e[1] >= det->n_slow || e[2] < 0 ||
            e[2] >= O * O || e[3] < 0 || e[3] >= det->n_layers || e[4] < 0 || e[4] >= beam->n_src ||
            e[5] < 0 || e[5] >= nrot)
            return fail(XRT_ERANGE, "term %lld: index out of range", (long long)q);
    }
    const size_t n_rot = (size_t)nrot;
    const size_t n_words = 9 * n_rot + xrt::SRC_STRIDE * (size_t)beam->n_src;
    std::vector<double> host(n_words);
    build_cell_mats(xtal, host.data());
    build_sources(beam, host.data() + 9 * n_rot);
    xrt::Params p;
    fill_params(det, beam, xtal, p);

    double *tables = nullptr, *dS = nullptr, *dh = nullptr;
    int32_t *didx = nullptr;
    hipError_t e = hipMalloc((void **)&tables, sizeof(double) * n_words);
    if (e == hipSuccess) e = hipMalloc((void **)&dS, sizeof(double) * 3 * n);
    if (e == hipSuccess) e = hipMalloc((void **)&dh, sizeof(double) * 3 * n);
    if (e == hipSuccess) e = hipMalloc((void **)&didx, sizeof(int32_t) * 6 * n);
    if (e == hipSuccess) e = hipMemcpy(tables, host.data(), sizeof(double) * n_words, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(didx, host_idx, sizeof(int32_t) * 6 * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        p.mats = tables;
        p.src = tables + 9 * n_rot;
        e = xrt::launch_trace(p, n, didx, dS, dh, nullptr);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(host_S, dS, sizeof(double) * 3 * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(host_h, dh, sizeof(double) * 3 * n, hipMemcpyDeviceToHost);
    (void)hipFree(tables);
    (void)hipFree(dS);
    (void)hipFree(dh);
    (void)hipFree(didx);
    if (e != hipSuccess) return hip_fail(e, "xrt_trace_terms");
    return XRT_OK;
}

xrt_status xrt_exp(const double *dev_x, int64_t n, double *dev_y, void *stream)
{
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(XRT_ERANGE, "n must be in [0, 2^40]");
    if (n == 0) return XRT_OK;
    if (!dev_x || !dev_y) return fail(XRT_EINVAL, "NULL array");
    const hipError_t e = xrt::launch_exp(dev_x, n, dev_y, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "xrt_exp");
    return XRT_OK;
}

xrt_status xrt_sinpi(const double *dev_x, int64_t n, double *dev_s64, float *dev_s32, void *stream)
{
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(XRT_ERANGE, "n must be in [0, 2^40]");
    if (n == 0) return XRT_OK;
    if (!dev_x || (!dev_s64 && !dev_s32)) return fail(XRT_EINVAL, "NULL array");
    const hipError_t e = xrt::launch_sinpi(dev_x, n, dev_s64, dev_s32, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "xrt_sinpi");
    return XRT_OK;
}

}  // extern "C"
