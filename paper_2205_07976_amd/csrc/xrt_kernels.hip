// xrt_kernels.hip -- HIP kernels of libxrt for CDNA4 (gfx950).
//
// The spots kernel (paper section III: the kernel that forms the Bragg spots
// from crystal orientation, mosaicity and photon energy) is a VALU-bound loop:
// per pixel term it computes h = M S, the reduced arguments, six sinpi
// polynomials, one division and one structure-factor gather, with no reuse
// that a matrix core could exploit.  Layout decisions:
//
//  * one pixel per lane, 8 x 8 pixels per wave, 16 x 16 per 256-lane
//    workgroup: neighbouring pixels have nearly equal h, so one gather of a
//    wave touches a handful of table lines;
//  * workgroup ids are remapped so that each of the 8 XCDs (dispatched
//    round-robin) gets one contiguous band of tiles and keeps the part of the
//    F^2 table its band needs in its own L2 (a small effect: the vector L1
//    already serves nearly every gather);
//  * the per-shot tables (cell matrices, sources) are indexed by loop
//    counters that are the same for the whole wave, so the standalone kernel
//    reads them with scalar loads into SGPRs (the persistent served kernel
//    stages them in LDS);
//  * loop order: sub-pixel and layer (geometry in binary64), source (S, P),
//    then the inner loop over spindle steps and mosaic domains, which is the
//    hot loop; the per-pixel result is stored once, coalesced per row;
//  * small regions split each pixel's outer iterations into parts summed by
//    different workgroups and added in part order afterwards.
//
// The file is compiled with -ffp-contract=off: S and h follow a fixed
// operation sequence (below), and every fused multiply-add is explicit.
#include "xrt_internal.h"
#include "xrt_math.h"

namespace xrt {

constexpr int TILE = 16;  // pixels per tile edge
constexpr int BLOCK = 256;

// ---------------------------------------------------------------------------
// Sample-point geometry, binary64, fixed operation order:
//   Fp = ((double)i_f + ((double)v + 0.5) / O) * pixel - beam_f  (Sp likewise)
//   r_i = (Fp fdet_i + Sp sdet_i) + (distance + t dt) odet_i
//   R = sqrt((r0 r0 + r1 r1) + r2 r2);  d_i = r_i / R
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sample_dir(const Params &p, int i_f, int i_s, int u, int v, int t,
                                           double d[3], double &R)
{
    const double O = (double)p.O;
    const double Fp = ((double)i_f + ((double)v + 0.5) / O) * p.pixel - p.beam_f;
    const double Sp = ((double)i_s + ((double)u + 0.5) / O) * p.pixel - p.beam_s;
    const double L = p.distance + (double)t * p.layer_dt;
    double r[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) r[i] = (Fp * p.fdet[i] + Sp * p.sdet[i]) + L * p.odet[i];
    R = __builtin_sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) d[i] = r[i] / R;
}

// dOmega * capture of a sample point: solid angle of the full pixel area
// (sub-pixels are averaged by the final 1/O^2) times the Beer-Lambert
// fraction absorbed in layer t, written exp(-a) (1 - exp(-(b - a))) with
// expm1 so that thin layers keep their relative accuracy.  The library's own
// exp and expm1 (xrt_math.h) rather than the device libm's: those carry
// special-case paths whose registers set the high-water mark of every kernel
// that evaluates a sample point (115 against 75 VGPRs in the binary64 spots
// kernel), for arguments that never occur here.
__device__ __forceinline__ double sample_weight(const Params &p, const double d[3], double R, int t)
{
    const double cosrho = (d[0] * p.odet[0] + d[1] * p.odet[1]) + d[2] * p.odet[2];
    const double domega = p.pixel * p.pixel * cosrho / (R * R);
    if (p.layer_dt == 0.0) return domega;
    const double l = p.atten_len * cosrho;
    return domega * exp_cw_f64(-(double)t * p.layer_dt / l) * -expm1_f64(-p.layer_dt / l);
}

// S = (d - dir_j) / lambda_j, binary64.
__device__ __forceinline__ void scatter(const double *src, const double d[3], double S[3])
{
    const double lam = src[SRC_LAMBDA];
#pragma unroll
    for (int i = 0; i < 3; ++i) S[i] = (d[i] - src[SRC_DIR + i]) / lam;
}

// Kahn factor with x = d.e_perp, y = d.(dir x e_perp): for a unit d,
// cos 2psi sin^2 2theta = x^2 - y^2, so P = (1 + c^2 - K (x^2 - y^2)) / 2.
__device__ __forceinline__ double polarization(const double *src, const double d[3], double K)
{
    const double c = (d[0] * src[SRC_DIR] + d[1] * src[SRC_DIR + 1]) + d[2] * src[SRC_DIR + 2];
    const double x = (d[0] * src[SRC_E] + d[1] * src[SRC_E + 1]) + d[2] * src[SRC_E + 2];
    const double y = (d[0] * src[SRC_B] + d[1] * src[SRC_B + 1]) + d[2] * src[SRC_B + 2];
    return 0.5 * (1.0 + c * c - K * (x * x - y * y));
}

// h_i = fma(M_i2, S_2, M_i0 S_0 + M_i1 S_1)
__device__ __forceinline__ void miller(const double *M, const double S[3], double h[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
        h[i] = __builtin_fma(M[3 * i + 2], S[2], M[3 * i] * S[0] + M[3 * i + 1] * S[1]);
}

// h_i = fma(M_i2, S_2, fma(M_i1, S_1, M_i0 S_0)): the mixed form, which has
// no bit-exact contract with the oracle, forms h in binary64 with three
// operations per index instead of four (the same accuracy: two roundings
// fewer).  Negating M negates h exactly, as in miller.
__device__ __forceinline__ void miller_fused(const double *M, const double S[3], double h[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
        h[i] = __builtin_fma(M[3 * i + 2], S[2], __builtin_fma(M[3 * i + 1], S[1], M[3 * i] * S[0]));
}

// Byte offset of the nearest reflection h0 in a padded F^2 table, from the
// rounded indices hr (exact small integers in binary64):
//   x = off + hr_c + hr_b*sb + hr_a*sa,   off = 2^B + (index of h0 = 0)
// by one addition and two FMAs, each with one scalar operand (no register
// copies).  Every partial sum is an integer below 2^51, so x is exact; for an
// element index i in [0, 2^28), x = 2^B + i has the exponent of 2^B and a
// mantissa field of i * 2^(52-B): with B = 49 the low 32 bits of x are 8 i,
// the byte offset of a binary64 entry, with B = 50 they are 4 i, that of a
// binary32 entry -- no float-to-int conversions.  CLAMP moves indices outside
// the padded box onto its border layer (F_default^2); without it the host has
// proven every h0 of the shot inside.
template <bool CLAMP>
__device__ __forceinline__ uint32_t table_offset(const Params &p, const double hr[3], double off)
{
    double v[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        v[i] = CLAMP ? __builtin_fmin(__builtin_fmax(hr[i], p.lo_d[i]), p.hi_d[i]) : hr[i];
    double x = v[2] + off;
    x = __builtin_fma(v[1], p.sb, x);
    x = __builtin_fma(v[0], p.sa, x);
    return (uint32_t)__builtin_bit_cast(uint64_t, x);
}

// Gathers through a buffer resource: a 32-bit offset per lane, no 64-bit
// address arithmetic, and the hardware range check returns 0 (never a fault)
// for an offset past the table.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t table_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ double load_f64(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

__device__ __forceinline__ float load_f32(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

// x in a vector register, opaque to the compiler.  A loop constant that an
// instruction needs in a vector register (its other constant operand takes
// the one scalar read an instruction has) is otherwise moved there again on
// every pass; passed through this once before the loop, it stays in one
// register.  Not volatile: a volatile asm statement counts as a memory side
// effect, and the loops' matrix reads would then leave the scalar cache.
__device__ __forceinline__ double vreg(double x)
{
    asm("" : "+v"(x));
    return x;
}

// 1 / d for the lattice ratio: the hardware reciprocal (relative error below
// 2^-24 on gfx950, measured 2^-24.4) and one Newton step, which squares that
// error: below 2^-48, plus a rounding.  The ratio q = n (1/d) then carries a
// relative error under 6e-15, and the term q^2 under 1.2e-14, far inside the
// 1e-12 pixel tolerance.  The lattice factor is not part of the bit-exact
// S/h sequence.
__device__ __forceinline__ double recip_newton(double d)
{
    const double r = __builtin_amdgcn_rcp(d);
    return __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
}

// ---------------------------------------------------------------------------
// One term F^2 L^2, binary64, added into s: s + (F^2 q) q for the sincg
// ratio q, s + F^2 L^2 for the Gaussian factor L^2 (one FMA each).
//
// The sincg ratio prod_i sin(pi g_i) / prod_i sin(pi f_i), with f = h - rint(h)
// and g = N f - rint(N f), is even in each f_i, so the signed f serves.  It is
// 0/0 when some f_i is exactly 0 (h_i an integer, e.g. S = 0 on the direct
// beam), where the lattice factor takes its limit N_i^2.  FLOORED = false
// evaluates the ratio as it stands: an exact zero gives NaN (0 times the
// infinite reciprocal), which the caller detects on the finished sum and
// answers by summing again with FLOORED = true, where |f| is replaced by
// max(|f|, 2^-32) and the ratio is within 3.3 N^2 2^-64 of its limit.  Any
// other f is at least ulp(h) (|h| >= 1/2) or, for |h| < 1/2, a product of
// matrix entries and a nonzero S component, so the denominator stays far
// above the binary64 underflow and the unfloored value is the better one.
// ---------------------------------------------------------------------------
template <int SHAPE, bool CLAMP, bool FLOORED>
__device__ __forceinline__ double term_f64_add(const Params &p, __amdgpu_buffer_rsrc_t tab, const double h[3],
                                               double s, double c6 = SINPI_C6, double e0 = 0.0,
                                               double c5 = EXP_C5)
{
    double hr[3];
    if (SHAPE == XRT_SHAPE_SINCG) {
        double num = 1.0, den = 1.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            hr[i] = __builtin_rint(h[i]);
            const double f = FLOORED ? __builtin_fmax(__builtin_fabs(h[i] - hr[i]), F_FLOOR) : h[i] - hr[i];
            const double t = p.N[i] * f;
            const double g = t - __builtin_rint(t);
            num *= sinpi_reduced(g, c6);
            den *= sinpi_reduced(f, c6);
        }
        const double q = num * recip_newton(den);
        const double F2 = load_f64(tab, table_offset<CLAMP>(p, hr, p.off64));
        return __builtin_fma(F2 * q, q, s);
    } else {
        double e = e0;  // ln(Na^2 Nb^2 Nc^2), held in a register by the caller's loop
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            hr[i] = __builtin_rint(h[i]);
            const double f = h[i] - hr[i];
            e = __builtin_fma(-p.gk[i], f * f, e);
        }
        const double F2 = load_f64(tab, table_offset<CLAMP>(p, hr, p.off64));
        return __builtin_fma(F2, exp_f64(e, c5), s);
    }
}

// One sincg term, mixed: h, f and g in binary64 (they decide the
// conditioning), everything after the reduced arguments in binary32.  As in
// term_f64_add, FLOORED = false takes the signed f as it stands; ok is false
// when the binary32 denominator is below 2^-100 (an exact integer index gives
// 0, and denominators in the binary32 denormal range have lost precision),
// and the caller then sums again with FLOORED = true.
template <bool CLAMP, bool FLOORED>
__device__ __forceinline__ float term_mixed_sincg(const Params &p, __amdgpu_buffer_rsrc_t tab, const double h[3],
                                                  bool &ok)
{
    double hr[3];
    float num = 1.0f, den = 1.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        hr[i] = __builtin_rint(h[i]);
        const double fa = FLOORED ? __builtin_fmax(__builtin_fabs(h[i] - hr[i]), F_FLOOR) : h[i] - hr[i];
        const double t = p.N[i] * fa;
        const float g = (float)(t - __builtin_rint(t));
        const float f = (float)fa;
        num *= sinpi_reduced(g);
        den *= sinpi_reduced(f);
    }
    ok = __builtin_fabsf(den) >= 0x1p-100f;
    const float q = num * __builtin_amdgcn_rcpf(den);
    return load_f32(tab, table_offset<CLAMP>(p, hr, p.off32)) * (q * q);
}

// The Gaussian lattice exponent e = ln(Na^2 Nb^2 Nc^2) - sum_i gk_i f_i^2 of
// h, in binary64 (the same sequence as the binary64 term), with the rounded
// indices hr and the reduced arguments f; e0 is ln(Na^2 Nb^2 Nc^2).
__device__ __forceinline__ double gauss_exponent(const Params &p, const double h[3], double hr[3], double f[3],
                                                 double e0)
{
    double e = e0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        hr[i] = __builtin_rint(h[i]);
        f[i] = h[i] - hr[i];
        e = __builtin_fma(-p.gk[i], f[i] * f[i], e);
    }
    return e;
}

// Mixed Gaussian sums: the exponents of the terms of one (sample point,
// source) span hundreds of e-folds (down to about -950 at N = 20 far from a
// spot), beyond the binary32 range and beyond what a binary32 exponent
// resolves (its rounding at |e| = 500 alone is a relative 3e-5).  The sum
// therefore keeps a reference exponent m in binary64 and adds the binary32
// terms F^2 exp(e - m): m is the exponent of the first term with a nonzero
// F^2 and is raised to a later such term's exponent when that exceeds it by
// more than GAUSS_REF_STEP, the sum so far being rescaled by exp(m_old - m).
// So the rounded (float)(e - m) of every term that matters is below the
// step in magnitude (an error of at most 2^-21 in the exponent), no term
// exceeds F^2 e^8, and a term is lost to the binary32 range only when it is
// more than e^87 below the reference.  Terms with F^2 = 0 never move m (their
// exponent is clamped to the step, so 0 * exp stays 0).  The value of the
// sum is exp(m) (s - c), formed in binary64 by the binary64 term's exp.
//
// A raise is rare (the first term with a nonzero F^2, then a few more), so
// the loops over the terms test for it with one comparison against the
// threshold mt = m + GAUSS_REF_STEP and leave their inner loop when some lane
// of the wave needs it (a wave-uniform exit); the raise, with its exponential,
// is made outside the inner loop and the loop resumes.  Each lane does the
// same operations in the same order as if the test were made term by term.
constexpr float GAUSS_REF_STEP = 8.0f;

struct GaussRef {
    double m = -__builtin_inf();
    double mt = -__builtin_inf();  // m + GAUSS_REF_STEP
    __device__ __forceinline__ bool needs_raise(double e, float F2) const { return F2 > 0.0f && e > mt; }
    // m := e; returns the factor exp(m_old - e) of the sums so far (0 for
    // the first raise, from m_old = -inf)
    __device__ __forceinline__ float raise(double e)
    {
        const float k = __expf((float)(m - e));
        m = e;
        mt = e + (double)GAUSS_REF_STEP;
        return k;
    }
};

__device__ __forceinline__ void kahan_add(float &s, float &c, float x)
{
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Workgroup id -> tile id: XCD x (workgroups x, x+8, x+16, ...) gets the
// contiguous range of tiles [start(x), start(x) + count(x)).
__device__ __forceinline__ int xcd_tile(int bid, int n_tiles)
{
    const int q = n_tiles >> 3, r = n_tiles & 7;
    const int x = bid & 7, k = bid >> 3;
    return x * q + (x < r ? x : r) + k;
}

// The pixel of this lane: workgroup -> (ROI, tile) through the XCD banding,
// lane -> 8 x 8 block of its wave.  Lanes past a ROI edge trace the ROI's
// last valid pixel (so loops stay uniform) and store nothing.
struct Pixel {
    int i_f, i_s;
    bool live;
    size_t out;  // element index in the [n_roi][roi_ns][roi_nf] output
};

__device__ __forceinline__ Pixel tile_pixel(const Params &p, int tile)
{
    const int roi = tile / p.tiles_per_roi, t = tile - roi * p.tiles_per_roi;
    const int tf = t % p.tiles_f, ts = t / p.tiles_f;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lf = tf * TILE + (wave & 1) * 8 + (lane & 7);
    const int ls = ts * TILE + (wave >> 1) * 8 + (lane >> 3);
    Pixel px;
    px.live = lf < p.roi_nf && ls < p.roi_ns;
    px.i_f = p.origins[2 * roi] + (lf < p.roi_nf ? lf : p.roi_nf - 1);
    px.i_s = p.origins[2 * roi + 1] + (ls < p.roi_ns ? ls : p.roi_ns - 1);
    px.out = ((size_t)roi * p.roi_ns + ls) * p.roi_nf + lf;
    return px;
}

// The spindle x domain sum of one (sample point, source), terms in the order
// r = 0, 1, ..., n_rot - 1: a plain binary64 sum, or a Kahan-compensated
// binary32 one in the mixed form.
template <int PREC, int SHAPE, bool CLAMP>
struct RotSum {
    static constexpr bool KAHAN_SINCG = PREC == XRT_MIXED && SHAPE == XRT_SHAPE_SINCG;
    static constexpr bool GAUSS64 = PREC == XRT_FP64 && SHAPE == XRT_SHAPE_GAUSS;
    double s64 = 0.0;
    float s = 0.0f, c = 0.0f;
    bool redo = false;  // mixed sincg: some term needs the floored ratio
    double c6 = SINPI_C6;  // binary64 sincg: sinpi_over_x's c6, set by rot_loop
    double c5 = EXP_C5;    // binary64 Gaussian: exp_f64's c5, set by rot_loop
    double e0 = 0.0;       // Gaussian: ln(Na^2 Nb^2 Nc^2), set by the term loops
    GaussRef ref;  // mixed Gaussian: reference exponent
    // h = M S by the sequence of this precision
    static __device__ __forceinline__ void hkl(const double M[9], const double S[3], double h[3])
    {
        if constexpr (PREC == XRT_FP64)
            miller(M, S, h);
        else
            miller_fused(M, S, h);
    }
    template <bool FLOORED = false>
    __device__ __forceinline__ void add(const Params &p, __amdgpu_buffer_rsrc_t tab, const double M[9],
                                        const double S[3])
    {
        double h[3];
        hkl(M, S, h);
        add_h<FLOORED>(p, tab, h);
    }
    template <bool FLOORED = false>
    __device__ __forceinline__ void add_h(const Params &p, __amdgpu_buffer_rsrc_t tab, const double h[3])
    {
        if constexpr (PREC == XRT_FP64) {
            s64 = term_f64_add<SHAPE, CLAMP, FLOORED>(p, tab, h, s64, c6, e0, c5);
        } else if constexpr (SHAPE == XRT_SHAPE_SINCG) {
            bool ok;
            kahan_add(s, c, term_mixed_sincg<CLAMP, FLOORED>(p, tab, h, ok));
            if (!FLOORED) redo |= !ok;
        } else {
            double e;
            float F2;
            gauss_term(p, tab, h, e0, e, F2);
            if (ref.needs_raise(e, F2)) rescale(ref.raise(e));
            add_gauss(e, F2);
        }
    }
    // Mixed Gaussian: the exponent and F^2 of the term at h; the sums scaled
    // by k; the term F^2 exp(e - m) added.
    static __device__ __forceinline__ void gauss_term(const Params &p, __amdgpu_buffer_rsrc_t tab, const double h[3],
                                                      double e0, double &e, float &F2)
    {
        double hr[3], f[3];
        e = gauss_exponent(p, h, hr, f, e0);
        F2 = load_f32(tab, table_offset<CLAMP>(p, hr, p.off32));
    }
    __device__ __forceinline__ void rescale(float k)
    {
        s *= k;
        c *= k;
    }
    __device__ __forceinline__ void add_gauss(double e, float F2)
    {
        kahan_add(s, c, F2 * __expf(__builtin_fminf((float)(e - ref.m), GAUSS_REF_STEP)));
    }
    // The sum in binary64 (mixed Gaussian: exp(m) (s - c)).
    __device__ __forceinline__ double value() const
    {
        if constexpr (PREC == XRT_FP64)
            return s64;
        else if constexpr (SHAPE == XRT_SHAPE_SINCG)
            return (double)(s - c);
        else
            return exp_f64(ref.m) * (double)(s - c);
    }
};

__device__ __forceinline__ void load9(double m[9], const double *src)
{
#pragma unroll
    for (int q = 0; q < 9; ++q) m[q] = src[q];
}

// The plain sum over r of the terms at h = M_r S.
template <bool FLOORED, bool PF, class Acc>
__device__ __forceinline__ void rot_loop(const Params &p, __amdgpu_buffer_rsrc_t tab, const double *mats,
                                         const double S[3], Acc &acc)
{
    const int n = p.n_rot;
    acc.c6 = vreg(SINPI_C6);
    acc.c5 = vreg(EXP_C5);
    acc.e0 = vreg(p.ln_n2);
    if (PF) {
        double m[9];
        load9(m, mats);
        for (int r = 0; r < n; ++r) {
            double h[3];
            acc.hkl(m, S, h);
            load9(m, mats + 9 * (r + 1 < n ? r + 1 : r));
            acc.template add_h<FLOORED>(p, tab, h);
        }
    } else if constexpr (Acc::KAHAN_SINCG) {
        // by two: the Kahan sum's registers then alternate instead of being
        // copied back once per term
#pragma unroll 2
        for (int r = 0; r < n; ++r) acc.template add<FLOORED>(p, tab, mats + 9 * r, S);
    } else if constexpr (Acc::GAUSS64) {
        // two terms per pass, written out (the exponential's inline asm keeps
        // the compiler from unrolling): their Horner chains interleave
        // instead of waiting out each other's dependent steps; the sum takes
        // the terms in the same order
        int r = 0;
        for (; r + 1 < n; r += 2) {
            acc.template add<FLOORED>(p, tab, mats + 9 * r, S);
            acc.template add<FLOORED>(p, tab, mats + 9 * (r + 1), S);
        }
        if (r < n) acc.template add<FLOORED>(p, tab, mats + 9 * r, S);
    } else {
        for (int r = 0; r < n; ++r) acc.template add<FLOORED>(p, tab, mats + 9 * r, S);
    }
}

// Without PF the matrix of term r is read where it is used (scalar loads in
// the standalone kernel).  With PF (tables in LDS) the matrix of term r is
// dead once h = M S is formed, so the reads of matrix r + 1 are issued into
// the same registers right then and complete while the rest of term r is
// evaluated: one register set, no copies between terms.
template <int PREC, int SHAPE, bool CLAMP, bool PF>
__device__ __forceinline__ void rot_sum(const Params &p, __amdgpu_buffer_rsrc_t tab, const double *mats,
                                        const double S[3], RotSum<PREC, SHAPE, CLAMP> &acc)
{
    const int n = p.n_rot;
    if constexpr (PREC == XRT_MIXED && SHAPE == XRT_SHAPE_GAUSS) {
        // the inner loop runs until some lane must raise its reference
        // exponent at term r (wave-uniform exit); the raise and term r are
        // done outside it
        double m[9];
        if (PF) load9(m, mats);
        acc.e0 = vreg(p.ln_n2);
        int r = 0;
        while (r < n) {
            double e = 0.0;
            float F2 = 0.0f;
            bool need = false;
            for (; r < n; ++r) {
                double h[3];
                if (PF) {
                    acc.hkl(m, S, h);
                    load9(m, mats + 9 * (r + 1 < n ? r + 1 : r));
                } else {
                    acc.hkl(mats + 9 * r, S, h);
                }
                acc.gauss_term(p, tab, h, acc.e0, e, F2);
                need = acc.ref.needs_raise(e, F2);
                if (__builtin_amdgcn_ballot_w64(need)) break;
                acc.add_gauss(e, F2);
            }
            if (r == n) break;
            if (need) acc.rescale(acc.ref.raise(e));
            acc.add_gauss(e, F2);
            ++r;
        }
        return;
    }
    rot_loop<false, PF>(p, tab, mats, S, acc);
    // a term with an exact integer index on this lane (0/0), or a binary32
    // denominator below 2^-100: the sum again with the floored ratio
    // (term_f64_add, term_mixed_sincg)
    if constexpr (PREC == XRT_FP64 && SHAPE == XRT_SHAPE_SINCG) {
        if (!__builtin_isfinite(acc.s64)) {
            acc.s64 = 0.0;
            rot_loop<true, PF>(p, tab, mats, S, acc);
        }
    } else if constexpr (SHAPE == XRT_SHAPE_SINCG) {
        if (acc.redo) {
            acc.s = acc.c = 0.0f;
            rot_loop<true, PF>(p, tab, mats, S, acc);
        }
    }
}

// The running state of one pixel's sum over its outer iterations: binary64,
// or for mixed sincg a Kahan-compensated binary32 sum (value s - c).  Carried
// from one run of pixel_run to the next, it continues the sum exactly as one
// uninterrupted run would.
struct PixelAcc {
    double acc64 = 0.0;
    float acc = 0.0f, accc = 0.0f;
};

template <int PREC, int SHAPE>
__device__ __forceinline__ double pixel_value(const PixelAcc &st)
{
    return PREC == XRT_MIXED && SHAPE == XRT_SHAPE_SINCG ? (double)(st.acc - st.accc) : st.acc64;
}

// The state as 8 bytes (binary64 sum, or the two binary32 words) and back.
template <int PREC, int SHAPE>
__device__ __forceinline__ uint64_t pixel_pack(const PixelAcc &st)
{
    if constexpr (PREC == XRT_MIXED && SHAPE == XRT_SHAPE_SINCG)
        return (uint64_t)__builtin_bit_cast(uint32_t, st.acc) | ((uint64_t)__builtin_bit_cast(uint32_t, st.accc) << 32);
    else
        return __builtin_bit_cast(uint64_t, st.acc64);
}

template <int PREC, int SHAPE>
__device__ __forceinline__ void pixel_unpack(PixelAcc &st, uint64_t v)
{
    if constexpr (PREC == XRT_MIXED && SHAPE == XRT_SHAPE_SINCG) {
        st.acc = __builtin_bit_cast(float, (uint32_t)v);
        st.accc = __builtin_bit_cast(float, (uint32_t)(v >> 32));
    } else {
        st.acc64 = __builtin_bit_cast(double, v);
    }
}

// The per-pixel sum of pixel (i_f, i_s), not normalised, over the part
// [q0, q1) of its outer iterations q = ((u O + v) T + t) n_src + j (sub-pixel
// (u, v), layer t, source j), each summing all spindle x domain terms, added
// into the running state st.  The whole range [0, O^2 T n_src) from a zero
// state runs the loops in the order of the plain sum.  mats and src are the
// shot's tables (global memory for the standalone kernel, LDS for the served
// one); the arithmetic is the same in both, so a shot gives the same bits
// through either path.  PF (tables in LDS): the next spindle x domain matrix
// is read while the current term is evaluated, so the LDS latency is hidden
// behind one term instead of stalling every term.
template <int PREC, int SHAPE, bool CLAMP, bool PF = false>
__device__ __forceinline__ void pixel_run(const Params &p, __amdgpu_buffer_rsrc_t tab, const double *mats,
                                          const double *srcs, int i_f, int i_s, int q0, int q1, PixelAcc &st)
{
    const int per_t = p.T, per_v = p.O * p.T;
    int uvt = q0 / p.n_src, j0 = q0 - uvt * p.n_src;
    for (int q = q0; q < q1; ++uvt) {
        const int u = uvt / per_v, v = (uvt - u * per_v) / per_t, t = uvt - u * per_v - v * per_t;
        double d[3], R;
        sample_dir(p, i_f, i_s, u, v, t, d, R);
        const double wgeo = sample_weight(p, d, R, t);
        const int j1 = min(p.n_src, j0 + (q1 - q));
        for (int j = j0; j < j1; ++j) {
            const double *src = srcs + SRC_STRIDE * j;
            double S[3];
            scatter(src, d, S);
            const double w = src[SRC_WEIGHT] * polarization(src, d, p.kahn) * wgeo;
            RotSum<PREC, SHAPE, CLAMP> rs;
            rot_sum<PREC, SHAPE, CLAMP, PF>(p, tab, mats, S, rs);
            // binary64 outer sum, except for mixed sincg (Kahan binary32):
            // the mixed Gaussian sums leave the binary32 range
            if constexpr (PREC == XRT_MIXED && SHAPE == XRT_SHAPE_SINCG)
                kahan_add(st.acc, st.accc, (float)w * (rs.s - rs.c));
            else
                st.acc64 = __builtin_fma(w, rs.value(), st.acc64);
        }
        q += j1 - j0;
        j0 = 0;
    }
}

// The sum over [q0, q1) from a zero state (pixel_run).
template <int PREC, int SHAPE, bool CLAMP, bool PF = false>
__device__ __forceinline__ double pixel_sum(const Params &p, __amdgpu_buffer_rsrc_t tab, const double *mats,
                                            const double *srcs, int i_f, int i_s, int q0, int q1)
{
    PixelAcc st;
    pixel_run<PREC, SHAPE, CLAMP, PF>(p, tab, mats, srcs, i_f, i_s, q0, q1, st);
    return pixel_value<PREC, SHAPE>(st);
}

// Part k of K of the outer iterations: [k n / K, (k + 1) n / K).
__device__ __forceinline__ int part_begin(int k, int K, int n) { return (int)((int64_t)k * n / K); }

// The stored value of a pixel and its store (with the accumulate option).
__device__ __forceinline__ void store_pixel(const Params &p, size_t o, double val)
{
    if (p.out_f64) {
        double *img = (double *)p.image;
        img[o] = p.accumulate ? img[o] + val : val;
    } else {
        float *img = (float *)p.image;
        img[o] = p.accumulate ? img[o] + (float)val : (float)val;
    }
}

// Sum of the K partial sums of one pixel, in part order.
__device__ __forceinline__ double sum_parts(const double *part, int K)
{
    double s = part[0];
    for (int k = 1; k < K; ++k) s += part[(size_t)k * BLOCK];
    return s;
}

// One workgroup per (tile, part): with p.split == 1 the whole sum of every
// pixel of a 16 x 16 tile, stored; with p.split = K > 1, part k of each sum,
// written to p.partial[tile][k][lane] for reduce_kernel.
template <int PREC, int SHAPE, bool CLAMP>
__global__ __launch_bounds__(BLOCK) void spots_kernel(const Params p)
{
    const __amdgpu_buffer_rsrc_t tab = PREC == XRT_FP64 ? table_rsrc(p.F2_64, p.bytes64)
                                                         : table_rsrc(p.F2_32, p.bytes32);
    const int unit = xcd_tile(blockIdx.x, p.n_tiles * p.split);
    const int tile = unit / p.split, k = unit - tile * p.split;
    const Pixel px = tile_pixel(p, tile);
    const int n_outer = p.O * p.O * p.T * p.n_src;
    const double sum = pixel_sum<PREC, SHAPE, CLAMP>(p, tab, p.mats, p.src, px.i_f, px.i_s,
                                                     part_begin(k, p.split, n_outer),
                                                     part_begin(k + 1, p.split, n_outer));
    if (p.split > 1) {
        p.partial[((size_t)tile * p.split + k) * BLOCK + threadIdx.x] = sum;
        return;
    }
    if (px.live) store_pixel(p, px.out, p.norm * sum);
}

// Split sums: each pixel's K partial sums added in part order, normalised,
// stored.
__global__ __launch_bounds__(BLOCK) void reduce_kernel(const Params p)
{
    const int tile = blockIdx.x;
    const Pixel px = tile_pixel(p, tile);
    const double sum = sum_parts(p.partial + (size_t)tile * p.split * BLOCK + threadIdx.x, p.split);
    if (px.live) store_pixel(p, px.out, p.norm * sum);
}

template <int PREC, int SHAPE>
static void launch_one(const Params &p, bool clamp, hipStream_t stream)
{
    dim3 grid(p.n_tiles * p.split), block(BLOCK);
    if (clamp)
        hipLaunchKernelGGL((spots_kernel<PREC, SHAPE, true>), grid, block, 0, stream, p);
    else
        hipLaunchKernelGGL((spots_kernel<PREC, SHAPE, false>), grid, block, 0, stream, p);
    if (p.split > 1) hipLaunchKernelGGL(reduce_kernel, dim3(p.n_tiles), block, 0, stream, p);
}

hipError_t launch_spots(const Params &p, int precision, bool clamp, hipStream_t stream)
{
    if (precision == XRT_FP64) {
        if (p.shape == XRT_SHAPE_SINCG)
            launch_one<XRT_FP64, XRT_SHAPE_SINCG>(p, clamp, stream);
        else
            launch_one<XRT_FP64, XRT_SHAPE_GAUSS>(p, clamp, stream);
    } else {
        if (p.shape == XRT_SHAPE_SINCG)
            launch_one<XRT_MIXED, XRT_SHAPE_SINCG>(p, clamp, stream);
        else
            launch_one<XRT_MIXED, XRT_SHAPE_GAUSS>(p, clamp, stream);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Background of an amorphous scatterer (section III's second kernel: the air
// and water around the crystal).  Per term (sample point, source):
// stol = |d - dir| / (2 lambda), the scattering curve F at stol, and
// w P F^2; no spindle or mosaic loop and no table gather, so it is a short
// VALU-bound kernel with the spots kernel's pixel layout (one pixel per lane,
// a 16 x 16 tile per workgroup).  The curve is staged in LDS as one record
// per interval.  The binary64 source loop reads the next source row while it
// evaluates the current one, so those loads overlap the term; the binary32
// loop, whose terms are shorter, is unrolled by two instead (either form
// loses 6-20 % in the other precision).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double max_r(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float max_r(float a, float b) { return __builtin_fmaxf(a, b); }

// |d - dir| from its square x in [0, 4] (unit vectors), within an ulp or two
// rather than correctly rounded (the curve is continuous, so this moves F by
// as little).  binary64: the hardware reciprocal square root y of
// x + 2^-1000 (the bias keeps x = 0 finite and is far below half an ulp of
// any nonzero x met here), one Goldschmidt step on (x y, y / 2) and one
// Newton correction of the root.  binary32: the hardware square root.
__device__ __forceinline__ double root_small(double x)
{
    x += 0x1p-1000;
    const double y = __builtin_amdgcn_rsq(x);
    double s = x * y, h = 0.5 * y;
    const double r = __builtin_fma(-h, s, 0.5);
    s = __builtin_fma(s, r, s);
    h = __builtin_fma(h, r, h);
    return __builtin_fma(__builtin_fma(-s, s, x), h, s);
}
__device__ __forceinline__ float root_small(float x) { return __builtin_amdgcn_sqrtf(x); }

// One interval of the curve in LDS: its knot, the next knot (NaN after the
// last), F and the slope (0 after the last knot: constant beyond it).
template <typename R>
struct alignas(4 * sizeof(R)) BgKnot {
    R x, xn, y, m;
};
// The curve at s.  The lane keeps the record c of its previous term's
// interval k in registers; successive terms of a pixel (sources of nearby
// wavelength, neighbouring sub-pixels) nearly always stay in it, so a lookup
// is two compares and no LDS read.  Otherwise it walks through the LDS
// records: down while the knot is above s, then up while the next knot is at
// or below s.  s is clamped to the first knot x0, so the downward walk stops
// at 0; the NaN after the last knot compares false, so the upward walk stops
// at n - 1.
template <typename R>
__device__ __forceinline__ R bg_curve(const BgKnot<R> *kt, BgKnot<R> &c, int &k, R x0, R s)
{
    s = max_r(s, x0);
    if (c.x > s || c.xn <= s) {
        while (c.x > s) c = kt[--k];
        while (c.xn <= s) c = kt[++k];
    }
    return fma_r(s - c.x, c.m, c.y);
}

// The fields of one source row that a background term reads (binary64, or
// the binary32 copy with its direction tails lo), held in registers so that
// the source loop can read row j + 1 while it evaluates row j.
template <typename R>
struct BgRow {
    R dir[3], lo[3], e[3], b[3], hil, w;
};

// The binary32 row with direction tails made from a binary64 row, as the
// host makes the standalone kernel's copies: head (float)x, tail
// (float)(x - (double)(float)x).
__device__ __forceinline__ void bg_row32(BgRow<float> &r, const double *src)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double x = src[SRC_DIR + i];
        r.dir[i] = (float)x;
        r.lo[i] = (float)(x - (double)r.dir[i]);
        r.e[i] = (float)src[SRC_E + i];
        r.b[i] = (float)src[SRC_B + i];
    }
    r.hil = (float)src[SRC_HIL];
    r.w = (float)src[SRC_WEIGHT];
}

template <typename R>
__device__ __forceinline__ void bg_row(BgRow<R> &r, const R *src, bool tails)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        r.dir[i] = src[SRC_DIR + i];
        r.lo[i] = tails ? src[SRC32_DIR_LO + i] : R(0);
        r.e[i] = src[SRC_E + i];
        r.b[i] = src[SRC_B + i];
    }
    r.hil = src[SRC_HIL];
    r.w = src[SRC_WEIGHT];
}

// Twice the Kahn factor of one source row, 2P = 1 + c^2 - K (x^2 - y^2) as
// in the spots kernel, by fused products; c = d.dir comes from the square
// q = |d - dir|^2 the curve lookup has formed, c = 1 - q/2 (for unit vectors
// |d - dir|^2 = 2 - 2 d.dir; the norms of d and dir differ from 1 by a few
// units of roundoff, which moves c by as much).  The factor 1/2 is applied
// once per sample point.
template <typename R>
__device__ __forceinline__ R bg_polarization2(const BgRow<R> &s, const R d[3], R K, R q)
{
    const R c = fma_r(R(-0.5), q, R(1));
    const R x = fma_r(d[2], s.e[2], fma_r(d[1], s.e[1], d[0] * s.e[0]));
    const R y = fma_r(d[2], s.b[2], fma_r(d[1], s.b[1], d[0] * s.b[0]));
    return fma_r(-K, fma_r(x, x, -(y * y)), fma_r(c, c, R(1)));
}

template <int PREC>
using BgReal = typename std::conditional<PREC == XRT_FP64, double, float>::type;

// The background sum of pixel (i_f, i_s), not normalised: the loops over
// sub-pixels, layers and sources of the standalone and the served kernels
// alike (kt: the curve records, in LDS or global memory; srcs and srcs32: the
// binary64 rows and their binary32 copies with direction tails), so a pixel
// has the same bits through either.  LEAN (the served kernel, whose register
// budget the spots sum sets): each row is read where it is used, with no
// next-row prefetch or unrolling, and the binary32 rows are made from the
// binary64 ones (srcs32 unused).
template <int PREC, bool LEAN = false>
__device__ __forceinline__ double bg_pixel_sum(const Params &p, const BgKnot<BgReal<PREC>> *kt, const double *srcs,
                                               const float *srcs32, int i_f, int i_s)
{
    using R = BgReal<PREC>;
    int k = 0;              // interval of the previous term
    BgKnot<R> ck = kt[0];   // its record
    const R x0 = ck.x;
    double acc64 = 0.0;
    float acc = 0.0f, accc = 0.0f;
    for (int u = 0; u < p.O; ++u)
        for (int v = 0; v < p.O; ++v)
            for (int t = 0; t < p.T; ++t) {
                double d[3], dist;
                sample_dir(p, i_f, i_s, u, v, t, d, dist);
                const double wgeo = sample_weight(p, d, dist, t);
                if constexpr (PREC == XRT_FP64) {
                    double sub = 0.0;
                    BgRow<double> cur, nxt;
                    bg_row(cur, srcs, false);
                    for (int j = 0; j < p.n_src; ++j) {
                        if (LEAN)
                            bg_row(cur, srcs + SRC_STRIDE * j, false);
                        else
                            bg_row(nxt, srcs + SRC_STRIDE * (j + 1 < p.n_src ? j + 1 : j), false);
                        const double e0 = d[0] - cur.dir[0], e1 = d[1] - cur.dir[1], e2 = d[2] - cur.dir[2];
                        const double q = __builtin_fma(e2, e2, __builtin_fma(e1, e1, e0 * e0));
                        const double F = bg_curve(kt, ck, k, x0, root_small(q) * cur.hil);
                        const double P2 = bg_polarization2(cur, d, p.kahn, q);
                        sub = __builtin_fma(cur.w * P2, F * F, sub);
                        if (!LEAN) cur = nxt;
                    }
                    acc64 = __builtin_fma(0.5 * wgeo, sub, acc64);
                } else {
                    // d - dir cancels near the direct beam: d and dir are
                    // each split into a binary32 head and the binary32 rest,
                    // the heads subtract exactly there (Sterbenz), and the
                    // rests add back what binary64 would have kept
                    const float d32[3] = {(float)d[0], (float)d[1], (float)d[2]};
                    const float dlo[3] = {(float)(d[0] - (double)d32[0]), (float)(d[1] - (double)d32[1]),
                                          (float)(d[2] - (double)d32[2])};
                    float s = 0.0f, c = 0.0f;
#pragma unroll LEAN ? 1 : 2
                    for (int j = 0; j < p.n_src; ++j) {
                        BgRow<float> cur;
                        if (LEAN)
                            bg_row32(cur, srcs + SRC_STRIDE * j);
                        else
                            bg_row(cur, srcs32 + SRC32_STRIDE * j, true);
                        const float e0 = (d32[0] - cur.dir[0]) + (dlo[0] - cur.lo[0]);
                        const float e1 = (d32[1] - cur.dir[1]) + (dlo[1] - cur.lo[1]);
                        const float e2 = (d32[2] - cur.dir[2]) + (dlo[2] - cur.lo[2]);
                        const float q = __builtin_fmaf(e2, e2, __builtin_fmaf(e1, e1, e0 * e0));
                        const float F = bg_curve(kt, ck, k, x0, root_small(q) * cur.hil);
                        const float P2 = bg_polarization2(cur, d32, (float)p.kahn, q);
                        kahan_add(s, c, cur.w * P2 * (F * F));
                    }
                    kahan_add(acc, accc, (float)(0.5 * wgeo) * (s - c));
                }
            }
    return PREC == XRT_FP64 ? acc64 : (double)(acc - accc);
}

template <int PREC>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void background_kernel(const BgParams b)
{
    using R = BgReal<PREC>;
    extern __shared__ double bg_lds[];
    const Params &p = b.p;
    BgKnot<R> *kt = reinterpret_cast<BgKnot<R> *>(bg_lds);  // [n]
    const R *kn;
    if constexpr (PREC == XRT_FP64)
        kn = b.knots64;
    else
        kn = b.knots32;
    for (int i = threadIdx.x; i < b.n_knots; i += BLOCK) {
        BgKnot<R> c;
        c.x = kn[3 * i];
        c.xn = i + 1 < b.n_knots ? kn[3 * i + 3] : R(NAN);
        c.y = kn[3 * i + 1];
        c.m = kn[3 * i + 2];
        kt[i] = c;
    }
    __syncthreads();
    const Pixel px = tile_pixel(p, xcd_tile(blockIdx.x, p.n_tiles));
    const double sum = bg_pixel_sum<PREC>(p, kt, p.src, b.src32, px.i_f, px.i_s);
    if (px.live) store_pixel(p, px.out, p.norm * sum);
}

hipError_t launch_background(const BgParams &b, int precision, hipStream_t stream)
{
    const dim3 grid(b.p.n_tiles), block(BLOCK);
    const size_t n = 4 * (size_t)b.n_knots;
    if (precision == XRT_FP64)
        hipLaunchKernelGGL(background_kernel<XRT_FP64>, grid, block, n * sizeof(double), stream, b);
    else
        hipLaunchKernelGGL(background_kernel<XRT_MIXED>, grid, block, n * sizeof(float), stream, b);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Persistent served-shot kernel (continuous batching).  Workgroups claim
// chunks of tiles from the published ring (a compare-and-swap on the claim
// counter, only below the published tail), stage the chunk's shot descriptor
// and tables in LDS (kept there while the next chunk belongs to the same shot),
// run the same per-pixel sum as the standalone kernel and set the chunk's done
// flag.  Like the standalone kernel, a shot whose every rint(h) the host has
// proven inside the padded table takes the clamp-free table index (both give
// the same bits where the clamp-free one is valid).  Registers: the next
// matrix's LDS reads are in flight during each term in the one register set
// of the current matrix; values that are the same for the whole workgroup
// (descriptor fields, chunk bounds, arena offsets) are moved into scalar
// registers; background chunks read the source rows where they are used and
// make their binary32 copies on the fly (the same values the host makes for
// the standalone kernel); the lane index of the staging and chunk loops is
// opaque to the compiler, so the addresses it forms are not kept through the
// whole kernel.  So the kernel fits 4 waves per SIMD (mixed sincg) or 3 (the
// other forms) without spilling to scratch.  The kernel leaves
// only when the whole device is idle: no workgroup holds a chunk, nothing
// published is unclaimed and no chunk finished for idle_ticks; the first
// workgroup to see that raises the exit flag and all workgroups leave together
// (a later progress call relaunches at full width).  The stop flag ends it once
// nothing published is left.  Every wait is bounded, so the kernel always
// drains.  Every read of descriptor data is a range-checked buffer load of the
// host arena and every image store is bounds-checked against the device arena:
// a malformed descriptor cannot reach memory outside the two arenas.
// ---------------------------------------------------------------------------
// A wave-uniform copy of the fields of an LDS-resident Params that the
// per-pixel sum reads, moved into scalar registers (readfirstlane), so the
// served kernel keeps the register budget of the standalone one.
__device__ __forceinline__ double uni(double x)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, lo | (hi << 32));
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni(uint64_t x)
{
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return lo | (hi << 32);
}

__device__ __forceinline__ Params uniform_params(const Params &s)
{
    Params q;
    q.pixel = uni(s.pixel);
    q.distance = uni(s.distance);
    q.beam_f = uni(s.beam_f);
    q.beam_s = uni(s.beam_s);
    for (int i = 0; i < 3; ++i) {
        q.fdet[i] = uni(s.fdet[i]);
        q.sdet[i] = uni(s.sdet[i]);
        q.odet[i] = uni(s.odet[i]);
        q.N[i] = uni(s.N[i]);
        q.gk[i] = uni(s.gk[i]);
        q.lo_d[i] = uni(s.lo_d[i]);
        q.hi_d[i] = uni(s.hi_d[i]);
    }
    q.layer_dt = uni(s.layer_dt);
    q.atten_len = uni(s.atten_len);
    q.O = uni(s.O);
    q.T = uni(s.T);
    q.n_src = uni(s.n_src);
    q.n_rot = uni(s.n_rot);
    q.roi_nf = uni(s.roi_nf);
    q.roi_ns = uni(s.roi_ns);
    q.tiles_f = uni(s.tiles_f);
    q.ln_n2 = uni(s.ln_n2);
    q.kahn = uni(s.kahn);
    q.norm = uni(s.norm);
    q.sa = uni(s.sa);
    q.sb = uni(s.sb);
    q.off64 = uni(s.off64);
    q.off32 = uni(s.off32);
    q.out_f64 = uni(s.out_f64);
    q.split = uni(s.split);
    return q;
}

// Claim the next published chunk (-1: nothing to claim).  Idle polling uses
// relaxed loads; the acquire that makes a published descriptor visible is
// taken only after a successful claim.
__device__ __forceinline__ long long serve_claim(const ServeArgs &a)
{
    const unsigned long long tail = __hip_atomic_load(&a.ctrl->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    unsigned long long n = __hip_atomic_load(a.next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (n < tail) {
        if (__hip_atomic_compare_exchange_strong(a.next, &n, n + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return (long long)n;
    }
    return -1;
}

template <int PREC, int SHAPE>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(PREC == XRT_MIXED && SHAPE == XRT_SHAPE_SINCG ? 4 : 3))) void serve_kernel(const ServeArgs a)
{
    __shared__ ShotDesc sd;
    __shared__ double smats[9 * SERVE_MAX_ROT];
    __shared__ double ssrc[SRC_STRIDE * SERVE_MAX_SRC];
    __shared__ long long s_claim;
    __shared__ uint64_t s_off, s_have_off;
    __shared__ int32_t s_tile0, s_ntiles, s_kind, s_seg;
    __shared__ uint32_t s_seq1, s_shot, s_have_shot;  // s_have_*: the descriptor now in LDS
    const __amdgpu_buffer_rsrc_t tab = PREC == XRT_FP64 ? table_rsrc(a.F2_64, a.bytes64)
                                                         : table_rsrc(a.F2_32, a.bytes32);
    if (threadIdx.x == 0) {
        s_have_off = ~0ull;
        s_have_shot = 0;
    }
    // idle polling interval, in units of s_sleep(127) (about 3.4 us): one
    // workgroup per XCD (the first eight) polls at most every 16 units, the
    // others at most every 256, so new work is seen within tens of us while
    // idle workgroups stay off the memory paths the busy ones use
    const int max_backoff = blockIdx.x < 8 ? 16 : 256;
    int backoff = 1;
    // the idle time counts from the launch (the host zeroes last_done)
    if (threadIdx.x == 0)
        __hip_atomic_fetch_max(a.last_done, (unsigned long long)__builtin_amdgcn_s_memrealtime(), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (threadIdx.x == 0) {
            long long c = -2;
            if (!__hip_atomic_load(a.exiting, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                // busy counts workgroups holding a claimed chunk; polling does
                // not touch it, so an idle device does see it at zero
                c = serve_claim(a);
                if (c >= 0) {
                    __hip_atomic_fetch_add(a.busy, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const ServeChunk *ch = a.ring + ((uint64_t)c & (SERVE_RING - 1));
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // the chunk and its descriptor
                    s_off = __hip_atomic_load(&ch->desc_off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    s_tile0 = __hip_atomic_load(&ch->tile0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    s_ntiles = __hip_atomic_load(&ch->n_tiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    s_seq1 = __hip_atomic_load(&ch->seq1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    s_shot = __hip_atomic_load(&ch->shot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    s_kind = __hip_atomic_load(&ch->kind, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    s_seg = __hip_atomic_load(&ch->seg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                } else if (__hip_atomic_load(&a.ctrl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
                    c = -2;  // stop is honoured once nothing published is left
                } else {
                    const uint64_t now = __builtin_amdgcn_s_memrealtime();
                    const uint64_t last = __hip_atomic_load(a.last_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (now - last > a.idle_ticks &&
                        __hip_atomic_load(a.busy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                        __hip_atomic_store(a.exiting, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        c = -2;
                    }
                }
            }
            s_claim = c;
        }
        __syncthreads();
        const long long c = s_claim;
        if (c == -2) break;
        if (c == -1) {
            // idle: poll again at a falling rate
            for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(127);
            backoff = backoff < max_backoff ? 2 * backoff : max_backoff;
            __syncthreads();
            continue;
        }
        backoff = 1;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // see the published descriptor
        const uint64_t off = s_off;
        if (off != s_have_off || s_shot != s_have_shot) {
            // a new shot for this workgroup: stage its descriptor and tables
            const bool ok = off < a.hdesc_bytes && (off & 7) == 0;
            const uint64_t room = ok ? a.hdesc_bytes - off : 0;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<char *>(a.hdesc) + (ok ? off : 0), 0, (int)(room < 0x7fffffffull ? room : 0x7fffffffull),
                0x00020000);
            // the lane index as an opaque value: the staging addresses are
            // formed here, not kept in registers through the whole kernel
            int tid = threadIdx.x;
            __asm__ volatile("" : "+v"(tid));
            for (int i = tid; i < (int)(sizeof(ShotDesc) / 4); i += BLOCK)
                reinterpret_cast<uint32_t *>(&sd)[i] = __builtin_amdgcn_raw_buffer_load_b32(rs, 4 * i, 0, 0);
            __syncthreads();
            // bound every loop extent of the descriptor
            const int n_rot = min(max(sd.p.n_rot, 0), SERVE_MAX_ROT);
            const int n_src = min(max(sd.p.n_src, 0), SERVE_MAX_SRC);
            for (int i = tid; i < 9 * n_rot; i += BLOCK)
                smats[i] = load_f64(rs, (uint32_t)(sd.mats_rel + 8 * (uint64_t)i));
            for (int i = tid; i < SRC_STRIDE * n_src; i += BLOCK)
                ssrc[i] = load_f64(rs, (uint32_t)(sd.src_rel + 8 * (uint64_t)i));
            __syncthreads();
            if (threadIdx.x == 0) {
                sd.p.n_rot = n_rot;
                sd.p.n_src = n_src;
                sd.p.O = min(max(sd.p.O, 0), 64);
                sd.p.T = min(max(sd.p.T, 0), 64);
                sd.p.tiles_f = max(sd.p.tiles_f, 1);
                sd.p.split = min(max(sd.p.split, 1), SERVE_MAX_SPLIT);
                s_have_off = off;
                s_have_shot = s_shot;
            }
            __syncthreads();
        }
        const Params p = uniform_params(sd.p);
        const int roi_f0 = uni(sd.roi_f0), roi_s0 = uni(sd.roi_s0);
        const int clamp = uni(sd.clamp);
        const int n_units = uni(min(max(s_ntiles, 0), SERVE_MAX_CHUNK));
        const int tile0 = uni(s_tile0), kind = uni(s_kind);
        const int split = p.split;
        const int n_seg = uni(max(sd.n_seg, 1)), seg = uni(min(max(s_seg, 0), n_seg - 1));
        const uint64_t state = uni(sd.state_off), state_bytes = uni(sd.state_bytes);
        const int n_outer = p.O * p.O * p.T * p.n_src;
        const uint64_t img = uni(sd.image_off), part = uni(sd.partial_off);
        const uint64_t image_bytes = uni(sd.image_bytes), partial_bytes = uni(sd.partial_bytes);
        int ctid = threadIdx.x;  // opaque, as in the staging above
        __asm__ volatile("" : "+v"(ctid));
        for (int i = 0; i < n_units; ++i) {
            // compute chunk: unit = tile * split + part; reduce chunk: unit = tile
            const int unit = tile0 + i;
            const int t = kind == CHUNK_COMPUTE ? unit / split : unit;
            const int k = kind == CHUNK_COMPUTE ? unit - t * split : 0;
            const int tf = t % p.tiles_f, ts = t / p.tiles_f;
            const int lane = ctid & 63, wave = ctid >> 6;
            const int lf = tf * TILE + (wave & 1) * 8 + (lane & 7);
            const int ls = ts * TILE + (wave >> 1) * 8 + (lane >> 3);
            const bool live = lf < p.roi_nf && ls < p.roi_ns;
            // partial sums of this tile and lane: [tile][part][lane] binary64
            const uint64_t pq = part + 8 * (((uint64_t)t * split) * BLOCK + ctid);
            const bool parts_ok = part <= a.arena_bytes && pq + 8 * ((uint64_t)(split - 1) * BLOCK + 1) <= a.arena_bytes &&
                                  8 * (((uint64_t)t * split + split) * BLOCK) <= partial_bytes;
            if (kind == CHUNK_BACKGROUND) {
                // the server's background added into the complete image, as
                // xrt_simulate_background with accumulate does
                if (!a.bg_knots) continue;
                const int i_f = roi_f0 + (lf < p.roi_nf ? lf : p.roi_nf - 1);
                const int i_s = roi_s0 + (ls < p.roi_ns ? ls : p.roi_ns - 1);
                const double bsum = bg_pixel_sum<PREC, true>(p, static_cast<const BgKnot<BgReal<PREC>> *>(a.bg_knots), ssrc,
                                                             nullptr, i_f, i_s);
                const double bval = uni(sd.bg_norm) * bsum;
                const uint64_t besz = p.out_f64 ? 8 : 4;
                const uint64_t bo = besz * ((uint64_t)ls * (uint64_t)p.roi_nf + (uint64_t)lf);
                if (live && bo + besz <= image_bytes && img <= a.arena_bytes && bo + besz <= a.arena_bytes - img) {
                    if (p.out_f64) {
                        double *q = reinterpret_cast<double *>(a.arena + img + bo);
                        *q = *q + bval;
                    } else {
                        float *q = reinterpret_cast<float *>(a.arena + img + bo);
                        *q = *q + (float)bval;
                    }
                }
                continue;
            }
            double sum;
            if (kind == CHUNK_COMPUTE) {
                const int i_f = roi_f0 + (lf < p.roi_nf ? lf : p.roi_nf - 1);
                const int i_s = roi_s0 + (ls < p.roi_ns ? ls : p.roi_ns - 1);
                // segment seg of part k's outer iterations, continuing the
                // running sum the previous segment left in the state slot
                const int q0 = part_begin(k, split, n_outer), q1 = part_begin(k + 1, split, n_outer);
                const int qa = q0 + part_begin(seg, n_seg, q1 - q0), qb = q0 + part_begin(seg + 1, n_seg, q1 - q0);
                const uint64_t so = state + 8 * ((uint64_t)unit * BLOCK + ctid);
                const bool state_ok = n_seg > 1 && state <= a.arena_bytes && so + 8 <= a.arena_bytes &&
                                      8 * ((uint64_t)unit * BLOCK + BLOCK) <= state_bytes;
                PixelAcc st;
                if (seg > 0 && state_ok) pixel_unpack<PREC, SHAPE>(st, *reinterpret_cast<const uint64_t *>(a.arena + so));
                if (clamp)
                    pixel_run<PREC, SHAPE, true, true>(p, tab, smats, ssrc, i_f, i_s, qa, qb, st);
                else
                    pixel_run<PREC, SHAPE, false, true>(p, tab, smats, ssrc, i_f, i_s, qa, qb, st);
                if (seg + 1 < n_seg) {
                    if (state_ok) *reinterpret_cast<uint64_t *>(a.arena + so) = pixel_pack<PREC, SHAPE>(st);
                    continue;
                }
                sum = pixel_value<PREC, SHAPE>(st);
                if (split > 1) {
                    if (parts_ok) *reinterpret_cast<double *>(a.arena + pq + 8 * (uint64_t)k * BLOCK) = sum;
                    continue;
                }
            } else {
                sum = parts_ok ? sum_parts(reinterpret_cast<const double *>(a.arena + pq), split) : 0.0;
            }
            const double val = p.norm * sum;
            const uint64_t esz = p.out_f64 ? 8 : 4;
            const uint64_t o = esz * ((uint64_t)ls * (uint64_t)p.roi_nf + (uint64_t)lf);
            if (live && o + esz <= image_bytes && img <= a.arena_bytes && o + esz <= a.arena_bytes - img) {
                if (p.out_f64)
                    *reinterpret_cast<double *>(a.arena + img + o) = val;
                else
                    *reinterpret_cast<float *>(a.arena + img + o) = (float)val;
            }
        }
        __threadfence_system();
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_store(a.done + ((uint64_t)c & (SERVE_RING - 1)), s_seq1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(a.last_done, (unsigned long long)__builtin_amdgcn_s_memrealtime(), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(a.busy, -1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

static const void *serve_fn(int precision, int shape)
{
    if (precision == XRT_FP64)
        return shape == XRT_SHAPE_SINCG ? (const void *)serve_kernel<XRT_FP64, XRT_SHAPE_SINCG>
                                        : (const void *)serve_kernel<XRT_FP64, XRT_SHAPE_GAUSS>;
    return shape == XRT_SHAPE_SINCG ? (const void *)serve_kernel<XRT_MIXED, XRT_SHAPE_SINCG>
                                    : (const void *)serve_kernel<XRT_MIXED, XRT_SHAPE_GAUSS>;
}

int serve_blocks_per_cu(int precision, int shape)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, serve_fn(precision, shape), BLOCK, 0) != hipSuccess)
        return 0;
    return n;
}

hipError_t launch_serve(const ServeArgs &a, int precision, int shape, int n_wg, hipStream_t stream)
{
    dim3 grid(n_wg), block(BLOCK);
    if (precision == XRT_FP64) {
        if (shape == XRT_SHAPE_SINCG)
            hipLaunchKernelGGL((serve_kernel<XRT_FP64, XRT_SHAPE_SINCG>), grid, block, 0, stream, a);
        else
            hipLaunchKernelGGL((serve_kernel<XRT_FP64, XRT_SHAPE_GAUSS>), grid, block, 0, stream, a);
    } else {
        if (shape == XRT_SHAPE_SINCG)
            hipLaunchKernelGGL((serve_kernel<XRT_MIXED, XRT_SHAPE_SINCG>), grid, block, 0, stream, a);
        else
            hipLaunchKernelGGL((serve_kernel<XRT_MIXED, XRT_SHAPE_GAUSS>), grid, block, 0, stream, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint of the Gaussian-shape sum (the refinement of per-crystal parameters
// against measured images, paper section II).  With g_p = dL/dI_p given, it
// accumulates over every term of every pixel
//   dL/dM0_{i,c} = sum g_p K w P dOmega C F^2 dL2/dh_i (Q^T S)_c,
//   dL/dN_i      = sum g_p K w P dOmega C F^2 dL2/dN_i,
//   dL/dscale    = sum g_p I_p / scale,
// where h_i = M0_i . (Q^T S), Q = umat_m R_k, L2 = prod N_i^2
// exp(-gk_i f_i^2) with gk_i = 2 N_i^2 / c, dL2/dh_i = -2 gk_i f_i L2 and
// dL2/dN_i = (2/N_i) (1 - gk_i f_i^2) L2.  The factors -2 gk_i and 2/N_i
// (and 1/scale) are the same for every term, so the term loops accumulate
// the sums without them (f_i (Q^T S)_c B, (1 - gk_i f_i^2) B and B, with B
// = g_p K w P dOmega C F^2 L2) and the final reduction applies them once.
// The binary64 loop accumulates f_i^2 B in place of (1 - gk_i f_i^2) B, and
// the reduction forms sum B - gk_i sum f_i^2 B (the difference can cancel,
// which costs at most a few binary64 roundings of either sum).
// Each lane owns a pixel; the 13 sums are reduced over the workgroup by a
// fixed tree and then over the workgroups by a fixed-order kernel, so the
// result is deterministic.
// ---------------------------------------------------------------------------
template <bool CLAMP>
__device__ __forceinline__ void grad_term_f64(const Params &p, __amdgpu_buffer_rsrc_t tab, const double *Q,
                                              const double S[3], double w, double acc[13], double e0,
                                              double c5)
{
    double Sp[3], hr[3], f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) Sp[c] = __builtin_fma(Q[6 + c], S[2], __builtin_fma(Q[3 + c], S[1], Q[c] * S[0]));
    double e = e0;  // ln(Na^2 Nb^2 Nc^2)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double h = __builtin_fma(p.m0[3 * i + 2], Sp[2], __builtin_fma(p.m0[3 * i + 1], Sp[1], p.m0[3 * i] * Sp[0]));
        hr[i] = __builtin_rint(h);
        f[i] = h - hr[i];
        e = __builtin_fma(-p.gk[i], f[i] * f[i], e);
    }
    const double base = w * load_f64(tab, table_offset<CLAMP>(p, hr, p.off64)) * exp_f64(e, c5);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double dh = base * f[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[3 * i + c] = __builtin_fma(dh, Sp[c], acc[3 * i + c]);
        acc[9 + i] = __builtin_fma(base, f[i] * f[i], acc[9 + i]);
    }
    acc[12] += base;
}

// Mixed: Q^T S, h, f and the exponent in binary64; the lattice factor, the
// derivatives and the products in binary32, as terms F^2 exp(e - m) against
// the reference exponent m of the forward's mixed Gaussian sums (the 13
// binary32 sums of one (sample point, source) are rescaled with m and added
// into binary64 as exp(m) times their value).  grad_prep_mixed forms what a
// term needs up to its exponent and F^2, grad_add_mixed adds it; the term loop
// raises the reference between the two, as the forward's does.  h is formed
// in binary64 from the forward's lab-frame matrix, h = M S (rows of M are
// Q m0_i, so h_i = m0_i . Q^T S), and the S' = Q^T S that the dL/dM0 sums
// multiply, in binary32 from binary32 copies of Q and S: it enters only the
// binary32 derivative products.
struct GradTerm {
    float f[3], Sf[3];
    double e;
    float F2;
};

template <bool CLAMP>
__device__ __forceinline__ void grad_prep_mixed(const Params &p, __amdgpu_buffer_rsrc_t tab, const double *M,
                                                const float *Q32, const double S[3], const float S32[3], double e0,
                                                GradTerm &g)
{
    double hr[3], fd[3], h[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        g.Sf[c] = __builtin_fmaf(Q32[6 + c], S32[2], __builtin_fmaf(Q32[3 + c], S32[1], Q32[c] * S32[0]));
    miller_fused(M, S, h);
    g.e = gauss_exponent(p, h, hr, fd, e0);
#pragma unroll
    for (int i = 0; i < 3; ++i) g.f[i] = (float)fd[i];
    g.F2 = load_f32(tab, table_offset<CLAMP>(p, hr, p.off32));
}

__device__ __forceinline__ void grad_add_mixed(const Params &p, const GradTerm &g, float w, float acc[13],
                                               const GaussRef &ref)
{
    const float base = w * g.F2 * __expf(__builtin_fminf((float)(g.e - ref.m), GAUSS_REF_STEP));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float dh = base * g.f[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[3 * i + c] = __builtin_fmaf(dh, g.Sf[c], acc[3 * i + c]);
        acc[9 + i] = __builtin_fmaf(base, __builtin_fmaf(-(float)p.gk[i], g.f[i] * g.f[i], 1.0f), acc[9 + i]);
    }
    acc[12] += base;
}

// The 13 binary32 sums of one (sample point, source) over its n_rot terms,
// leaving the inner loop only when some lane must raise its reference
// exponent (as rot_sum does for the forward sums).
template <bool CLAMP>
__device__ __forceinline__ void grad_rot_mixed(const Params &p, __amdgpu_buffer_rsrc_t tab, const double S[3], float w,
                                               float acc[13], GaussRef &ref)
{
    const int n = p.n_rot;
    const float S32[3] = {(float)S[0], (float)S[1], (float)S[2]};
    const double e0 = vreg(p.ln_n2);
    int r = 0;
    while (r < n) {
        GradTerm g;
        bool need = false;
        for (; r < n; ++r) {
            grad_prep_mixed<CLAMP>(p, tab, p.mats + 9 * r, p.qmats32 + 10 * r, S, S32, e0, g);
            need = ref.needs_raise(g.e, g.F2);
            if (__builtin_amdgcn_ballot_w64(need)) break;
            grad_add_mixed(p, g, w, acc, ref);
        }
        if (r == n) break;
        if (need) {
            const float k = ref.raise(g.e);
#pragma unroll
            for (int c = 0; c < 13; ++c) acc[c] *= k;
        }
        grad_add_mixed(p, g, w, acc, ref);
        ++r;
    }
}

// Sum of v over the 256 lanes of a workgroup by a fixed tree: xor-shuffles
// within each wave, then the four wave sums in order.  Valid in lane 0.
__device__ __forceinline__ double block_sum(double v, double *lds)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    return (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

template <int PREC, bool CLAMP>
__global__ __launch_bounds__(BLOCK) void grad_kernel(const Params p, const void *dLdI, int dLdI_f64,
                                                     double *partial)
{
    __shared__ double lds[4];
    const __amdgpu_buffer_rsrc_t tab = PREC == XRT_FP64 ? table_rsrc(p.F2_64, p.bytes64)
                                                         : table_rsrc(p.F2_32, p.bytes32);
    const Pixel px = tile_pixel(p, xcd_tile(blockIdx.x, p.n_tiles));
    double gp = 0.0;
    if (px.live) gp = dLdI_f64 ? ((const double *)dLdI)[px.out] : (double)((const float *)dLdI)[px.out];
    double acc[13];
#pragma unroll
    for (int c = 0; c < 13; ++c) acc[c] = 0.0;
    for (int u = 0; u < p.O; ++u)
        for (int v = 0; v < p.O; ++v)
            for (int t = 0; t < p.T; ++t) {
                double d[3], R;
                sample_dir(p, px.i_f, px.i_s, u, v, t, d, R);
                const double wgeo = gp * p.norm * sample_weight(p, d, R, t);
                for (int j = 0; j < p.n_src; ++j) {
                    const double *src = p.src + SRC_STRIDE * j;
                    double S[3];
                    scatter(src, d, S);
                    const double w = src[SRC_WEIGHT] * polarization(src, d, p.kahn) * wgeo;
                    if (PREC == XRT_FP64) {
                        const double e0 = vreg(p.ln_n2), c5 = vreg(EXP_C5);
                        int r = 0;  // two terms per pass, as in rot_loop
                        for (; r + 1 < p.n_rot; r += 2) {
                            grad_term_f64<CLAMP>(p, tab, p.qmats + 9 * r, S, w, acc, e0, c5);
                            grad_term_f64<CLAMP>(p, tab, p.qmats + 9 * (r + 1), S, w, acc, e0, c5);
                        }
                        if (r < p.n_rot) grad_term_f64<CLAMP>(p, tab, p.qmats + 9 * r, S, w, acc, e0, c5);
                    } else {
                        float a32[13];
#pragma unroll
                        for (int c = 0; c < 13; ++c) a32[c] = 0.0f;
                        GaussRef ref;
                        grad_rot_mixed<CLAMP>(p, tab, S, (float)w, a32, ref);
                        const double em = exp_f64(ref.m);
#pragma unroll
                        for (int c = 0; c < 13; ++c) acc[c] = __builtin_fma(em, (double)a32[c], acc[c]);
                    }
                }
            }
    for (int c = 0; c < 13; ++c) {
        const double s = block_sum(acc[c], lds);
        if (threadIdx.x == 0) partial[13 * (size_t)blockIdx.x + c] = s;
    }
}

// The gradient from the 13 sums s: grad[c] = k[c] s[c], and for the three
// dL/dN_i also + kb[i] s[12] (binary64: k = -2 gk_i / N_i on the sum of
// f_i^2 B, kb = 2/N_i; mixed: k = 2/N_i on the sum of (1 - gk_i f_i^2) B,
// kb = 0).  k is -2 gk_i for dL/dM0 row i and 1/scale for dL/dscale.
struct GradScale {
    double k[13];
    double kb[3];
};

// grad13 from the sums over workgroups b of partial[b][c], each in a fixed
// order: lane t adds b = t, t + 256, ... sequentially, then the fixed block
// tree.
__global__ __launch_bounds__(BLOCK) void grad_reduce_kernel(const double *partial, int n_blocks, double *grad13,
                                                            const GradScale g)
{
    __shared__ double lds[4];
    double s[13];
    for (int c = 0; c < 13; ++c) {
        double v = 0.0;
        for (int b = threadIdx.x; b < n_blocks; b += BLOCK) v += partial[13 * (size_t)b + c];
        s[c] = block_sum(v, lds);
    }
    if (threadIdx.x == 0) {
        for (int c = 0; c < 13; ++c) grad13[c] = s[c] * g.k[c];
        for (int i = 0; i < 3; ++i) grad13[9 + i] = __builtin_fma(g.kb[i], s[12], grad13[9 + i]);
    }
}

template <int PREC>
static void launch_grad_one(const Params &p, bool clamp, const void *dLdI, int f64, double *partial,
                            hipStream_t stream)
{
    if (clamp)
        hipLaunchKernelGGL((grad_kernel<PREC, true>), dim3(p.n_tiles), dim3(BLOCK), 0, stream, p, dLdI, f64, partial);
    else
        hipLaunchKernelGGL((grad_kernel<PREC, false>), dim3(p.n_tiles), dim3(BLOCK), 0, stream, p, dLdI, f64, partial);
}

hipError_t launch_grad(const Params &p, int precision, bool clamp, const void *dLdI, int dLdI_f64,
                       double *partial, double *grad13, double inv_scale, hipStream_t stream)
{
    if (precision == XRT_FP64)
        launch_grad_one<XRT_FP64>(p, clamp, dLdI, dLdI_f64, partial, stream);
    else
        launch_grad_one<XRT_MIXED>(p, clamp, dLdI, dLdI_f64, partial, stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    GradScale g;
    for (int i = 0; i < 3; ++i) {
        for (int c = 0; c < 3; ++c) g.k[3 * i + c] = p.m2gk[i];
        g.k[9 + i] = precision == XRT_FP64 ? -p.gk[i] * p.inv2N[i] : p.inv2N[i];
        g.kb[i] = precision == XRT_FP64 ? p.inv2N[i] : 0.0;
    }
    g.k[12] = inv_scale;
    hipLaunchKernelGGL(grad_reduce_kernel, dim3(1), dim3(BLOCK), 0, stream, partial, p.n_tiles, grad13, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ensemble sum (section III's add-image kernel, which adds the results of the
// other kernels into one binary64 image): a region image of nf x ns pixels,
// binary32 or binary64, added into a binary64 accumulator of acc_nf columns
// at (f0, s0).  Memory-bound: per pixel one image read and one accumulator
// read and write.  Rows are spread over blockIdx.y, columns over lanes, so
// every wave reads and writes 64 consecutive pixels of one row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void add_image_kernel(double *acc, int64_t acc_nf, const void *img, int img_f64,
                                                          int nf, int ns, int f0, int s0)
{
    for (int r = blockIdx.y; r < ns; r += gridDim.y) {
        double *row = acc + (int64_t)(s0 + r) * acc_nf + f0;
        const int64_t base = (int64_t)r * nf;
        for (int c = blockIdx.x * BLOCK + threadIdx.x; c < nf; c += gridDim.x * BLOCK) {
            const double x = img_f64 ? ((const double *)img)[base + c] : (double)((const float *)img)[base + c];
            row[c] = row[c] + x;
        }
    }
}

// The same when the image covers whole accumulator rows (a contiguous run of
// n pixels) and both starts are 16-byte aligned: four pixels per lane and
// step, as one 16-byte image load (binary32; two for binary64) and two
// 16-byte accumulator loads and stores; the n mod 4 last pixels one by one.
__global__ __launch_bounds__(BLOCK) void add_image_flat_kernel(double *acc, const void *img, int img_f64, int64_t n)
{
    const int64_t n4 = n >> 2, stride = (int64_t)gridDim.x * BLOCK;
    double2 *a2 = reinterpret_cast<double2 *>(acc);
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n4; i += stride) {
        double2 x0, x1;
        if (img_f64) {
            const double2 *g = reinterpret_cast<const double2 *>(img);
            x0 = g[2 * i];
            x1 = g[2 * i + 1];
        } else {
            const float4 f = reinterpret_cast<const float4 *>(img)[i];
            x0 = make_double2(f.x, f.y);
            x1 = make_double2(f.z, f.w);
        }
        double2 a0 = a2[2 * i], a1 = a2[2 * i + 1];
        a0.x = a0.x + x0.x;
        a0.y = a0.y + x0.y;
        a1.x = a1.x + x1.x;
        a1.y = a1.y + x1.y;
        a2[2 * i] = a0;
        a2[2 * i + 1] = a1;
    }
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
        const int64_t j = (n4 << 2) + threadIdx.x;
        acc[j] = acc[j] + (img_f64 ? ((const double *)img)[j] : (double)((const float *)img)[j]);
    }
}

hipError_t launch_add_image(double *acc, int64_t acc_nf, const void *img, int img_f64, int32_t nf, int32_t ns,
                            int32_t f0, int32_t s0, hipStream_t stream)
{
    double *start = acc + (int64_t)s0 * acc_nf + f0;
    if (f0 == 0 && nf == acc_nf && ((uintptr_t)start & 15) == 0 && ((uintptr_t)img & 15) == 0) {
        const int64_t n = (int64_t)nf * ns;
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(((n >> 2) + BLOCK - 1) / BLOCK, 8192));
        hipLaunchKernelGGL(add_image_flat_kernel, dim3(grid), dim3(BLOCK), 0, stream, start, img, img_f64, n);
        return hipGetLastError();
    }
    const unsigned bx = (unsigned)std::min<int64_t>((nf + BLOCK - 1) / BLOCK, 64);
    const unsigned by = (unsigned)std::min<int64_t>(ns, 8192);
    hipLaunchKernelGGL(add_image_kernel, dim3(bx, by), dim3(BLOCK), 0, stream, acc, acc_nf, img, img_f64, nf, ns,
                       f0, s0);
    return hipGetLastError();
}

// Many whole images into one accumulator: each lane takes a pixel, reads its
// accumulator value once, adds the images' pixels in image order and writes
// once, so the bits are those of one call per image in the same order while
// the accumulator moves 16 bytes per pixel for the whole batch instead of per
// image.
__global__ __launch_bounds__(BLOCK) void add_images_kernel(double *acc, int64_t n_pix, const AddBatch b, int n_img,
                                                           int img_f64)
{
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n_pix; i += stride) {
        double a = acc[i];
        if (img_f64) {
            for (int k = 0; k < n_img; ++k) a = a + ((const double *)b.img[k])[i];
        } else {
            for (int k = 0; k < n_img; ++k) a = a + (double)((const float *)b.img[k])[i];
        }
        acc[i] = a;
    }
}

// The same with four pixels per lane and 16-byte accesses (every pointer
// 16-byte aligned, binary32 images); the n_pix mod 4 last pixels one by one.
__global__ __launch_bounds__(BLOCK) void add_images4_kernel(double *acc, int64_t n_pix, const AddBatch b, int n_img)
{
    const int64_t n4 = n_pix >> 2, stride = (int64_t)gridDim.x * BLOCK;
    double2 *a2 = reinterpret_cast<double2 *>(acc);
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n4; i += stride) {
        double2 a0 = a2[2 * i], a1 = a2[2 * i + 1];
        for (int k = 0; k < n_img; ++k) {
            const float4 f = reinterpret_cast<const float4 *>(b.img[k])[i];
            a0.x = a0.x + (double)f.x;
            a0.y = a0.y + (double)f.y;
            a1.x = a1.x + (double)f.z;
            a1.y = a1.y + (double)f.w;
        }
        a2[2 * i] = a0;
        a2[2 * i + 1] = a1;
    }
    if (blockIdx.x == 0 && threadIdx.x < (n_pix & 3)) {
        const int64_t j = (n4 << 2) + threadIdx.x;
        double a = acc[j];
        for (int k = 0; k < n_img; ++k) a = a + (double)((const float *)b.img[k])[j];
        acc[j] = a;
    }
}

hipError_t launch_add_images(double *acc, int64_t n_pix, const AddBatch &b, int n_img, int img_f64,
                             hipStream_t stream)
{
    bool aligned = ((uintptr_t)acc & 15) == 0;
    for (int k = 0; k < n_img; ++k) aligned = aligned && ((uintptr_t)b.img[k] & 15) == 0;
    if (!img_f64 && aligned) {
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(((n_pix >> 2) + BLOCK - 1) / BLOCK, 16384));
        hipLaunchKernelGGL(add_images4_kernel, dim3(grid), dim3(BLOCK), 0, stream, acc, n_pix, b, n_img);
        return hipGetLastError();
    }
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n_pix + BLOCK - 1) / BLOCK, 16384));
    hipLaunchKernelGGL(add_images_kernel, dim3(grid), dim3(BLOCK), 0, stream, acc, n_pix, b, n_img, img_f64);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Padded F^2 tables: entry (a, b, c) of the (na+2P)(nb+2P)(nc+2P) box holds
// F(a-P, b-P, c-P)^2 inside the tabulated range and F_default^2 elsewhere.
// ---------------------------------------------------------------------------
__global__ void pad_table_kernel(const void *src, int src_f64, int na, int nb, int nc, int pad,
                                 double F_default, double *F2_64, float *F2_32)
{
    const int pb = nb + 2 * pad, pc = nc + 2 * pad;
    const int64_t total = (int64_t)(na + 2 * pad) * pb * pc;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % pc) - pad;
        const int b = (int)((i / pc) % pb) - pad;
        const int a = (int)(i / ((int64_t)pb * pc)) - pad;
        double F = F_default;
        if (a >= 0 && a < na && b >= 0 && b < nb && c >= 0 && c < nc) {
            const int64_t s = ((int64_t)a * nb + b) * nc + c;
            F = src_f64 ? ((const double *)src)[s] : (double)((const float *)src)[s];
        }
        F2_64[i] = F * F;
        F2_32[i] = (float)(F * F);
    }
}

hipError_t launch_pad_table(const void *src, int src_f64, int32_t na, int32_t nb, int32_t nc,
                            int32_t pad, double F_default, double *F2_64, float *F2_32,
                            hipStream_t stream)
{
    hipLaunchKernelGGL(pad_table_kernel, dim3(1024), dim3(256), 0, stream, src, src_f64, na, nb,
                       nc, pad, F_default, F2_64, F2_32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagnostics: S and h of single terms by the code of the spots kernel.
// ---------------------------------------------------------------------------
__global__ void trace_kernel(const Params p, int64_t n, const int32_t *idx, double *S_out,
                             double *h_out)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int32_t *e = idx + 6 * q;
    double d[3], R, S[3], h[3];
    sample_dir(p, e[0], e[1], e[2] / p.O, e[2] % p.O, e[3], d, R);
    scatter(p.src + SRC_STRIDE * e[4], d, S);
    miller(p.mats + 9 * e[5], S, h);
    for (int i = 0; i < 3; ++i) {
        S_out[3 * q + i] = S[i];
        h_out[3 * q + i] = h[i];
    }
}

__global__ void sinpi_kernel(const double *x, int64_t n, double *s64, float *s32)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    if (s64) s64[q] = sinpi_reduced(x[q]);
    if (s32) s32[q] = sinpi_reduced((float)x[q]);
}

hipError_t launch_sinpi(const double *x, int64_t n, double *s64, float *s32, hipStream_t stream)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(sinpi_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, x, n, s64, s32);
    return hipGetLastError();
}

__global__ void exp_kernel(const double *x, int64_t n, double *y)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < n) y[q] = exp_f64(x[q]);
}

hipError_t launch_exp(const double *x, int64_t n, double *y, hipStream_t stream)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(exp_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, x, n, y);
    return hipGetLastError();
}

hipError_t launch_trace(const Params &p, int64_t n, const int32_t *idx, double *S, double *h,
                        hipStream_t stream)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(trace_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, idx, S, h);
    return hipGetLastError();
}

}  // namespace xrt
