// xrt_math.h -- device math for the lattice factor.
//
// sin(pi x) = x * P(x^2) on |x| <= 1/2 with P the relative-minimax polynomial
// from the Remez exchange algorithm (fit_sinpi.py in this directory, 50-digit
// mpmath).  Maximum relative error of x * P(x^2) with the coefficients as
// stored (exact Horner): 2.1e-16 (binary64, degree 7 in x^2) and 4.2e-8
// (binary32, degree 4 in x^2).  Evaluated by Horner's rule with fused
// multiply-adds.
#pragma once

#include <hip/hip_runtime.h>

namespace xrt {

// a * b + c, rounded once, as the three-address v_fma_f64 with c held in
// scalar registers.  For a Horner step with a constant coefficient c the
// compiler otherwise emits the two-address v_fmac_f64, whose accumulator is
// c, after copying c from the vector registers that hold it across the loop:
// one 64-bit move per step.  The value is the same either way (one rounding).
__device__ __forceinline__ double fma_sc(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

// a * b + c, rounded once, as the three-address v_fma_f64 with a in scalar
// registers and c in vector registers.  For the first Horner step, whose
// operands a and c are both constants, the compiler otherwise emits the
// two-address v_fmac_f64 with c as its accumulator and copies c into place
// on every pass of a loop (one 64-bit move per evaluation); here c stays in
// a vector register that the loop does not overwrite (the result is an
// early-clobber operand, so it never takes c's register).
__device__ __forceinline__ double fma_svv(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=&v"(d) : "s"(a), "v"(b), "v"(c));
    return d;
}

// The constant term of the first Horner step of the binary64 sin(pi x)/x.
constexpr double SINPI_C6 = 0.00046597761697049093;

// y = x^2, returns sin(pi x)/x.  c6 is SINPI_C6; a loop that evaluates many
// sines passes a copy that the compiler cannot see through, which then stays
// in one vector register for the whole loop instead of being moved into one
// again for every term (the first step's other constant takes the one scalar
// operand an instruction may read).
__device__ __forceinline__ double sinpi_over_x(double y, double c6 = SINPI_C6)
{
    double p = fma_svv(-2.1122952923797757e-05, y, c6);
    p = __builtin_fma(p, y, -0.0073703610716640494);
    p = __builtin_fma(p, y, 0.08214587825654909);
    p = __builtin_fma(p, y, -0.5992645287757093);
    p = __builtin_fma(p, y, 2.5501640398597765);
    p = __builtin_fma(p, y, -5.167712780049753);
    p = __builtin_fma(p, y, 3.1415926535897927);
    return p;
}

__device__ __forceinline__ float sinpi_over_x(float y)
{
    float p = 0.07756038755178452f;
    p = __builtin_fmaf(p, y, -0.5982421040534973f);
    p = __builtin_fmaf(p, y, 2.550069808959961f);
    p = __builtin_fmaf(p, y, -5.167709827423096f);
    p = __builtin_fmaf(p, y, 3.1415927410125732f);
    return p;
}

// e^x and e^x - 1 in binary64 for the layer capture, without a table (they
// run once per sample point and layer, where the table's registers would
// cost the term loops occupancy): x = n ln2 + r with n = rint(x / ln2) and r
// reduced by two fused multiply-adds against ln2 split into a binary64 head
// and tail (Cody and Waite's reduction); exp(r) on |r| <= ln2/2 is a
// degree-11 relative-minimax polynomial 1 + r q(r) (fit_exp.py in this
// directory: 2.3e-17 with the coefficients as stored), evaluated by Horner's
// rule with fused multiply-adds; 2^n is applied by ldexp, which also yields
// the subnormal results and 0 below the binary64 range.  The Horner steps
// with coefficients other than 1 use fma_sc.  x is raised to -1100 first,
// where the results are 0 and -1 either way, so n fits an int.  For x <= 709.
__device__ __forceinline__ double exp_q(double r)  // e^r = 1 + r q(r) on |r| <= ln2/2
{
    double p = 2.4994304884817207e-08;
    p = fma_sc(p, r, 2.7632293279459877e-07);
    p = fma_sc(p, r, 2.7557622530872255e-06);
    p = fma_sc(p, r, 2.4801486521427463e-05);
    p = fma_sc(p, r, 0.00019841269432679237);
    p = fma_sc(p, r, 0.0013888888951223987);
    p = fma_sc(p, r, 0.00833333333355927);
    p = fma_sc(p, r, 0.04166666666649277);
    p = fma_sc(p, r, 0.1666666666666617);
    p = fma_sc(p, r, 0.5000000000000018);
    return __builtin_fma(p, r, 1.0);
}

// Cody-Waite reduction: e = n ln2 + r, |r| <= ln2/2 (e raised to -1100 first).
__device__ __forceinline__ double exp_reduce(double &e, double &n)
{
    e = __builtin_fmax(e, -1100.0);
    n = __builtin_rint(e * 1.4426950408889634);
    const double r = __builtin_fma(-n, 0.6931471805599453, e);
    return __builtin_fma(-n, 2.3190468138462996e-17, r);
}

__device__ __forceinline__ double exp_cw_f64(double x)
{
    double n;
    const double r = exp_reduce(x, n);
    return __builtin_ldexp(__builtin_fma(exp_q(r), r, 1.0), (int)n);
}

// e^x - 1: r q(r) when n = 0 (|x| <= ln2/2, where e^x - 1 would cancel),
// otherwise 2^n (1 + r q(r)) - 1, whose subtraction loses at most a bit or
// two (for n = -1 the difference is at least 1 - e^(-ln2/2) = 0.29).
__device__ __forceinline__ double expm1_f64(double x)
{
    double n;
    const double r = exp_reduce(x, n);
    const double q = exp_q(r);
    return n == 0.0 ? r * q : __builtin_ldexp(__builtin_fma(q, r, 1.0), (int)n) - 1.0;
}

// 2^(j/64), j = 0..63, each rounded to nearest binary64 (fit_exp.py prints them).
__device__ const double EXP2_J64[64] = {
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0,
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0,
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0,
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0,
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0,
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0,
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0,
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0,
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0,
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0,
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0,
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0,
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0,
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0,
};

// The leading coefficient of exp_f64's polynomial.  A loop that evaluates
// many exponentials passes a copy that the compiler cannot see through (the
// first Horner step's other constant takes the one scalar operand), as with
// SINPI_C6.
constexpr double EXP_C5 = 0.008333324607332198;

// exp(e) in binary64 for the Gaussian lattice factor, by Tang's table-driven
// method: e = n ln2/64 + r with n the integer nearest e 64/ln2, so that
// exp(e) = 2^k 2^(j/64) exp(r) for n = 64 k + j, 0 <= j < 64, |r| <= ln2/128.
// n comes from one fused multiply-add: e 64/ln2 + 1.5 2^52 rounds the exact
// product to an integer, which the low word of the result holds in two's
// complement, and subtracting 1.5 2^52 again gives n exactly.  r is reduced
// by two fused multiply-adds against ln2/64 split into a binary64 head and
// tail (Cody and Waite); exp(r) = 1 + r q(r) with q of degree 4 (a degree-5
// relative-minimax polynomial, fit_exp.py: 2.2e-18 with the coefficients as
// stored), and the result 2^(j/64) + 2^(j/64) r q(r) is formed by one fused
// multiply-add and scaled by ldexp, which also yields the subnormal results
// and 0 below the binary64 range.  Error: half an ulp from the table entry,
// half from the last rounding, a few hundredths from the rest.  For e <= 709
// (the lattice exponents are at most log(Na^2 Nb^2 Nc^2)); e is raised to
// -1100 first, where the result is 0 either way, so |n| stays below 2^17.

__device__ __forceinline__ double exp_f64(double e, double c5 = EXP_C5)
{
    constexpr double SHIFT = 0x1.8p52;
    e = __builtin_fmax(e, -1100.0);
    const double t = __builtin_fma(e, 92.33248261689366, SHIFT);
    const double n = t - SHIFT;
    const int ni = (int)(uint32_t)__builtin_bit_cast(uint64_t, t);
    double r = __builtin_fma(-n, 0.010830424696249145, e);
    r = __builtin_fma(-n, 3.623510646634843e-19, r);
    const double T = EXP2_J64[ni & 63];
    double q = fma_sc(c5, r, 0.04166672775933016);
    q = fma_sc(q, r, 0.16666666666721047);
    q = fma_sc(q, r, 0.4999999999993282);
    q = __builtin_fma(q, r, 1.0);
    return __builtin_ldexp(__builtin_fma(T, r * q, T), ni >> 6);
}

// sin(pi x) for |x| <= 1/2, composed as the lattice factor uses it.
__device__ __forceinline__ double sinpi_reduced(double x, double c6 = SINPI_C6) { return x * sinpi_over_x(x * x, c6); }
__device__ __forceinline__ float sinpi_reduced(float x) { return x * sinpi_over_x(x * x); }

}  // namespace xrt
