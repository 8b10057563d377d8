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

// exp(e) in binary64 for the Gaussian lattice factor: e = n ln2 + r with
// n = rint(e / ln2) and r reduced by two fused multiply-adds against ln2 split
// into a binary64 head and tail (Cody and Waite's reduction); exp(r) on
// |r| <= ln2/2 is a degree-11 relative-minimax polynomial (fit_exp.py in this
// directory: 2.3e-17 with the coefficients as stored), evaluated by Horner's
// rule with fused multiply-adds; 2^n is applied by ldexp, which also yields
// the subnormal results and 0 below the binary64 range.  The Horner steps
// with coefficients other than 1 use fma_sc.  For e <= 709 (the
// lattice exponents are at most log(Na^2 Nb^2 Nc^2)); e is raised to -1100
// first, where the result is 0 either way, so n fits an int.
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

__device__ __forceinline__ double exp_f64(double e)
{
    double n;
    const double r = exp_reduce(e, n);
    return __builtin_ldexp(__builtin_fma(exp_q(r), r, 1.0), (int)n);
}

// e^x - 1 in binary64 with the same reduction and polynomial: r q(r) when
// n = 0 (|x| <= ln2/2, where e^x - 1 would cancel), otherwise
// 2^n (1 + r q(r)) - 1, whose subtraction loses at most a bit or two (for
// n = -1 the difference is at least 1 - e^(-ln2/2) = 0.29).  For x <= 709.
__device__ __forceinline__ double expm1_f64(double x)
{
    double n;
    const double r = exp_reduce(x, n);
    const double q = exp_q(r);
    return n == 0.0 ? r * q : __builtin_ldexp(__builtin_fma(q, r, 1.0), (int)n) - 1.0;
}

// sin(pi x) for |x| <= 1/2, composed as the lattice factor uses it.
__device__ __forceinline__ double sinpi_reduced(double x, double c6 = SINPI_C6) { return x * sinpi_over_x(x * x, c6); }
__device__ __forceinline__ float sinpi_reduced(float x) { return x * sinpi_over_x(x * x); }

}  // namespace xrt
