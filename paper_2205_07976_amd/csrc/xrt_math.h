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

__device__ __forceinline__ double sinpi_over_x(double y)  // y = x^2, returns sin(pi x)/x
{
    double p = -2.1122952923797757e-05;
    p = __builtin_fma(p, y, 0.00046597761697049093);
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

// sin(pi x) for |x| <= 1/2, composed as the lattice factor uses it.
__device__ __forceinline__ double sinpi_reduced(double x) { return x * sinpi_over_x(x * x); }
__device__ __forceinline__ float sinpi_reduced(float x) { return x * sinpi_over_x(x * x); }

}  // namespace xrt
