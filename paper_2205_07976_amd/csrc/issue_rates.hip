// issue_rates.hip -- measured issue rates of the VALU instruction classes the
// spots kernel is built from, on the current GPU.
//
// Each kernel runs 8 interleaved dependency chains of one instruction (so a
// chain's next use is 8 instructions away and never waits on latency), on
// 8 waves per SIMD, and reports SIMD cycles per wave64 instruction at the
// shader clock measured alongside (s_memtime counts shader cycles,
// s_memrealtime a fixed 100 MHz reference).  These rates price the
// per-term operation list of the lattice sum (cycles per wave-term).
//
// Build: hipcc --offload-arch=gfx950 -O3 -o issue_rates issue_rates.hip
#include <hip/hip_runtime.h>

#include <cstdio>
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                      \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            fprintf(stderr, "%s:%d %s\n", __FILE__, __LINE__, hipGetErrorString(e_)); \
            exit(1);                                                                  \
        }                                                                             \
    } while (0)

constexpr int UNROLL = 16;  // instructions per chain per loop iteration
constexpr int CHAINS = 8;

#define R8(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

// one instruction class per kernel: a is the chain register, b/c operands
#define KERNEL_F64(name, asmstr)                                                      \
    __global__ void name(double *out, int iters, double b, double c)                  \
    {                                                                                 \
        double a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4,   \
               a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;                                 \
        for (int it = 0; it < iters; ++it) {                                          \
            _Pragma("unroll") for (int u = 0; u < UNROLL; ++u)                        \
            {                                                                         \
                _Pragma("unroll") for (int k = 0; k < 1; ++k)                         \
                {                                                                     \
                    asm volatile(asmstr : "+v"(a0) : "v"(b), "v"(c));                 \
                    asm volatile(asmstr : "+v"(a1) : "v"(b), "v"(c));                 \
                    asm volatile(asmstr : "+v"(a2) : "v"(b), "v"(c));                 \
                    asm volatile(asmstr : "+v"(a3) : "v"(b), "v"(c));                 \
                    asm volatile(asmstr : "+v"(a4) : "v"(b), "v"(c));                 \
                    asm volatile(asmstr : "+v"(a5) : "v"(b), "v"(c));                 \
                    asm volatile(asmstr : "+v"(a6) : "v"(b), "v"(c));                 \
                    asm volatile(asmstr : "+v"(a7) : "v"(b), "v"(c));                 \
                }                                                                     \
            }                                                                         \
        }                                                                             \
        out[blockIdx.x * blockDim.x + threadIdx.x] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7; \
    }

#define KERNEL_T(name, T, asmstr)                                                     \
    __global__ void name(T *out, int iters, T b, T c)                                 \
    {                                                                                 \
        T a0 = (T)threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4,     \
          a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;                                      \
        for (int it = 0; it < iters; ++it) {                                          \
            _Pragma("unroll") for (int u = 0; u < UNROLL; ++u)                        \
            {                                                                         \
                asm volatile(asmstr : "+v"(a0) : "v"(b), "v"(c));                     \
                asm volatile(asmstr : "+v"(a1) : "v"(b), "v"(c));                     \
                asm volatile(asmstr : "+v"(a2) : "v"(b), "v"(c));                     \
                asm volatile(asmstr : "+v"(a3) : "v"(b), "v"(c));                     \
                asm volatile(asmstr : "+v"(a4) : "v"(b), "v"(c));                     \
                asm volatile(asmstr : "+v"(a5) : "v"(b), "v"(c));                     \
                asm volatile(asmstr : "+v"(a6) : "v"(b), "v"(c));                     \
                asm volatile(asmstr : "+v"(a7) : "v"(b), "v"(c));                     \
            }                                                                         \
        }                                                                             \
        out[blockIdx.x * blockDim.x + threadIdx.x] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7; \
    }

// binary64 arithmetic
KERNEL_F64(k_fma_f64, "v_fma_f64 %0, %0, %1, %2")
KERNEL_F64(k_mul_f64, "v_mul_f64 %0, %0, %1")
KERNEL_F64(k_add_f64, "v_add_f64 %0, %0, %1")
KERNEL_F64(k_max_f64, "v_max_f64 %0, |%0|, %1")
KERNEL_F64(k_rndne_f64, "v_rndne_f64 %0, %0")
KERNEL_F64(k_rcp_f64, "v_rcp_f64 %0, %0")
// binary32 arithmetic
KERNEL_T(k_fma_f32, float, "v_fma_f32 %0, %0, %1, %2")
KERNEL_T(k_mul_f32, float, "v_mul_f32 %0, %0, %1")
KERNEL_T(k_add_f32, float, "v_add_f32 %0, %0, %1")
KERNEL_T(k_rcp_f32, float, "v_rcp_f32 %0, %0")
KERNEL_T(k_exp_f32, float, "v_exp_f32 %0, %0")
KERNEL_T(k_sin_f32, float, "v_sin_f32 %0, %0")
KERNEL_T(k_rndne_f32, float, "v_rndne_f32 %0, %0")
// 32-bit integer
KERNEL_T(k_max_i32, int, "v_max_i32 %0, %0, %1")
KERNEL_T(k_med3_i32, int, "v_med3_i32 %0, %0, %1, %2")
KERNEL_T(k_mad_u24, int, "v_mad_u32_u24 %0, %0, %1, %2")
KERNEL_T(k_add3_u32, int, "v_add3_u32 %0, %0, %1, %2")

// conversions: source and destination differ, so chain through a second op
__global__ void k_cvt_f32_f64(float *out, int iters, double b, double c)
{
    float a[CHAINS];
    double d[CHAINS];
    for (int k = 0; k < CHAINS; ++k) d[k] = threadIdx.x + k + b;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int k = 0; k < CHAINS; ++k) asm volatile("v_cvt_f32_f64 %0, %1" : "=v"(a[k]) : "v"(d[k]));
    }
    float s = 0;
    for (int k = 0; k < CHAINS; ++k) s += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s + (float)c;
}

__global__ void k_cvt_i32_f64(int *out, int iters, double b, double c)
{
    int a[CHAINS];
    double d[CHAINS];
    for (int k = 0; k < CHAINS; ++k) d[k] = threadIdx.x + k + b;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int k = 0; k < CHAINS; ++k) asm volatile("v_cvt_i32_f64 %0, %1" : "=v"(a[k]) : "v"(d[k]));
    }
    int s = 0;
    for (int k = 0; k < CHAINS; ++k) s += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s + (int)c;
}

__global__ void k_cvt_f64_f32(double *out, int iters, double b, double c)
{
    double a[CHAINS];
    float d[CHAINS];
    for (int k = 0; k < CHAINS; ++k) d[k] = threadIdx.x + k + (float)b;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int k = 0; k < CHAINS; ++k) asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(a[k]) : "v"(d[k]));
    }
    double s = 0;
    for (int k = 0; k < CHAINS; ++k) s += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s + c;
}

__global__ void k_lshl_add_u64(uint64_t *out, int iters, double b, double c)
{
    uint64_t a[CHAINS];
    uint64_t s = (uint64_t)b;
    for (int k = 0; k < CHAINS; ++k) a[k] = threadIdx.x + k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int k = 0; k < CHAINS; ++k) asm volatile("v_lshl_add_u64 %0, %0, 2, %1" : "+v"(a[k]) : "v"(s));
    }
    uint64_t t = 0;
    for (int k = 0; k < CHAINS; ++k) t += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t + (uint64_t)c;
}

// shader clock: s_memtime (shader cycles) against s_memrealtime (100 MHz)
__global__ void k_clock(uint64_t *out, int iters, double b, double c)
{
    uint64_t t0 = __builtin_amdgcn_s_memtime();
    uint64_t r0 = __builtin_amdgcn_s_memrealtime();
    double a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(a0) : "v"(b), "v"(c));
            asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(a1) : "v"(b), "v"(c));
            asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(a2) : "v"(b), "v"(c));
            asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(a3) : "v"(b), "v"(c));
        }
    }
    uint64_t t1 = __builtin_amdgcn_s_memtime();
    uint64_t r1 = __builtin_amdgcn_s_memrealtime();
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    out[3 * g] = t1 - t0;
    out[3 * g + 1] = r1 - r0;
    out[3 * g + 2] = (uint64_t)(a0 + a1 + a2 + a3);
}

// accuracy of the hardware reciprocals: r = rcp(x) for x in [1, 2)
__global__ void k_rcp_acc(const double *x, double *r64, float *r32, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    r64[i] = __builtin_amdgcn_rcp(x[i]);
    r32[i] = __builtin_amdgcn_rcpf((float)x[i]);
}

struct Entry {
    const char *name;
    void (*launch)(void *, int, hipStream_t);
};

template <typename T, typename K>
void run(K kernel, void *buf, int iters, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), 0, s, (T *)buf, iters, (T)1.0000001, (T)1e-9);
}

int main(int argc, char **argv)
{
    int dev = 0;
    CHECK(hipSetDevice(dev));
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, dev));
    const int cus = prop.multiProcessorCount;
    const int simds = cus * 4;
    const int blocks = cus * 8;  // 8 waves per SIMD (4 waves per block of 256)
    const int iters = argc > 1 ? atoi(argv[1]) : 256;
    const size_t lanes = (size_t)blocks * 256;
    void *buf = nullptr;
    CHECK(hipMalloc(&buf, lanes * 3 * sizeof(uint64_t)));
    hipStream_t s;
    CHECK(hipStreamCreate(&s));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));

    // shader clock
    hipLaunchKernelGGL(k_clock, dim3(blocks), dim3(256), 0, s, (uint64_t *)buf, iters * 8, 1.0000001, 1e-9);
    CHECK(hipStreamSynchronize(s));
    std::vector<uint64_t> h(lanes * 3);
    CHECK(hipMemcpy(h.data(), buf, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
    double cyc = 0, real = 0;
    for (size_t i = 0; i < lanes; i += 64) {
        cyc += (double)h[3 * i];
        real += (double)h[3 * i + 1];
    }
    const double clock_ghz = cyc / real * 0.1;  // s_memrealtime runs at 100 MHz
    printf("device %s, %d CUs, shader clock under FP64 load %.3f GHz\n", prop.name, cus, clock_ghz);
    printf("%-16s %12s %14s %16s\n", "instruction", "ms", "cycles/wave-op", "Glane-op/s");

#define RUN(T, K)                                                                           \
    {                                                                                       \
        run<T>(K, buf, iters, blocks, s);                                                   \
        CHECK(hipEventRecord(e0, s));                                                       \
        run<T>(K, buf, iters, blocks, s);                                                   \
        CHECK(hipEventRecord(e1, s));                                                       \
        CHECK(hipEventSynchronize(e1));                                                     \
        float ms = 0;                                                                       \
        CHECK(hipEventElapsedTime(&ms, e0, e1));                                            \
        const double wave_ops = (double)blocks * 4 * iters * UNROLL * CHAINS;               \
        const double per_simd = wave_ops / simds;                                           \
        const double cyc_per = ms * 1e-3 * clock_ghz * 1e9 / per_simd;                      \
        printf("%-16s %12.3f %14.3f %16.1f\n", &(#K)[2], ms, cyc_per, wave_ops * 64 / (ms * 1e-3) / 1e9); \
    }
    RUN(double, k_fma_f64) RUN(double, k_mul_f64) RUN(double, k_add_f64) RUN(double, k_max_f64)
    RUN(double, k_rndne_f64) RUN(double, k_rcp_f64)
    RUN(float, k_fma_f32) RUN(float, k_mul_f32) RUN(float, k_add_f32) RUN(float, k_rcp_f32)
    RUN(float, k_exp_f32) RUN(float, k_sin_f32) RUN(float, k_rndne_f32)
    RUN(int, k_max_i32) RUN(int, k_med3_i32) RUN(int, k_mad_u24) RUN(int, k_add3_u32)
    RUN(float, k_cvt_f32_f64) RUN(int, k_cvt_i32_f64) RUN(double, k_cvt_f64_f32)
    RUN(uint64_t, k_lshl_add_u64)
    {
        const int n = 1 << 20;
        std::vector<double> hx(n), h64(n);
        std::vector<float> h32(n);
        uint64_t st = 88172645463325252ull;  // xorshift64
        for (int i = 0; i < n; ++i) {
            st ^= st << 13; st ^= st >> 7; st ^= st << 17;
            hx[i] = 1.0 + (double)(st >> 11) * 0x1.0p-53;
        }
        double *dx, *d64;
        float *d32;
        CHECK(hipMalloc(&dx, n * sizeof(double)));
        CHECK(hipMalloc(&d64, n * sizeof(double)));
        CHECK(hipMalloc(&d32, n * sizeof(float)));
        CHECK(hipMemcpy(dx, hx.data(), n * sizeof(double), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_rcp_acc, dim3(n / 256), dim3(256), 0, s, dx, d64, d32, n);
        CHECK(hipStreamSynchronize(s));
        CHECK(hipMemcpy(h64.data(), d64, n * sizeof(double), hipMemcpyDeviceToHost));
        CHECK(hipMemcpy(h32.data(), d32, n * sizeof(float), hipMemcpyDeviceToHost));
        long double e64 = 0, e32 = 0;
        for (int i = 0; i < n; ++i) {
            const long double x = hx[i];
            e64 = std::max(e64, fabsl((long double)h64[i] * x - 1.0L));
            e32 = std::max(e32, fabsl((long double)h32[i] * (long double)(float)hx[i] - 1.0L));
        }
        printf("v_rcp_f64 max rel err %.3Le (2^%.1f), v_rcp_f32 max rel err %.3Le (2^%.1f)\n", e64,
               (double)log2l(e64), e32, (double)log2l(e32));
        CHECK(hipFree(dx));
        CHECK(hipFree(d64));
        CHECK(hipFree(d32));
    }
    CHECK(hipFree(buf));
    return 0;
}
