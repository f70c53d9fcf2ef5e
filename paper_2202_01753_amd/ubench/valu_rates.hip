// Issue rates of the VALU instructions the sampling kernels are made of, on
// the GPU it runs on: the measurement behind the per-sample operation model
// that bench.py prices the sampling kernels with (which instructions count
// as one full-rate issue slot and which as more).
//
// Each kernel runs 8 independent dependency chains per lane, 16 steps per
// loop iteration, over 2048 workgroups of 256 threads (8 waves per SIMD), so
// issue rather than latency bounds it.  Prints, per instruction, the wave
// instructions issued per SIMD per nanosecond and the cycles per wave
// instruction at 2.4 GHz (4.0 = one wave64 instruction per 4 clocks on a
// 16-lane SIMD, the full rate).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#define CHK(x)                                                                           \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);   \
            return 1;                                                                    \
        }                                                                                \
    } while (0)

namespace {

constexpr int kSteps = 16, kChains = 8;

template <typename T, typename Op>
__device__ __forceinline__ void chains(T (&x)[kChains], int n, Op op) {
    for (int it = 0; it < n; ++it)
#pragma unroll
        for (int r = 0; r < kSteps; ++r)
#pragma unroll
            for (int i = 0; i < kChains; ++i) x[i] = op(x[i]);
}

template <typename T>
__device__ __forceinline__ void store(double *out, const T (&x)[kChains]) {
    double s = 0.0;
    for (int i = 0; i < kChains; ++i) s += (double)x[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void fma_f64(double *out, double a, double b, int n) {
    double x[kChains];
    for (int i = 0; i < kChains; ++i) x[i] = threadIdx.x * 1e-3 + i;
    chains(x, n, [=](double v) { return __builtin_fma(v, a, b); });
    store(out, x);
}

__global__ void add_f64(double *out, double a, double, int n) {
    double x[kChains];
    for (int i = 0; i < kChains; ++i) x[i] = threadIdx.x * 1e-3 + i;
    chains(x, n, [=](double v) { return v + a; });
    store(out, x);
}

__global__ void fma_f32(double *out, double a, double b, int n) {
    float x[kChains];
    for (int i = 0; i < kChains; ++i) x[i] = threadIdx.x * 1e-3f + i;
    const float fa = (float)a, fb = (float)b;
    chains(x, n, [=](float v) { return __builtin_fmaf(v, fa, fb); });
    store(out, x);
}

__global__ void mad_u64_u32(double *out, double a, double, int n) {
    uint64_t x[kChains];
    for (int i = 0; i < kChains; ++i) x[i] = threadIdx.x * 7u + i;
    const uint32_t m = (uint32_t)a;
    // one v_mad_u64_u32: (low word) * m + the whole 64-bit value
    chains(x, n, [=](uint64_t v) { return (uint64_t)(uint32_t)v * m + v; });
    store(out, x);
}

__global__ void bitop3_b32(double *out, double a, double b, int n) {
    uint32_t x[kChains];
    for (int i = 0; i < kChains; ++i) x[i] = threadIdx.x * 7u + i;
    const uint32_t p = (uint32_t)a, q = (uint32_t)b;
    chains(x, n, [=](uint32_t v) { return __builtin_amdgcn_bitop3_b32(v, p, q, 0x96); });
    store(out, x);
}

__global__ void exp_f32(double *out, double a, double, int n) {
    float x[kChains];
    for (int i = 0; i < kChains; ++i) x[i] = -1e-3f * i;
    const float fa = (float)a;
    // v_exp_f32 (2^x) and a full-rate v_mul_f32 per step, on values that stay
    // in range (the pair's cycles less 4 are the exponential's)
    chains(x, n, [=](float v) { return __builtin_amdgcn_exp2f(v) * fa; });
    store(out, x);
}

__global__ void rcp_f64(double *out, double, double, int n) {
    double x[kChains];
    for (int i = 0; i < kChains; ++i) x[i] = 1.0 + 1e-3 * i;
    chains(x, n, [=](double v) { return __builtin_amdgcn_rcp(v); });
    store(out, x);
}

using Kernel = void (*)(double *, double, double, int);

int run(const char *name, Kernel k, double a, double b, int insts_per_step, double *d, int blocks,
        int threads, int n) {
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));
    hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), 0, 0, d, a, b, 10);
    CHK(hipGetLastError());
    CHK(hipDeviceSynchronize());
    CHK(hipEventRecord(e0));
    hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), 0, 0, d, a, b, n);
    CHK(hipGetLastError());
    CHK(hipEventRecord(e1));
    CHK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, e0, e1));
    int dev = 0, cus = 0;
    CHK(hipGetDevice(&dev));
    CHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const double wave_insts = (double)blocks * threads / 64.0 * n * kSteps * kChains * insts_per_step;
    const double per_simd_ns = wave_insts / (4.0 * cus) / (ms * 1e6);
    std::printf("%-12s %8.3f ms   wave instructions per SIMD per ns %.4f   cycles each at 2.4 GHz %.2f\n",
                name, ms, per_simd_ns, 2.4 / per_simd_ns);
    CHK(hipEventDestroy(e0));
    CHK(hipEventDestroy(e1));
    return 0;
}

}  // namespace

int main() {
    const int blocks = 256 * 8, threads = 256, n = 2000;
    double *d = nullptr;
    CHK(hipMalloc(&d, sizeof(double) * blocks * threads));
    int rc = 0;
    rc |= run("fma_f64", fma_f64, 1.0000001, 1e-7, 1, d, blocks, threads, n);
    rc |= run("add_f64", add_f64, 1e-7, 0.0, 1, d, blocks, threads, n);
    rc |= run("fma_f32", fma_f32, 1.0000001, 1e-7, 1, d, blocks, threads, n);
    rc |= run("mad_u64_u32", mad_u64_u32, 2654435769.0, 0.0, 1, d, blocks, threads, n);
    rc |= run("bitop3_b32", bitop3_b32, 12345.0, 777.0, 1, d, blocks, threads, n);
    rc |= run("exp_f32", exp_f32, 0.5, 0.0, 2, d, blocks, threads, n);
    rc |= run("rcp_f64", rcp_f64, 0.0, 0.0, 1, d, blocks, threads, n);
    CHK(hipFree(d));
    return rc;
}
