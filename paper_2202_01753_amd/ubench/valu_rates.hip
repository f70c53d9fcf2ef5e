// Issue rates of the VALU instructions the sampling kernels are made of, on
// the GPU it runs on: the measurement behind the per-sample cost model that
// bench.py prices the sampling kernels with (which instructions take one
// 4-cycle issue slot of a SIMD, which take half of one, which take more).
//
// Each kernel runs 8 independent dependency chains per lane, 16 steps per
// loop iteration, over 2048 workgroups of 256 threads (8 waves per SIMD), so
// issue rather than latency bounds it.  In the integer kernels an empty asm
// statement after each step keeps the compiler from folding steps together
// (x + p + p ... into one multiply-add), and so does the FP64 conversion
// pair, which is idempotent; other floating-point steps are not folded.  The shader clock is read at the
// start and end of the first workgroup (clock64 against the constant-rate
// wall clock), since a long run of dense arithmetic can lower it below the
// nominal 2.4 GHz.  Prints per kernel the time, the measured clock, and the
// cycles per step per SIMD at that clock and at 2.4 GHz; a step is the listed
// instructions (a step of two pairs the instruction of interest with one
// whose cost another line gives).
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

template <typename T>
__device__ __forceinline__ void keep(T &x) {
    asm volatile("" : "+v"(x));
}

// clocks[2 * blockIdx.x ...]: shader-clock and wall-clock ticks between the
// start and the end of the workgroup's first thread
template <bool KEEP, typename T, typename Op>
__device__ __forceinline__ void chains(T (&x)[kChains], int n, Op op, long long *clocks) {
    long long c0 = 0, w0 = 0;
    if (threadIdx.x == 0) {
        w0 = wall_clock64();
        c0 = clock64();
    }
    for (int it = 0; it < n; ++it)
#pragma unroll
        for (int r = 0; r < kSteps; ++r)
#pragma unroll
            for (int i = 0; i < kChains; ++i) {
                x[i] = op(x[i]);
                if constexpr (KEEP) keep(x[i]);
            }
    if (threadIdx.x == 0) {
        const long long c1 = clock64(), w1 = wall_clock64();
        clocks[2 * blockIdx.x] = c1 - c0;
        clocks[2 * blockIdx.x + 1] = w1 - w0;
    }
}

template <typename T>
__device__ __forceinline__ void store(double *out, const T (&x)[kChains]) {
    double s = 0.0;
    for (int i = 0; i < kChains; ++i) s += (double)x[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

struct Args {
    double *out;
    long long *clocks;
    double a, b;
    int n;
};

#define FLOAT_KERNEL(NAME, KEEP, T, INIT, EXPR)                                         \
    __global__ void NAME(Args g) {                                                \
        T x[kChains];                                                             \
        for (int i = 0; i < kChains; ++i) x[i] = (T)(INIT);                       \
        const T a = (T)g.a, b = (T)g.b;                                           \
        chains<KEEP>(x, g.n, [=](T v) { return EXPR; }, g.clocks);                \
        store(g.out, x);                                                          \
    }

// y a + v with a per-lane y, so that the compiler can use the two-operand
// form that accumulates into its destination
#define ACC_KERNEL(NAME, T, EXPR)                                                 \
    __global__ void NAME(Args g) {                                                \
        T x[kChains];                                                             \
        for (int i = 0; i < kChains; ++i) x[i] = (T)(threadIdx.x * 1e-3 + i);     \
        const T a = (T)g.a, y = (T)(threadIdx.x * 1e-4 + 1.0);                    \
        chains<false>(x, g.n, [=](T v) { return EXPR; }, g.clocks);               \
        store(g.out, x);                                                          \
    }

#define UINT_KERNEL(NAME, T, EXPR)                                                \
    __global__ void NAME(Args g) {                                                \
        T x[kChains];                                                             \
        for (int i = 0; i < kChains; ++i) x[i] = (T)(threadIdx.x * 7u + i);       \
        const uint32_t p = (uint32_t)g.a, q = (uint32_t)g.b;                      \
        chains<true>(x, g.n, [=](T v) { return EXPR; }, g.clocks);                \
        store(g.out, x);                                                          \
    }

// 64-bit class
FLOAT_KERNEL(fma_f64, false, double, threadIdx.x * 1e-3 + i, __builtin_fma(v, a, b))
FLOAT_KERNEL(add_f64, false, double, threadIdx.x * 1e-3 + i, v + a)
FLOAT_KERNEL(mul_f64, false, double, threadIdx.x * 1e-3 + i, v * a)
UINT_KERNEL(mad_u64_u32, uint64_t, (uint64_t)(uint32_t)v * p + v)
// 32-bit class
FLOAT_KERNEL(fma_f32, false, float, threadIdx.x * 1e-3f + i, __builtin_fmaf(v, a, b))
FLOAT_KERNEL(add_f32, false, float, threadIdx.x * 1e-3f + i, v + a)
FLOAT_KERNEL(mul_f32, false, float, threadIdx.x * 1e-3f + i, v * a)
UINT_KERNEL(add_u32, uint32_t, v + p)
UINT_KERNEL(lshl_add_u32, uint32_t, (v << 3) + p)
UINT_KERNEL(bitop3_b32, uint32_t, __builtin_amdgcn_bitop3_b32(v, p, q, 0x96))
UINT_KERNEL(mul_lo_u32, uint32_t, v * p)
UINT_KERNEL(mul_hi_u32, uint32_t, __umulhi(v, p))
UINT_KERNEL(alignbit_b32, uint32_t, __builtin_amdgcn_alignbit(v, p, 12))
// accumulating forms (the chain runs through the addend)
ACC_KERNEL(fmac_f32, float, __builtin_fmaf(y, a, v))
ACC_KERNEL(fmac_f64, double, __builtin_fma(y, a, v))
// steps of two
UINT_KERNEL(cvt_f32_u32_pair, uint32_t, (uint32_t)(float)v)
FLOAT_KERNEL(cvt_f64_i32_pair, true, double, threadIdx.x * 1e-3 + i, (double)(int)v)
FLOAT_KERNEL(floor_f32_add, false, float, threadIdx.x * 1e-3f + i, __builtin_floorf(v + a))
FLOAT_KERNEL(floor_f64_add, false, double, threadIdx.x * 1e-3 + i, __builtin_floor(v + a))
FLOAT_KERNEL(min_f32_mul, false, float, threadIdx.x * 1e-3f + i, __builtin_fminf(v * a, b))
FLOAT_KERNEL(min_f64_mul, false, double, threadIdx.x * 1e-3 + i, __builtin_fmin(v * a, b))
FLOAT_KERNEL(exp_f32_mul, false, float, -1e-3f * i, __builtin_amdgcn_exp2f(v) * a)
// reciprocals
FLOAT_KERNEL(rcp_f32, false, float, 1.0f + 1e-3f * i, __builtin_amdgcn_rcpf(v))
FLOAT_KERNEL(rcp_f64, false, double, 1.0 + 1e-3 * i, __builtin_amdgcn_rcp(v))

using Kernel = void (*)(Args);

struct Case {
    const char *name;
    Kernel k;
    double a, b;
    const char *step;
};

int run(const Case &c, double *d, long long *clk, long long *h_clk, int blocks, int threads, int n,
        int cus, double wall_khz) {
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));
    Args g{d, clk, c.a, c.b, 10};
    hipLaunchKernelGGL(c.k, dim3(blocks), dim3(threads), 0, 0, g);
    CHK(hipGetLastError());
    CHK(hipDeviceSynchronize());
    g.n = n;
    CHK(hipEventRecord(e0));
    hipLaunchKernelGGL(c.k, dim3(blocks), dim3(threads), 0, 0, g);
    CHK(hipGetLastError());
    CHK(hipEventRecord(e1));
    CHK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, e0, e1));
    CHK(hipMemcpy(h_clk, clk, sizeof(long long) * 2 * blocks, hipMemcpyDeviceToHost));
    double cyc = 0.0, wall = 0.0;
    for (int i = 0; i < blocks; ++i) {
        cyc += (double)h_clk[2 * i];
        wall += (double)h_clk[2 * i + 1];
    }
    const double ghz = cyc / (wall / (wall_khz * 1e3)) / 1e9;
    const double wave_steps = (double)blocks * threads / 64.0 * n * kSteps * kChains;
    const double steps_per_simd_ns = wave_steps / (4.0 * cus) / (ms * 1e6);
    std::printf("%-17s %8.3f ms  clock %.2f GHz  cycles per step %.2f (at 2.4 GHz %.2f)  step: %s\n",
                c.name, ms, ghz, ghz / steps_per_simd_ns, 2.4 / steps_per_simd_ns, c.step);
    CHK(hipEventDestroy(e0));
    CHK(hipEventDestroy(e1));
    return 0;
}

}  // namespace

int main() {
    const int blocks = 256 * 8, threads = 256, n = 2000;
    int dev = 0, cus = 0, wall_khz = 0;
    CHK(hipGetDevice(&dev));
    CHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CHK(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
    std::printf("%d compute units, wall clock %d kHz\n", cus, wall_khz);
    double *d = nullptr;
    long long *clk = nullptr;
    CHK(hipMalloc(&d, sizeof(double) * blocks * threads));
    CHK(hipMalloc(&clk, sizeof(long long) * 2 * blocks));
    static long long h_clk[2 * blocks];
    const Case cases[] = {
        {"fma_f64", fma_f64, 1.0000001, 1e-7, "v_fma_f64"},
        {"add_f64", add_f64, 1e-7, 0.0, "v_add_f64"},
        {"mul_f64", mul_f64, 1.0000001, 0.0, "v_mul_f64"},
        {"mad_u64_u32", mad_u64_u32, 2654435769.0, 0.0, "v_mad_u64_u32"},
        {"fma_f32", fma_f32, 1.0000001, 1e-7, "v_fma_f32"},
        {"add_f32", add_f32, 1e-7, 0.0, "v_add_f32"},
        {"mul_f32", mul_f32, 1.0000001, 0.0, "v_mul_f32"},
        {"add_u32", add_u32, 12345.0, 0.0, "v_add_u32"},
        {"lshl_add_u32", lshl_add_u32, 12345.0, 0.0, "v_lshl_add_u32"},
        {"bitop3_b32", bitop3_b32, 12345.0, 777.0, "v_bitop3_b32"},
        {"mul_lo_u32", mul_lo_u32, 2654435769.0, 0.0, "v_mul_lo_u32"},
        {"mul_hi_u32", mul_hi_u32, 2654435769.0, 0.0, "v_mul_hi_u32"},
        {"alignbit_b32", alignbit_b32, 12345.0, 0.0, "v_alignbit_b32"},
        {"fmac_f32", fmac_f32, 1e-7, 0.0, "v_fmac_f32"},
        {"fmac_f64", fmac_f64, 1e-7, 0.0, "v_fmac_f64"},
        {"cvt_f32_u32_pair", cvt_f32_u32_pair, 0.0, 0.0, "v_cvt_f32_u32 + v_cvt_u32_f32"},
        {"cvt_f64_i32_pair", cvt_f64_i32_pair, 0.0, 0.0, "v_cvt_i32_f64 + v_cvt_f64_i32"},
        {"floor_f32_add", floor_f32_add, 0.25, 0.0, "v_add_f32 + v_floor_f32"},
        {"floor_f64_add", floor_f64_add, 0.25, 0.0, "v_add_f64 + v_floor_f64"},
        {"min_f32_mul", min_f32_mul, 1.0000001, 1e30, "v_mul_f32 + v_min_f32"},
        {"min_f64_mul", min_f64_mul, 1.0000001, 1e300, "v_mul_f64 + v_min_f64"},
        {"exp_f32_mul", exp_f32_mul, 0.5, 0.0, "v_exp_f32 + v_mul_f32"},
        {"rcp_f32", rcp_f32, 0.0, 0.0, "v_rcp_f32"},
        {"rcp_f64", rcp_f64, 0.0, 0.0, "v_rcp_f64"},
    };
    int rc = 0;
    for (const Case &c : cases) rc |= run(c, d, clk, h_clk, blocks, threads, n, cus, (double)wall_khz);
    CHK(hipFree(d));
    CHK(hipFree(clk));
    return rc;
}
