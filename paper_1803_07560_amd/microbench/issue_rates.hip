// VALU issue rates on gfx950: the per-class costs behind the issue roofline of
// the Monte Carlo kernels.
//
// Every probe kernel runs eight independent chains of one register-to-register
// VALU instruction per lane (no memory operation inside the timed loop), on
// 8 blocks of 256 threads per CU, and reports the achieved rate relative to one
// 64-lane instruction per CU per cycle at 2.4 GHz (the FP64 FMA rate of the
// chip: 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 lane-operations/s).  A rate of 2
// means the class retires two wave-instructions per CU-cycle.
//
// Usage: issue_rates [repeats]   (prints one line per instruction class)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kChains = 8;
constexpr int kIters = 8192;

#define CHECK(x)                                                                    \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
            std::exit(1);                                                           \
        }                                                                           \
    } while (0)

// In-place 32-bit integer/logic instruction on chain value v with operand s.
#define U32_PROBE(NAME, ASM)                                                        \
    __global__ void NAME(uint32_t *out, uint32_t s)                                 \
    {                                                                               \
        uint32_t v[kChains];                                                        \
        for (int i = 0; i < kChains; ++i)                                           \
            v[i] = threadIdx.x + i * s;                                             \
        const uint32_t t = threadIdx.x * 7u;                                        \
        for (int it = 0; it < kIters; ++it) {                                       \
            _Pragma("unroll") for (int c = 0; c < kChains; ++c)                     \
                asm volatile(ASM : "+v"(v[c]) : "v"(s), "v"(t));                   \
        }                                                                           \
        uint32_t r = 0;                                                             \
        for (int i = 0; i < kChains; ++i)                                           \
            r ^= v[i];                                                              \
        out[blockIdx.x * blockDim.x + threadIdx.x] = r;                             \
    }

// In-place floating-point instruction of type T with operands a, b.
#define FP_PROBE(NAME, T, ASM)                                                      \
    __global__ void NAME(uint32_t *out, uint32_t s)                                 \
    {                                                                               \
        T v[kChains];                                                               \
        for (int i = 0; i < kChains; ++i)                                           \
            v[i] = static_cast<T>(0.25) + static_cast<T>(threadIdx.x + i) * static_cast<T>(1e-3); \
        const T a = static_cast<T>(0.999999), b = static_cast<T>(1e-9) * static_cast<T>(s); \
        for (int it = 0; it < kIters; ++it) {                                       \
            _Pragma("unroll") for (int c = 0; c < kChains; ++c)                     \
                asm volatile(ASM : "+v"(v[c]) : "v"(a), "v"(b));                   \
        }                                                                           \
        T r = 0;                                                                    \
        for (int i = 0; i < kChains; ++i)                                           \
            r += v[i];                                                              \
        out[blockIdx.x * blockDim.x + threadIdx.x] = static_cast<uint32_t>(r * static_cast<T>(1e3)); \
    }

U32_PROBE(k_mul_lo, "v_mul_lo_u32 %0, %0, %1")
U32_PROBE(k_mul_hi, "v_mul_hi_u32 %0, %0, %1")
U32_PROBE(k_xor, "v_xor_b32 %0, %0, %1")
U32_PROBE(k_bitop3, "v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96")
U32_PROBE(k_add_u32, "v_add_u32 %0, %0, %1")
FP_PROBE(k_fma64, double, "v_fma_f64 %0, %0, %1, %2")
FP_PROBE(k_add64, double, "v_add_f64 %0, %0, %2")
// operand forms of the FP64 fma: accumulator as the addend, the two-address
// v_fmac_f64, a square, an inline-constant addend, the chain as the second
// multiplicand; and the multiply
FP_PROBE(k_fma64_acc, double, "v_fma_f64 %0, %1, %2, %0")
FP_PROBE(k_fmac64, double, "v_fmac_f64 %0, %1, %2")
FP_PROBE(k_fma64_sq, double, "v_fma_f64 %0, %0, %0, %1")
FP_PROBE(k_fma64_k, double, "v_fma_f64 %0, %0, %1, 1.0")
FP_PROBE(k_mul64, double, "v_mul_f64 %0, %0, %1")
FP_PROBE(k_fma64_src1, double, "v_fma_f64 %0, %1, %0, %2")

// A Horner step p = p r + c_j with the coefficient c_j changing every step
// (twelve coefficients in registers), the chain value as the first or the
// second multiplicand.
#define HORNER_PROBE(NAME, ASM)                                                     \
    __global__ void NAME(uint32_t *out, uint32_t s)                                 \
    {                                                                               \
        double v[kChains];                                                          \
        for (int i = 0; i < kChains; ++i)                                           \
            v[i] = 0.25 + static_cast<double>(threadIdx.x + i) * 1e-3;              \
        const double r = 0.3 + 1e-9 * s;                                            \
        double c[12];                                                               \
        for (int j = 0; j < 12; ++j) {                                              \
            c[j] = 1.0 / (j + 2 + s);                                               \
            asm volatile("" : "+v"(c[j]));                                          \
        }                                                                           \
        for (int it = 0; it < kIters / 12; ++it) {                                  \
            _Pragma("unroll") for (int j = 0; j < 12; ++j)                          \
                _Pragma("unroll") for (int ch = 0; ch < kChains; ++ch)              \
                    asm volatile(ASM : "+v"(v[ch]) : "v"(r), "v"(c[j]));           \
        }                                                                           \
        double t = 0;                                                               \
        for (int i = 0; i < kChains; ++i)                                           \
            t += v[i];                                                              \
        out[blockIdx.x * blockDim.x + threadIdx.x] = static_cast<uint32_t>(t * 1e3); \
    }
HORNER_PROBE(k_horner_src0, "v_fma_f64 %0, %0, %1, %2")
HORNER_PROBE(k_horner_src1, "v_fma_f64 %0, %1, %0, %2")
FP_PROBE(k_fma32, float, "v_fma_f32 %0, %0, %1, %2")
FP_PROBE(k_add32, float, "v_add_f32 %0, %0, %2")
FP_PROBE(k_exp32, float, "v_exp_f32 %0, %0")
FP_PROBE(k_log32, float, "v_log_f32 %0, %0")
FP_PROBE(k_sqrt32, float, "v_sqrt_f32 %0, %0")
FP_PROBE(k_sin32, float, "v_sin_f32 %0, %0")

// 32x32 -> 64-bit multiply-add (the Philox round), carry-out to vcc.
__global__ void k_mad64(uint32_t *out, uint32_t s)
{
    uint64_t v[kChains];
    for (int i = 0; i < kChains; ++i)
        v[i] = threadIdx.x + i * s;
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c)
            asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0"
                         : "+v"(v[c])
                         : "v"(static_cast<uint32_t>(v[c])), "v"(s)
                         : "vcc");
    }
    uint64_t r = 0;
    for (int i = 0; i < kChains; ++i)
        r ^= v[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = static_cast<uint32_t>(r);
}

// Conversions: the destination is rewritten from a source that the chain
// also updates, so every iteration issues one conversion per chain.
#define CVT_PROBE(NAME, TD, TS, ASM)                                                \
    __global__ void NAME(uint32_t *out, uint32_t s)                                 \
    {                                                                               \
        TD d[kChains];                                                              \
        TS x[kChains];                                                              \
        for (int i = 0; i < kChains; ++i) {                                         \
            x[i] = static_cast<TS>(threadIdx.x + i + s);                            \
            d[i] = 0;                                                               \
        }                                                                           \
        for (int it = 0; it < kIters; ++it) {                                       \
            _Pragma("unroll") for (int c = 0; c < kChains; ++c)                     \
                asm volatile(ASM : "=v"(d[c]) : "v"(x[c]));                        \
        }                                                                           \
        double r = 0;                                                               \
        for (int i = 0; i < kChains; ++i)                                           \
            r += static_cast<double>(d[i]);                                         \
        out[blockIdx.x * blockDim.x + threadIdx.x] = static_cast<uint32_t>(r);      \
    }

CVT_PROBE(k_cvt_f64_u32, double, uint32_t, "v_cvt_f64_u32 %0, %1")
CVT_PROBE(k_cvt_f32_u32, float, uint32_t, "v_cvt_f32_u32 %0, %1")
CVT_PROBE(k_cvt_f64_f32, double, float, "v_cvt_f64_f32 %0, %1")

// The library's double-precision exp, counted per call.
__global__ void k_exp64_lib(uint32_t *out, uint32_t s)
{
    double v[kChains];
    for (int i = 0; i < kChains; ++i)
        v[i] = -(threadIdx.x + i + s) * 1e-3;
    for (int it = 0; it < kIters / 8; ++it)
        for (int c = 0; c < kChains; ++c)
            v[c] = exp(-v[c] * 0.5 - 1.0);
    double r = 0;
    for (int i = 0; i < kChains; ++i)
        r += v[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = static_cast<uint32_t>(r * 1e6);
}

using Probe = void (*)(uint32_t *, uint32_t);

struct Entry {
    const char *name;
    Probe fn;
    double ops_per_iter;  // instructions per chain per loop iteration
};

}  // namespace

int main(int argc, char **argv)
{
    const int repeats = argc > 1 ? std::atoi(argv[1]) : 5;
    if (repeats < 1 || repeats > 1000) {
        std::fprintf(stderr, "repeats must be in [1, 1000]\n");
        return 2;
    }
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const int block = 256, blocks = cus * 8;
    std::printf("device %s, %d CUs\n", prop.gcnArchName, cus);
    uint32_t *out = nullptr;
    CHECK(hipMalloc(&out, sizeof(uint32_t) * block * blocks));
    const Entry probes[] = {
        {"v_fma_f64", k_fma64, 1},         {"v_add_f64", k_add64, 1},
        {"v_fma_f64 (acc addend)", k_fma64_acc, 1}, {"v_fmac_f64", k_fmac64, 1},
        {"v_fma_f64 (square)", k_fma64_sq, 1},
        {"v_fma_f64 (const addend)", k_fma64_k, 1}, {"v_mul_f64", k_mul64, 1},
        {"v_fma_f64 (chain in src1)", k_fma64_src1, 1},
        {"Horner, chain in src0", k_horner_src0, 12.0 * (kIters / 12) / kIters},
        {"Horner, chain in src1", k_horner_src1, 12.0 * (kIters / 12) / kIters},
        {"v_fma_f32", k_fma32, 1},         {"v_add_f32", k_add32, 1},
        {"v_mad_u64_u32", k_mad64, 1},     {"v_mul_lo_u32", k_mul_lo, 1},
        {"v_mul_hi_u32", k_mul_hi, 1},     {"v_xor_b32", k_xor, 1},
        {"v_bitop3_b32", k_bitop3, 1},     {"v_add_u32", k_add_u32, 1},
        {"v_cvt_f64_u32", k_cvt_f64_u32, 1}, {"v_cvt_f32_u32", k_cvt_f32_u32, 1},
        {"v_cvt_f64_f32", k_cvt_f64_f32, 1}, {"v_exp_f32", k_exp32, 1},
        {"v_log_f32", k_log32, 1},         {"v_sqrt_f32", k_sqrt32, 1},
        {"v_sin_f32", k_sin32, 1},         {"exp(double) calls", k_exp64_lib, 1.0 / 8},
    };
    hipEvent_t start, stop;
    CHECK(hipEventCreate(&start));
    CHECK(hipEventCreate(&stop));
    const double peak = static_cast<double>(cus) * 64 * 2.4e9;
    // one untimed pass over every probe first, so that the clocks have settled
    // before the first measurement
    for (const Entry &p : probes)
        for (int r = 0; r < repeats; ++r)
            hipLaunchKernelGGL(p.fn, dim3(blocks), dim3(block), 0, 0, out, 3u);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    std::printf("%-26s %12s %10s\n", "instruction", "Tops/s", "per CU-cycle");
    for (const Entry &p : probes) {
        hipLaunchKernelGGL(p.fn, dim3(blocks), dim3(block), 0, 0, out, 3u);
        CHECK(hipGetLastError());
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(start));
        for (int r = 0; r < repeats; ++r)
            hipLaunchKernelGGL(p.fn, dim3(blocks), dim3(block), 0, 0, out, 3u);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(stop));
        CHECK(hipEventSynchronize(stop));
        float ms = 0;
        CHECK(hipEventElapsedTime(&ms, start, stop));
        const double ops = static_cast<double>(repeats) * blocks * block * kIters * kChains *
                           p.ops_per_iter;
        const double rate = ops / (ms * 1e-3);
        std::printf("%-26s %12.3f %10.3f\n", p.name, rate / 1e12, rate / peak);
    }
    CHECK(hipFree(out));
    return 0;
}
