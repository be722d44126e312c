// Throughput of the gfx950 arithmetic instructions the half-step kernels are
// built on: FP64 / FP32 / BF16 matrix-core products and FP64 vector FMAs, each
// as 8 (or 16) independent accumulation chains per wave with no memory
// traffic, 4 waves per SIMD. The mixed case runs matrix-core and vector waves
// side by side to see whether the two FP64 paths share execution resources;
// the last cases take the vector FMA's second factor from memory through
// scalar loads.
// Build: hipcc --offload-arch=gfx950 -O3 -o mfma_rate mfma_rate.hip
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

template <int KIND>
__global__ __launch_bounds__(256) void k(double* out, int iters) {
    const int lane = threadIdx.x & 63;
    if constexpr (KIND == 0) {
        d4 acc[8];
        for (int p = 0; p < 8; ++p) acc[p] = d4{0, 0, 0, 0};
        double a = 1.0 + lane * 1e-3, b = 0.5 - lane * 1e-3;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int p = 0; p < 8; ++p) acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[p], 0, 0, 0);
        }
        double s = 0;
        for (int p = 0; p < 8; ++p) s += acc[p][0] + acc[p][1] + acc[p][2] + acc[p][3];
        out[blockIdx.x * blockDim.x + threadIdx.x] = s;
    } else if constexpr (KIND == 1) {
        f4 acc[8];
        for (int p = 0; p < 8; ++p) acc[p] = f4{0, 0, 0, 0};
        float a = 1.0f + lane * 1e-3f, b = 0.5f - lane * 1e-3f;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int p = 0; p < 8; ++p) acc[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[p], 0, 0, 0);
        }
        float s = 0;
        for (int p = 0; p < 8; ++p) s += acc[p][0] + acc[p][1] + acc[p][2] + acc[p][3];
        out[blockIdx.x * blockDim.x + threadIdx.x] = s;
    } else if constexpr (KIND == 2) {
        f4 acc[8];
        for (int p = 0; p < 8; ++p) acc[p] = f4{0, 0, 0, 0};
        s4 a = s4{(short)(0x3f80 + lane), 0x3f80, 0x3f00, 0x3f80}, b = s4{0x3f80, (short)(0x3f00 + lane), 0x3f80, 0x3f80};
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int p = 0; p < 8; ++p) acc[p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[p], 0, 0, 0);
        }
        float s = 0;
        for (int p = 0; p < 8; ++p) s += acc[p][0] + acc[p][1] + acc[p][2] + acc[p][3];
        out[blockIdx.x * blockDim.x + threadIdx.x] = s;
    } else if constexpr (KIND == 4) {
        // half the waves on FP64 MFMA, half on FP64 VALU FMA (co-execution test)
        const int wave = threadIdx.x >> 6;
        double s = 0;
        if (wave & 1) {
            d4 acc[8];
            for (int p = 0; p < 8; ++p) acc[p] = d4{0, 0, 0, 0};
            double a = 1.0 + lane * 1e-3, b = 0.5 - lane * 1e-3;
            for (int it = 0; it < iters; ++it) {
#pragma unroll
                for (int p = 0; p < 8; ++p) acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[p], 0, 0, 0);
            }
            for (int p = 0; p < 8; ++p) s += acc[p][0] + acc[p][1] + acc[p][2] + acc[p][3];
        } else {
            double acc[16];
            for (int p = 0; p < 16; ++p) acc[p] = lane * 1e-3 + p;
            const double a = 0.999999, b = 1e-7;
            for (int it = 0; it < iters; ++it) {
#pragma unroll
                for (int r = 0; r < 8; ++r)
#pragma unroll
                    for (int p = 0; p < 16; ++p) acc[p] = __builtin_fma(acc[p], a, b);
            }
            for (int p = 0; p < 16; ++p) s += acc[p];
        }
        out[blockIdx.x * blockDim.x + threadIdx.x] = s;
    } else if constexpr (KIND == 5) {
        typedef short s8 __attribute__((ext_vector_type(8)));
        f4 acc[8];
        for (int p = 0; p < 8; ++p) acc[p] = f4{0, 0, 0, 0};
        s8 a = s8{(short)(0x3f80 + lane), 0x3f80, 0x3f00, 0x3f80, 0x3f80, 0x3f80, 0x3f80, 0x3f80};
        s8 b = s8{0x3f80, (short)(0x3f00 + lane), 0x3f80, 0x3f80, 0x3f80, 0x3f80, 0x3f80, 0x3f80};
        typedef __bf16 b8 __attribute__((ext_vector_type(8)));
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int p = 0; p < 8; ++p)
                acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), acc[p], 0, 0, 0);
        }
        float s = 0;
        for (int p = 0; p < 8; ++p) s += acc[p][0] + acc[p][1] + acc[p][2] + acc[p][3];
        out[blockIdx.x * blockDim.x + threadIdx.x] = s;
    } else if constexpr (KIND == 6) {
        // FP64 matrix cores in 4x4 tiles: v_mfma_f64_4x4x4f64, 4 blocks per instruction
        double acc[8];
        for (int p = 0; p < 8; ++p) acc[p] = 0.0;
        double a = 1.0 + lane * 1e-3, b = 0.5 - lane * 1e-3;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int p = 0; p < 8; ++p) acc[p] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, acc[p], 0, 0, 0);
        }
        double s = 0;
        for (int p = 0; p < 8; ++p) s += acc[p];
        out[blockIdx.x * blockDim.x + threadIdx.x] = s;
    } else {
        // FP64 VALU FMA chains for comparison
        double acc[16];
        for (int p = 0; p < 16; ++p) acc[p] = lane * 1e-3 + p;
        const double a = 0.999999, b = 1e-7;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int p = 0; p < 16; ++p) acc[p] = __builtin_fma(acc[p], a, b);
        }
        double s = 0;
        for (int p = 0; p < 16; ++p) s += acc[p];
        out[blockIdx.x * blockDim.x + threadIdx.x] = s;
    }
}

// FP64 vector FMAs whose second factor is a wave-uniform operator entry read
// from memory (scalar loads into scalar registers), as a vector-ALU
// contraction with a shared operator needs: 64 accumulators per lane, per
// column 64 FMAs with the column's 64 entries (operator slice of opc columns,
// cycled) plus 8 multiplies that keep the per-lane inputs live.
__global__ __launch_bounds__(256) void kop(const double* __restrict__ op, int opc, double* __restrict__ out,
                                           int iters) {
    const int lane = threadIdx.x & 63;
    double acc[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) acc[r] = lane * 1e-3 + r;
    double x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = 1.0 - (lane + k) * 1e-4;
    for (int it = 0; it < iters; ++it) {
#pragma unroll 1
        for (int c = 0; c < 128; ++c) {
            const double* __restrict__ o = op + (size_t)(c % opc) * 64;
#pragma unroll
            for (int r = 0; r < 64; ++r) acc[r] = __builtin_fma(o[r], x[r & 7], acc[r]);
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = x[k] * 0.999999;
        }
    }
    double s = 0;
#pragma unroll
    for (int r = 0; r < 64; ++r) s += acc[r];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

void run_scalar_operand(int opc) {
    const int blocks = 512, threads = 256, iters = 40;
    double *op = nullptr, *out = nullptr;
    if (hipMalloc(&op, 128 * 64 * sizeof(double)) != hipSuccess ||
        hipMalloc(&out, (size_t)blocks * threads * sizeof(double)) != hipSuccess)
        std::exit(1);
    if (hipMemset(op, 0, 128 * 64 * sizeof(double)) != hipSuccess) std::exit(1);
    hipLaunchKernelGGL(kop, dim3(blocks), dim3(threads), 0, 0, op, opc, out, 2);
    hipEvent_t e0, e1; hipEventCreate(&e0); hipEventCreate(&e1);
    hipEventRecord(e0);
    hipLaunchKernelGGL(kop, dim3(blocks), dim3(threads), 0, 0, op, opc, out, iters);
    hipEventRecord(e1); hipEventSynchronize(e1);
    if (hipGetLastError() != hipSuccess) std::exit(1);
    float ms; hipEventElapsedTime(&ms, e0, e1);
    const double fma = (double)blocks * threads * iters * 128 * 64;
    printf("v_fma_f64, scalar operand, operator %6d B: %8.3f ms  %8.2f TFLOP/s (FMAs only)\n", opc * 64 * 8, ms,
           2 * fma / ms / 1e9);
    hipFree(op);
    hipFree(out);
}

template <int KIND>
void run(const char* name, double flops_per_inst_wave, int insts_per_iter) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        std::printf("no device\n");
        std::exit(1);
    }
    const int blocks = cus * 4, threads = 256, iters = 2000;
    double* out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * threads * sizeof(double)) != hipSuccess) std::exit(1);
    hipLaunchKernelGGL(k<KIND>, dim3(blocks), dim3(threads), 0, 0, out, 10);
    hipDeviceSynchronize();
    hipEvent_t e0, e1; hipEventCreate(&e0); hipEventCreate(&e1);
    hipEventRecord(e0);
    hipLaunchKernelGGL(k<KIND>, dim3(blocks), dim3(threads), 0, 0, out, iters);
    hipEventRecord(e1); hipEventSynchronize(e1);
    float ms; hipEventElapsedTime(&ms, e0, e1);
    const double waves = (double)blocks * threads / 64;
    const double insts = waves * iters * insts_per_iter;
    const double flops = insts * flops_per_inst_wave;
    // cycles per instruction per SIMD at 2.4 GHz
    const double simds = cus * 4.0;
    printf("%-28s %8.3f ms  %8.2f TFLOP/s  %6.1f cycles/inst/SIMD @2.4GHz\n", name, ms, flops / ms / 1e9,
           ms * 1e-3 * 2.4e9 * simds / insts);
    hipFree(out);
}

int main() {
    run<0>("mfma_f64_16x16x4", 2.0 * 16 * 16 * 4, 8);
    run<1>("mfma_f32_16x16x4", 2.0 * 16 * 16 * 4, 8);
    run<2>("mfma_f32_16x16x16_bf16", 2.0 * 16 * 16 * 16, 8);
    run<3>("v_fma_f64 (VALU)", 2.0 * 64, 128);
    // co-execution: per wave pair, one MFMA wave (8 MFMAs/iter) + one VALU wave (128 FMAs/iter);
    // time to compare with half the MFMA-only time + half the VALU-only time (independent units)
    // or their sum (shared units). Reported TFLOP/s counts both kinds.
    run<4>("mixed f64 mfma+valu waves", 0.5 * (2.0 * 16 * 16 * 4 * 8) + 0.5 * (2.0 * 64 * 128), 1);
    run<5>("mfma_f32_16x16x32_bf16", 2.0 * 16 * 16 * 32, 8);
    run<6>("mfma_f64_4x4x4 (4 blocks)", 2.0 * 4 * 4 * 4 * 4, 8);
    run_scalar_operand(2);     // 1 KB: always in the scalar cache
    run_scalar_operand(128);   // 64 KB streamed per wave
    return 0;
}
