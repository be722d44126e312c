// Throughput of the gfx950 arithmetic instructions the half-step kernels are
// built on: FP64 / FP32 / BF16 matrix-core products and FP64 vector FMAs, each
// as 8 (or 16) independent accumulation chains per wave with no memory
// traffic, 4 waves per SIMD. The mixed case runs matrix-core and vector waves
// side by side to see whether the two FP64 paths share execution resources.
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
    return 0;
}
