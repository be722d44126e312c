// Fused Hermite half step of the advection equation u_t = c (u_x1 + u_x2 +
// u_x3) (Sec. 2, Eq. 1; c = 1 is the paper's equation), FP64.
//
// In the cell variable xi = (x - x_c)/h and the half-step time, the Taylor
// series of Sec. 3.2 (Eq. 5, Alg. 4) with q >= 3(2m+1) stages is exact and
// equals a translation: the evolved polynomial is p(xi + lam (1, 1, 1)),
// lam = c tau / h. So interpolation (Eq. 3, Alg. 1-2), evolution and
// truncation compose into one 1D operator per axis,
//   K1 = T E H   (M x 2M; H: 1D Hermite matrix, E[j][k] = C(k, j) lam^(k-j),
//                 T: keep j <= m),
// and the half step of a cell is the separable contraction
//   y[j3][j2][j1] = sum_a K1[j3][a3] K1[j2][a2] K1[j1][a1] x[a3][a2][a1]
// over the 8 vertices' data x (a = side M + derivative order). It runs sum-
// factorised, 14 M^4 FMAs per cell (m = 3: 3,584 for 64 new values), with
// one lane per cell: the lane streams over (a3, a2), loads the 2M values of
// one x1-line of corners (64 consecutive cells per load instruction),
// contracts it along x1, accumulates the x2 contraction, and after each a3
// the x3 contraction into its M^3 outputs. K1 (2 M^2 entries) is
// wave-uniform and enters the FMAs as scalar operands. At about 7 flop/B the
// kernel is bound by memory traffic, not arithmetic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fused_common.h"
#include "kernels.h"

namespace hermite {
namespace {

using fused::Cell16;
using fused::cell_nodes;
using fused::cell_writing;

constexpr int kThreads = 256;
// At m = 3 the 64 accumulators and the 8-value x1-line fit in about 200
// registers; left alone the compiler takes all 256 (one wave per SIMD, no
// latency hiding), so the bound asks for two.
template <int M>
constexpr int kMinWaves = M == 4 ? 2 : 1;

template <int M>
struct AxisOp {
    double k[M * 2 * M];  // K1[j][a], row-major
};

// The x1-lines of corner data, (a3, a2) = line L / P, L % P in the order
// high derivative orders (small terms) first. Line L's 2M values come from
// the 2 corners along x1 of its (s2, s3) and the M derivative orders d1.
template <int M, int L>
__device__ __forceinline__ void load_line(const double* __restrict__ src, size_t pitch, const Cell16& c, double* x) {
    constexpr int P = 2 * M, a3i = L / P, a2i = L % P;
    constexpr int s3 = a3i & 1, d3 = M - 1 - (a3i >> 1), s2 = a2i & 1, d2 = M - 1 - (a2i >> 1);
#pragma unroll
    for (int a1 = 0; a1 < P; ++a1) {
        const int s1 = a1 / M, d1 = a1 % M;
        x[a1] = src[(size_t)((d3 * M + d2) * M + d1) * pitch + c.corner[s1 + 2 * s2 + 4 * s3]];
    }
}

// Lines requested ahead of the one being contracted (a ring of registers;
// two at m = 3, where the accumulators leave room for no more without
// spilling); the scheduling barrier after each line keeps the compiler from
// pulling the loads back next to their use.
template <int M>
constexpr int kLineAhead = M == 4 ? 2 : 3;
template <int M>
constexpr int kLineRing = kLineAhead<M> + 1;

template <int M, int L>
struct LinePrologue {
    __device__ __forceinline__ static void run(const double* __restrict__ src, size_t pitch, const Cell16& c,
                                               double (*ring)[2 * M]) {
        load_line<M, L>(src, pitch, c, ring[L]);
        if constexpr (L + 1 < kLineAhead<M>) LinePrologue<M, L + 1>::run(src, pitch, c, ring);
    }
};

template <int M, int L>
struct Lines {
    __device__ __forceinline__ static void run(const double* __restrict__ src, size_t pitch, const Cell16& c,
                                               const AxisOp<M>& K, double* y, double* Y, double (*ring)[2 * M]) {
        constexpr int P = 2 * M, a3i = L / P, a2i = L % P;
        constexpr int a3 = (a3i & 1) * M + M - 1 - (a3i >> 1), a2 = (a2i & 1) * M + M - 1 - (a2i >> 1);
        constexpr int A = kLineAhead<M>, R = kLineRing<M>;
        if constexpr (L + A < P * P) load_line<M, L + A>(src, pitch, c, ring[(L + A) % R]);
        const double* x = ring[L % R];
        if constexpr (a2i == 0) {
#pragma unroll
            for (int t = 0; t < M * M; ++t) Y[t] = 0.0;
        }
#pragma unroll
        for (int j1 = 0; j1 < M; ++j1) {
            double z = 0.0;
#pragma unroll
            for (int d1 = M - 1; d1 >= 0; --d1) {
                z = __builtin_fma(K.k[j1 * P + d1], x[d1], z);
                z = __builtin_fma(K.k[j1 * P + M + d1], x[M + d1], z);
            }
#pragma unroll
            for (int j2 = 0; j2 < M; ++j2) Y[j2 * M + j1] = __builtin_fma(K.k[j2 * P + a2], z, Y[j2 * M + j1]);
        }
        if constexpr (a2i == P - 1) {
#pragma unroll
            for (int j3 = 0; j3 < M; ++j3)
#pragma unroll
                for (int t = 0; t < M * M; ++t)
                    y[j3 * M * M + t] = __builtin_fma(K.k[j3 * P + a3], Y[t], y[j3 * M * M + t]);
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (L + 1 < P * P) Lines<M, L + 1>::run(src, pitch, c, K, y, Y, ring);
    }
};

template <int M>
__global__ __launch_bounds__(kThreads, kMinWaves<M>) void advect_kernel(const double* __restrict__ src,
                                                                        double* __restrict__ dst, AxisOp<M> K,
                                                                        uint32_t n, size_t pitch, uint32_t off) {
    constexpr int P = 2 * M, M3 = M * M * M;
    const uint32_t node = blockIdx.x * kThreads + threadIdx.x;  // new node this lane writes
    if (node >= n * n * n) return;
    const Cell16 c = cell_writing(node, n, off);
    double y[M3], Y[M * M];
#pragma unroll
    for (int t = 0; t < M3; ++t) y[t] = 0.0;
    double ring[kLineRing<M>][P];
    LinePrologue<M, 0>::run(src, pitch, c, ring);
    Lines<M, 0>::run(src, pitch, c, K, y, Y, ring);
#pragma unroll
    for (int t = 0; t < M3; ++t) dst[(size_t)t * pitch + c.out] = y[t];
}

template <int M>
hipError_t launch_m(const double* src, double* dst, const double* K1, int n, size_t pitch, int off, hipStream_t st) {
    AxisOp<M> op;
    for (int i = 0; i < M * 2 * M; ++i) op.k[i] = K1[i];
    const uint32_t ncell = (uint32_t)n * n * n;
    hipLaunchKernelGGL(advect_kernel<M>, dim3((ncell + kThreads - 1) / kThreads), dim3(kThreads), 0, st, src, dst,
                       op, (uint32_t)n, pitch, (uint32_t)off);
    return hipGetLastError();
}

// Two-kernel variant, evolution half: R holds each cell's monomial
// coefficients R[k3][k2][k1] (P^3 columns); the evolved polynomial
// p(xi + lam (1,1,1)) keeps y[j] = sum_k E1[j3][k3] E1[j2][k2] E1[j1][k1] R[k],
// j <= m, sum-factorised like the fused kernel (one lane per cell, streaming
// over (k3, k2), E1 as scalar operands): M P^3 + M^2 P^2 + M^3 P FMAs.
template <int M>
struct EvolveOp {
    double e[M * 2 * M];  // E1[j][k], row-major, k < P
};

template <int M>
__global__ __launch_bounds__(kThreads, kMinWaves<M>) void advect_evolve_kernel(const double* __restrict__ R,
                                                                 double* __restrict__ dst, EvolveOp<M> E,
                                                                 uint32_t n, size_t pitch, uint32_t off) {
    constexpr int P = 2 * M, M3 = M * M * M;
    const uint32_t cell = blockIdx.x * kThreads + threadIdx.x;
    if (cell >= n * n * n) return;
    const Cell16 c = cell_nodes(cell, n, off);
    double y[M3];
#pragma unroll
    for (int t = 0; t < M3; ++t) y[t] = 0.0;
    // high orders (small terms) first
#pragma unroll
    for (int k3 = P - 1; k3 >= 0; --k3) {
        double Y[M * M];
#pragma unroll
        for (int t = 0; t < M * M; ++t) Y[t] = 0.0;
#pragma unroll
        for (int k2 = P - 1; k2 >= 0; --k2) {
            double x[P];
#pragma unroll
            for (int k1 = 0; k1 < P; ++k1) x[k1] = R[(size_t)((k3 * P + k2) * P + k1) * pitch + cell];
#pragma unroll
            for (int j1 = 0; j1 < M; ++j1) {
                double z = 0.0;
#pragma unroll
                for (int k1 = P - 1; k1 >= j1; --k1) z = __builtin_fma(E.e[j1 * P + k1], x[k1], z);
#pragma unroll
                for (int j2 = 0; j2 < M; ++j2)
                    if (k2 >= j2) Y[j2 * M + j1] = __builtin_fma(E.e[j2 * P + k2], z, Y[j2 * M + j1]);
            }
        }
#pragma unroll
        for (int j3 = 0; j3 < M; ++j3)
            if (k3 >= j3)
#pragma unroll
                for (int t = 0; t < M * M; ++t)
                    y[j3 * M * M + t] = __builtin_fma(E.e[j3 * P + k3], Y[t], y[j3 * M * M + t]);
    }
#pragma unroll
    for (int t = 0; t < M3; ++t) dst[(size_t)t * pitch + c.out] = y[t];
}

template <int M>
hipError_t launch_evolve_m(const double* R, double* dst, const double* E1, int n, size_t pitch, int off,
                           hipStream_t st) {
    EvolveOp<M> op;
    for (int i = 0; i < M * 2 * M; ++i) op.e[i] = E1[i];
    const uint32_t ncell = (uint32_t)n * n * n;
    hipLaunchKernelGGL(advect_evolve_kernel<M>, dim3((ncell + kThreads - 1) / kThreads), dim3(kThreads), 0, st, R,
                       dst, op, (uint32_t)n, pitch, (uint32_t)off);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_advect_evolve(int m, const double* R, double* dst, const double* E1, int n, size_t pitch, int off,
                                hipStream_t st) {
    switch (m) {
        case 1: return launch_evolve_m<2>(R, dst, E1, n, pitch, off, st);
        case 2: return launch_evolve_m<3>(R, dst, E1, n, pitch, off, st);
        case 3: return launch_evolve_m<4>(R, dst, E1, n, pitch, off, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_advect(int m, const double* src, double* dst, const double* K1, int n, size_t pitch, int off,
                         hipStream_t st) {
    switch (m) {
        case 1: return launch_m<2>(src, dst, K1, n, pitch, off, st);
        case 2: return launch_m<3>(src, dst, K1, n, pitch, off, st);
        case 3: return launch_m<4>(src, dst, K1, n, pitch, off, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hermite
