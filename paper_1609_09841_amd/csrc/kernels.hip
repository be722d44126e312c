// Hermite half-step kernels for gfx950 (CDNA4): the two-kernel variant
// (interpolation, then evolution, Sec. 3.1-3.2) and the state scaling.
//
// Cell data flow (Sec. 2, Eq. 3; Sec. 3.1-3.2): gather the 8 vertices of a
// cell, interpolate (tensor Hermite, degree 2m+1 per axis), evolve through the
// half step, keep the coefficients with every index <= m as the new node data.
//
// Parity classes. The 1D Hermite matrix satisfies H[j][(L,k)] = (-1)^(j+k)
// H[j][(R,k)], so along each axis the coefficients of parity p depend only on
// c_p[k] = R_k + (-1)^(p+k) L_k (a sum or a difference of the two end values).
// Second derivatives shift an index by 2, so the evolution keeps parity too.
// A cell therefore splits into 8 independent parity classes p = (p1,p2,p3):
// the 8 corner values of one derivative multi-index d combine by a signed
// 2x2x2 butterfly into one input per class, and each class is an independent
// small dense map from its 2 M^3 inputs to its outputs.
//
// Accumulation order: inputs of high derivative order are small for smooth
// data and the d = 0 inputs are the largest, so every dot product runs from
// the highest |d| down to |d| = 0 (small terms first), which keeps FP64
// rounding of the sums below that of a plain ascending loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace hermite {
namespace {

__host__ __device__ constexpr int nout_c(int M, int p) { return (M + 1 - p) / 2; }

struct CellIdx {
    uint32_t corner[8];  // node index (k*n + j)*n + i of corner s = s1 + 2 s2 + 4 s3
    uint32_t out;        // destination node index
};

__device__ __forceinline__ CellIdx cell_index(uint32_t cell, uint32_t n, uint32_t off) {
    const uint32_t i = cell % n, t = cell / n, j = t % n, k = t / n;
    const uint32_t i1 = (i + 1 == n) ? 0 : i + 1, j1 = (j + 1 == n) ? 0 : j + 1, k1 = (k + 1 == n) ? 0 : k + 1;
    CellIdx c;
    const uint32_t xs[2] = {i, i1}, ys[2] = {j, j1}, zs[2] = {k, k1};
#pragma unroll
    for (int s = 0; s < 8; ++s) c.corner[s] = (zs[s >> 2] * n + ys[(s >> 1) & 1]) * n + xs[s & 1];
    const uint32_t oi = off ? i1 : i, oj = off ? j1 : j, ok = off ? k1 : k;
    c.out = (ok * n + oj) * n + oi;
    return c;
}

// Class input of one derivative multi-index: the signed butterfly
// sum_s prod_x sigma_x v[s] over the 8 corners, with sigma_x = 1 on the right
// (s_x = 1) and (-1)^(p_x + d_x) on the left. sg* are exactly +-1.
__device__ __forceinline__ double class_input(const double* __restrict__ b, const CellIdx& c, double sg1, double sg2,
                                              double sg3) {
    double v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = b[c.corner[s]];
    double a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = __builtin_fma(sg1, v[2 * q], v[2 * q + 1]);
    const double b0 = __builtin_fma(sg2, a[0], a[1]);
    const double b1 = __builtin_fma(sg2, a[2], a[3]);
    return __builtin_fma(sg3, b0, b1);
}

__device__ __forceinline__ double parity_sign(int p, int d) { return ((p + d) & 1) ? -1.0 : 1.0; }

// ---------------------------------------------------------------------------
// Two-kernel variant, interpolation: one thread per (cell, class, field);
// (field, class) is the fastest-varying part of the block index, so the 16
// blocks reading the same cells' corners run together.
// Applies the parity blocks of H along x1, x2, x3 (Alg. 2 restricted to one
// class) and writes the monomial coefficients R[f][k3][k2][k1][cell].
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(256) void interp_kernel(const double* __restrict__ src, double* __restrict__ R,
                                                     const double* __restrict__ Hp, uint32_t n, size_t pitch,
                                                     uint32_t nf) {
    constexpr int M3 = M * M * M, P = 2 * M, P3 = P * P * P;
    const uint32_t ncell = n * n * n;
    // blocks: (cell group, class, field) with field (of nf) fastest
    const uint32_t cell = (blockIdx.x / (8 * nf)) * 256u + threadIdx.x;
    if (cell >= ncell) return;
    const CellIdx c = cell_index(cell, n, 0);
    const int f = (int)(blockIdx.x % nf), pc = (int)((blockIdx.x / nf) & 7);
    const int p1 = pc & 1, p2 = (pc >> 1) & 1, p3 = pc >> 2;
    const double* __restrict__ H1 = Hp + p1 * M * M;
    const double* __restrict__ H2 = Hp + p2 * M * M;
    const double* __restrict__ H3 = Hp + p3 * M * M;
    const size_t plane = pitch;
    const double* __restrict__ srcf = src + (size_t)f * M3 * plane;
    double C[M3], T[M3];
#pragma unroll
    for (int d3 = 0; d3 < M; ++d3)
#pragma unroll
        for (int d2 = 0; d2 < M; ++d2)
#pragma unroll
            for (int d1 = 0; d1 < M; ++d1) {
                const int dd = (d3 * M + d2) * M + d1;
                C[dd] = class_input(srcf + (size_t)dd * plane, c, parity_sign(p1, d1), parity_sign(p2, d2),
                                    parity_sign(p3, d3));
            }
    // x1: T[d3][d2][i1] = sum_d1 H1[i1][d1] C[d3][d2][d1], highest order first
#pragma unroll
    for (int d3 = 0; d3 < M; ++d3)
#pragma unroll
        for (int d2 = 0; d2 < M; ++d2)
#pragma unroll
            for (int i1 = 0; i1 < M; ++i1) {
                double a = 0.0;
#pragma unroll
                for (int d1 = M - 1; d1 >= 0; --d1) a = __builtin_fma(H1[i1 * M + d1], C[(d3 * M + d2) * M + d1], a);
                T[(d3 * M + d2) * M + i1] = a;
            }
    // x2: C[d3][i2][i1] = sum_d2 H2[i2][d2] T[d3][d2][i1]
#pragma unroll
    for (int d3 = 0; d3 < M; ++d3)
#pragma unroll
        for (int i2 = 0; i2 < M; ++i2)
#pragma unroll
            for (int i1 = 0; i1 < M; ++i1) {
                double a = 0.0;
#pragma unroll
                for (int d2 = M - 1; d2 >= 0; --d2) a = __builtin_fma(H2[i2 * M + d2], T[(d3 * M + d2) * M + i1], a);
                C[(d3 * M + i2) * M + i1] = a;
            }
    // x3: R[i3][i2][i1] = sum_d3 H3[i3][d3] C[d3][i2][i1], stored at k = p + 2i
#pragma unroll
    for (int i3 = 0; i3 < M; ++i3)
#pragma unroll
        for (int i2 = 0; i2 < M; ++i2)
#pragma unroll
            for (int i1 = 0; i1 < M; ++i1) {
                double a = 0.0;
#pragma unroll
                for (int d3 = M - 1; d3 >= 0; --d3) a = __builtin_fma(H3[i3 * M + d3], C[(d3 * M + i2) * M + i1], a);
                const int k1 = p1 + 2 * i1, k2 = p2 + 2 * i2, k3 = p3 + 2 * i3;
                R[(size_t)(f * P3 + (k3 * P + k2) * P + k1) * plane + cell] = a;
            }
}

// ---------------------------------------------------------------------------
// Two-kernel variant, evolution: one thread per (cell, class, i3); the G
// lanes of a (cell, class) group hold the x3 slices of the class tensor and
// exchange the x3 neighbour for the Laplacian by a wavefront shuffle.
// The cell operator is L(a, b) = lam (b, Lap a) in the half-step time.
// ---------------------------------------------------------------------------
// Overwrites (Y_u, Y_v) by lam (Y_v, Lap Y_u) on this lane's x3 slice; nb is
// the slice i3+1 (zero above the top); (k+1)(k+2) at k = p + 2i. The update
// runs in ascending slice order, so the x1/x2 neighbours read are still old.
template <int M, int G>
__device__ __forceinline__ void apply_L(double* Yu, double* Yv, double lam, int i3, int p1, int p2, int p3) {
    constexpr int S2 = M * M;
    double nb[S2];
    const bool top = (i3 + 1 >= M);
#pragma unroll
    for (int x = 0; x < S2; ++x) {
        const double t = __shfl_down(Yu[x], 1, G);
        nb[x] = top ? 0.0 : t;
    }
    const int k3 = p3 + 2 * i3;
    const double c3 = (double)((k3 + 1) * (k3 + 2));
#pragma unroll
    for (int i2 = 0; i2 < M; ++i2)
#pragma unroll
        for (int i1 = 0; i1 < M; ++i1) {
            const int x = i2 * M + i1;
            double lap = c3 * nb[x];
            if (i2 + 1 < M) lap = __builtin_fma((double)((p2 + 2 * i2 + 1) * (p2 + 2 * i2 + 2)), Yu[x + M], lap);
            if (i1 + 1 < M) lap = __builtin_fma((double)((p1 + 2 * i1 + 1) * (p1 + 2 * i1 + 2)), Yu[x + 1], lap);
            const double t = Yv[x];
            Yv[x] = lam * lap;
            Yu[x] = lam * t;
        }
}

template <int M>
__global__ __launch_bounds__(256) void evolve_kernel(const double* __restrict__ R, double* __restrict__ dst,
                                                     uint32_t n, size_t pitch, uint32_t off, int evolution, int q,
                                                     int S, double lam) {
    constexpr int G = (M <= 2) ? 2 : 4;
    constexpr int SLOTS = 256 / G;
    constexpr int S2 = M * M, M3 = M * M * M, P = 2 * M, P3 = P * P * P;
    const uint32_t ncell = n * n * n;
    const int i3 = threadIdx.x % G;
    const uint32_t cell = (blockIdx.x >> 3) * SLOTS + threadIdx.x / G;
    const bool valid = cell < ncell;
    const uint32_t cc = valid ? cell : 0u;
    const CellIdx c = cell_index(cc, n, off);
    const int pc = blockIdx.x & 7;
    const int p1 = pc & 1, p2 = (pc >> 1) & 1, p3 = pc >> 2;
    const int k3 = p3 + 2 * i3;
    const bool live = valid && (i3 < M);
    const int k3r = live ? k3 : p3;  // padding lanes address a valid slice and discard it
    double Wu[S2], Wv[S2];
#pragma unroll
    for (int i2 = 0; i2 < M; ++i2)
#pragma unroll
        for (int i1 = 0; i1 < M; ++i1) {
            const int k1 = p1 + 2 * i1, k2 = p2 + 2 * i2;
            const size_t o = (size_t)((k3r * P + k2) * P + k1) * pitch + cc;
            Wu[i2 * M + i1] = live ? R[o] : 0.0;
            Wv[i2 * M + i1] = live ? R[o + (size_t)P3 * pitch] : 0.0;
        }
    if (evolution == 0) {
        // Alg. 4: W <- R + (1/k) L W for k = q..1 (simultaneous update)
        double Ru[S2], Rv[S2];
#pragma unroll
        for (int x = 0; x < S2; ++x) { Ru[x] = Wu[x]; Rv[x] = Wv[x]; }
        for (int kq = q; kq >= 1; --kq) {
            const double a = lam / (double)kq;
            apply_L<M, G>(Wu, Wv, a, i3, p1, p2, p3);
#pragma unroll
            for (int x = 0; x < S2; ++x) { Wu[x] += Ru[x]; Wv[x] += Rv[x]; }
        }
    } else {
        // classical RK4 on dW/dsigma = L W, S substeps of length 1/S
        const double dl = 1.0 / (double)S;
        for (int sub = 0; sub < S; ++sub) {
            double Yu[S2], Yv[S2], Au[S2], Av[S2];
#pragma unroll
            for (int x = 0; x < S2; ++x) { Yu[x] = Wu[x]; Yv[x] = Wv[x]; }
            apply_L<M, G>(Yu, Yv, lam, i3, p1, p2, p3);  // K1
#pragma unroll
            for (int x = 0; x < S2; ++x) {
                Au[x] = Yu[x]; Av[x] = Yv[x];
                Yu[x] = __builtin_fma(0.5 * dl, Yu[x], Wu[x]); Yv[x] = __builtin_fma(0.5 * dl, Yv[x], Wv[x]);
            }
            apply_L<M, G>(Yu, Yv, lam, i3, p1, p2, p3);  // K2
#pragma unroll
            for (int x = 0; x < S2; ++x) {
                Au[x] = __builtin_fma(2.0, Yu[x], Au[x]); Av[x] = __builtin_fma(2.0, Yv[x], Av[x]);
                Yu[x] = __builtin_fma(0.5 * dl, Yu[x], Wu[x]); Yv[x] = __builtin_fma(0.5 * dl, Yv[x], Wv[x]);
            }
            apply_L<M, G>(Yu, Yv, lam, i3, p1, p2, p3);  // K3
#pragma unroll
            for (int x = 0; x < S2; ++x) {
                Au[x] = __builtin_fma(2.0, Yu[x], Au[x]); Av[x] = __builtin_fma(2.0, Yv[x], Av[x]);
                Yu[x] = __builtin_fma(dl, Yu[x], Wu[x]); Yv[x] = __builtin_fma(dl, Yv[x], Wv[x]);
            }
            apply_L<M, G>(Yu, Yv, lam, i3, p1, p2, p3);  // K4
#pragma unroll
            for (int x = 0; x < S2; ++x) {
                Au[x] += Yu[x]; Av[x] += Yv[x];
                Wu[x] = __builtin_fma(dl / 6.0, Au[x], Wu[x]); Wv[x] = __builtin_fma(dl / 6.0, Av[x], Wv[x]);
            }
        }
    }
    if (!live || k3 > M - 1) return;
    const size_t plane = pitch;
#pragma unroll
    for (int i2 = 0; i2 < M; ++i2)
#pragma unroll
        for (int i1 = 0; i1 < M; ++i1) {
            const int k1 = p1 + 2 * i1, k2 = p2 + 2 * i2;
            if (k1 > M - 1 || k2 > M - 1) continue;
            const int dd = (k3 * M + k2) * M + k1;
            dst[(size_t)dd * plane + c.out] = Wu[i2 * M + i1];
            dst[(size_t)(M3 + dd) * plane + c.out] = Wv[i2 * M + i1];
        }
}

// dst[r * dpitch + c] = s * src[r * spitch + c] for rows r < gridDim.y and
// columns c < cols (dst may equal src).
__global__ void scale_kernel(double* __restrict__ dst, size_t dpitch, const double* __restrict__ src, size_t spitch,
                             double s, size_t cols) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const double* __restrict__ a = src + (size_t)blockIdx.y * spitch;
    double* __restrict__ b = dst + (size_t)blockIdx.y * dpitch;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cols; i += stride) b[i] = s * a[i];
}

// flag = 1 if any of rows x cols entries (row r at r * pitch) is NaN or Inf.
__global__ void nonfinite_kernel(const double* __restrict__ g, size_t pitch, size_t cols, int* __restrict__ flag) {
    const double* __restrict__ a = g + (size_t)blockIdx.y * pitch;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cols; i += stride) bad |= !isfinite(a[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

}  // namespace

hipError_t launch_nonfinite(const double* g, size_t pitch, size_t cols, int rows, int* flag, hipStream_t st) {
    const uint32_t bx = (uint32_t)std::min<size_t>((cols + 255) / 256, 1024);
    hipLaunchKernelGGL(nonfinite_kernel, dim3(bx, rows), dim3(256), 0, st, g, pitch, cols, flag);
    return hipGetLastError();
}

hipError_t launch_interp(int m, const double* src, double* R, const double* Hp, int n, size_t pitch, int nf,
                         hipStream_t st) {
    if (nf != 1 && nf != 2) return hipErrorInvalidValue;
    const uint32_t ncell = (uint32_t)n * n * n;
    const dim3 grid(8 * nf * ((ncell + 255) / 256)), block(256);
    const uint32_t un = (uint32_t)n, unf = (uint32_t)nf;
    switch (m) {
        case 1: hipLaunchKernelGGL(interp_kernel<2>, grid, block, 0, st, src, R, Hp, un, pitch, unf); break;
        case 2: hipLaunchKernelGGL(interp_kernel<3>, grid, block, 0, st, src, R, Hp, un, pitch, unf); break;
        case 3: hipLaunchKernelGGL(interp_kernel<4>, grid, block, 0, st, src, R, Hp, un, pitch, unf); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_evolve(int m, const double* R, double* dst, int n, size_t pitch, int off, int evolution, int q,
                         int S, double lam, hipStream_t st) {
    const uint32_t ncell = (uint32_t)n * n * n;
    const int G = (m + 1 <= 2) ? 2 : 4;
    const uint32_t slots = 256 / G;
    const dim3 grid(8 * ((ncell + slots - 1) / slots)), block(256);
    switch (m) {
        case 1: hipLaunchKernelGGL(evolve_kernel<2>, grid, block, 0, st, R, dst, (uint32_t)n, pitch, (uint32_t)off, evolution, q, S, lam); break;
        case 2: hipLaunchKernelGGL(evolve_kernel<3>, grid, block, 0, st, R, dst, (uint32_t)n, pitch, (uint32_t)off, evolution, q, S, lam); break;
        case 3: hipLaunchKernelGGL(evolve_kernel<4>, grid, block, 0, st, R, dst, (uint32_t)n, pitch, (uint32_t)off, evolution, q, S, lam); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_scale(double* dst, size_t dpitch, const double* src, size_t spitch, double s, size_t cols,
                        int rows, hipStream_t st) {
    if (cols == 0 || rows == 0) return hipSuccess;
    size_t blocks = (cols + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks, (unsigned)rows), dim3(256), 0, st, dst, dpitch, src, spitch,
                       s, cols);
    return hipGetLastError();
}

}  // namespace hermite
