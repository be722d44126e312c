// Adjoint (transpose) of the fused wave half step, and the receiver and
// source-gradient kernels of the adjoint sweep (FP64).
//
// Forward, per cell: the 8 vertices' values of each derivative index d
// combine by the signed 2x2x2 butterfly into one input per parity class,
// T_t[d] = sum_s sg(t, s) v_s[d] with sg(t, s) = prod_x (t_x ? (s_x ? 1 : -1)
// : 1), class p takes t = p xor par(d), and y_p = K_p x_p (the class
// operators of the fused kernels). Transposed, the adjoint of vertex s of a
// cell is
//   g_s[d] = sum_p sg(p xor par(d), s) sum_r K_p[r][d] lam_y[p, r],
// lam_y the adjoint of the cell's new node. A node is vertex s of the cell
// whose lower corner is node - s (per axis, periodic), whose new node is
// node - s + off; the kernel gathers the 8 contributions at each node (no
// scatter, no atomics, a fixed summation order).
//
// One lane per (node, input field fi): M^3 accumulators. The 8 cells are a
// runtime loop; classes, class rows and columns are unrolled, so the
// operator entries are wave-uniform scalar operands.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace hermite {
namespace {

constexpr int kThreads = 256;

template <int M>
struct AdjLayout {
    static constexpr int M3 = M * M * M;
    static constexpr int RM = 2 * ((M + 1) / 2) * ((M + 1) / 2) * ((M + 1) / 2);  // rows_max
    int nrows[8];
    int row_col[8][RM];  // destination column f * M^3 + (j3 M + j2) M + j1 of class row r
    constexpr AdjLayout() : nrows(), row_col() {
        for (int p = 0; p < 8; ++p) {
            const int p1 = p & 1, p2 = (p >> 1) & 1, p3 = p >> 2;
            const int n1 = (M + 1 - p1) / 2, n2 = (M + 1 - p2) / 2, n3 = (M + 1 - p3) / 2;
            int r = 0;
            for (int fo = 0; fo < 2; ++fo)
                for (int o3 = 0; o3 < n3; ++o3)
                    for (int o2 = 0; o2 < n2; ++o2)
                        for (int o1 = 0; o1 < n1; ++o1)
                            row_col[p][r++] = fo * M3 + ((p3 + 2 * o3) * M + (p2 + 2 * o2)) * M + (p1 + 2 * o1);
            nrows[p] = r;
        }
    }
    static constexpr int par(int d) {
        const int d1 = d % M, d2 = (d / M) % M, d3 = d / (M * M);
        return (d1 & 1) | ((d2 & 1) << 1) | ((d3 & 1) << 2);
    }
};

template <int M>
__global__ __launch_bounds__(kThreads) void adjoint_kernel(const double* __restrict__ lam_dst,
                                                           double* __restrict__ lam_src,
                                                           const double* __restrict__ K, uint32_t n, size_t pitch,
                                                           uint32_t off) {
    constexpr AdjLayout<M> L{};
    constexpr int M3 = AdjLayout<M>::M3, RM = AdjLayout<M>::RM;
    const uint32_t fi = blockIdx.x & 1;
    const uint32_t node = (blockIdx.x >> 1) * kThreads + threadIdx.x;
    if (node >= n * n * n) return;
    const uint32_t i = node % n, t = node / n, j = t % n, k = t / n;
    const double* __restrict__ Kf = K + (size_t)fi * M3;  // columns of input field fi
    double acc[M3];
#pragma unroll
    for (int d = 0; d < M3; ++d) acc[d] = 0.0;
    for (int s = 0; s < 8; ++s) {
        const uint32_t s1 = s & 1, s2 = (s >> 1) & 1, s3 = s >> 2;
        // new node of the cell with lower corner node - s: node - s + off
        const uint32_t oi = (i + n - s1 + off) % n, oj = (j + n - s2 + off) % n, ok = (k + n - s3 + off) % n;
        const size_t out = ((size_t)ok * n + oj) * n + oi;
        double sg[8];
#pragma unroll
        for (int tt = 0; tt < 8; ++tt) sg[tt] = (__builtin_popcount((unsigned)tt & ~(unsigned)s & 7u) & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            double lp[RM];
#pragma unroll
            for (int r = 0; r < L.nrows[p]; ++r) lp[r] = lam_dst[(size_t)L.row_col[p][r] * pitch + out];
#pragma unroll
            for (int d = 0; d < M3; ++d) {
                double h = 0.0;
#pragma unroll
                for (int r = 0; r < L.nrows[p]; ++r) h = __builtin_fma(Kf[((size_t)p * RM + r) * 2 * M3 + d], lp[r], h);
                acc[d] = __builtin_fma(sg[p ^ AdjLayout<M>::par(d)], h, acc[d]);
            }
        }
    }
#pragma unroll
    for (int d = 0; d < M3; ++d) lam_src[(size_t)(fi * M3 + d) * pitch + node] = acc[d];
}

// traces[r] = u (d = 0) at receiver node nodes[r] of the primal grid.
__global__ void record_kernel(const double* __restrict__ grid, const uint32_t* __restrict__ nodes, uint32_t nr,
                              double* __restrict__ traces) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nr) traces[r] = grid[nodes[r]];
}

// lam[col 0][nodes[r]] += res[r], in receiver order by one thread (two
// receivers may share a node).
__global__ void inject_kernel(double* __restrict__ lam, const uint32_t* __restrict__ nodes, uint32_t nr,
                              const double* __restrict__ res) {
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (uint32_t r = 0; r < nr; ++r) lam[nodes[r]] += res[r];
}

}  // namespace

hipError_t launch_adjoint(int m, const double* lam_dst, double* lam_src, const double* K, int n, size_t pitch, int off,
                          hipStream_t st) {
    const uint32_t ncell = (uint32_t)n * n * n;
    const dim3 grid(2 * ((ncell + kThreads - 1) / kThreads)), block(kThreads);
    switch (m) {
        case 1: hipLaunchKernelGGL(adjoint_kernel<2>, grid, block, 0, st, lam_dst, lam_src, K, (uint32_t)n, pitch, (uint32_t)off); break;
        case 2: hipLaunchKernelGGL(adjoint_kernel<3>, grid, block, 0, st, lam_dst, lam_src, K, (uint32_t)n, pitch, (uint32_t)off); break;
        case 3: hipLaunchKernelGGL(adjoint_kernel<4>, grid, block, 0, st, lam_dst, lam_src, K, (uint32_t)n, pitch, (uint32_t)off); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_record(const double* grid, const uint32_t* nodes, uint32_t nr, double* traces, hipStream_t st) {
    if (nr == 0) return hipSuccess;
    hipLaunchKernelGGL(record_kernel, dim3((nr + 255) / 256), dim3(256), 0, st, grid, nodes, nr, traces);
    return hipGetLastError();
}

hipError_t launch_inject(double* lam, const uint32_t* nodes, uint32_t nr, const double* res, hipStream_t st) {
    if (nr == 0) return hipSuccess;
    hipLaunchKernelGGL(inject_kernel, dim3(1), dim3(64), 0, st, lam, nodes, nr, res);
    return hipGetLastError();
}

}  // namespace hermite
