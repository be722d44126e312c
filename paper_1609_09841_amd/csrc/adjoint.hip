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
// m = 1, 2 (adjoint_kernel): one lane per (node, input field fi), M^3
// accumulators; the 8 cells are a runtime loop, classes, class rows and
// columns are unrolled, so the operator entries are wave-uniform scalar
// operands. This repeats each cell's transposed contraction at its 8
// vertices; m = 3 (adjoint_mfma_kernel below) computes it once per cell on
// the matrix cores and sums the vertex contributions in a second pass.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fused_common.h"
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

// ---------------------------------------------------------------------------
// m = 3 on the FP64 matrix cores, scatter form. Per batch of 16 cells of one
// x-row (the forward kernels' XCD-blocked sweep), the transposed class
// products G_p = K_p^T Lam_p (128 columns x 16 cells, K = the 16 class rows)
// run as 8 column tiles x 8 classes x 4 K-steps of v_mfma_f64_16x16x4f64 -
// as many as the forward half step. The tile rows are ordered so that
// register r of lane quarter g holds column d = f 64 + (d3 4 + d2) 4 + d1 with
//   d1 = 2 (T & 1) + (r & 1), d2 = 2 ((T >> 1) & 1) + (r >> 1),
//   d3 = 2 (g & 1) + (T >> 2), f = g >> 1     (T: tile),
// so the parity of d, which says which class feeds which butterfly output,
// depends on (T, r) only. The transposed butterfly then gives the cell's 8
// vertex contributions e_s[d], stored to E[s][d][cell]; a second kernel sums,
// per node, the 8 contributions of the cells around it.
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kMfWaves = 8;
constexpr int kAdjOpDoubles = 8 * 8 * 4 * 64;  // [class][tile][K-step][lane]

struct AdjSrcCols {
    int col[8][4][4];  // [class][K-step][quarter] -> destination column of class row 4 ks + q
    constexpr AdjSrcCols() : col() {
        constexpr AdjLayout<4> L{};
        for (int p = 0; p < 8; ++p)
            for (int ks = 0; ks < 4; ++ks)
                for (int q = 0; q < 4; ++q) col[p][ks][q] = L.row_col[p][4 * ks + q];
    }
};
__constant__ AdjSrcCols kAdjSrcCols = AdjSrcCols();

__host__ __device__ constexpr int adj_col(int T, int g, int r) {
    const int d1 = 2 * (T & 1) + (r & 1), d2 = 2 * ((T >> 1) & 1) + (r >> 1), d3 = 2 * (g & 1) + (T >> 2);
    return (g >> 1) * 64 + (d3 * 4 + d2) * 4 + d1;
}
__host__ __device__ constexpr int adj_par(int T, int r) { return (r & 1) | (((r >> 1) & 1) << 1) | ((T >> 2) << 2); }

// e_s = sum_t sg(t, s) T_t: per axis, s_x = 0 takes T(t_x=0) - T(t_x=1), s_x = 1 the sum.
__device__ __forceinline__ void butterfly8_T(const double* T, double* e) {
    double a[8], b[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        a[2 * q] = T[2 * q] - T[2 * q + 1];
        a[2 * q + 1] = T[2 * q] + T[2 * q + 1];
    }
#pragma unroll
    for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
        for (int t3 = 0; t3 < 2; ++t3) {
            const double l = a[s1 + 4 * t3], r = a[s1 + 2 + 4 * t3];
            b[s1 + 4 * t3] = l - r;
            b[s1 + 2 + 4 * t3] = l + r;
        }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        e[k] = b[k] - b[k + 4];
        e[k + 4] = b[k] + b[k + 4];
    }
}

__global__ __launch_bounds__(kMfWaves * 64) void adjoint_mfma_kernel(const double* __restrict__ lam_dst,
                                                                     double* __restrict__ E,
                                                                     const double* __restrict__ KT, uint32_t n,
                                                                     size_t pitch, uint32_t off) {
    __shared__ double sK[kAdjOpDoubles];
    for (int i = threadIdx.x; i < kAdjOpDoubles; i += blockDim.x) sK[i] = KT[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane & 15, q = lane >> 4;
    fused::sweep_rows(n, wave, kMfWaves, [&](uint32_t x0, uint32_t y, uint32_t z) {
        const uint32_t x = x0 + cl;
        const bool valid = x < n;
        const uint32_t cell = (z * n + y) * n + (valid ? x : n - 1);
        const fused::Cell16 c = fused::cell_nodes(cell, n, off);
        // B operands: Lam_p rows 4 ks + q of this lane's cell (its new node)
        double lb[8][4];
#pragma unroll
        for (int p = 0; p < 8; ++p)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) lb[p][ks] = lam_dst[(size_t)kAdjSrcCols.col[p][ks][q] * pitch + c.out];
#pragma unroll
        for (int T = 0; T < 8; ++T) {
            d4 acc[8];
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                acc[p] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
                    acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(sK[((p * 8 + T) * 4 + ks) * 64 + lane], lb[p][ks],
                                                                  acc[p], 0, 0, 0);
            }
            if (valid) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // butterfly output t is fed by class t xor par(column), par fixed by (T, r)
                    const int par = adj_par(T, r);
                    double Tv[8], e[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) Tv[t] = acc[t ^ par][r];
                    butterfly8_T(Tv, e);
                    const int d = adj_col(T, q, r);
#pragma unroll
                    for (int sv = 0; sv < 8; ++sv) E[((size_t)sv * 128 + d) * pitch + cell] = e[sv];
                }
            }
        }
    });
}

// lam_src[col][node] = sum_s E[s][col][node - s] (periodic), in s order.
__global__ __launch_bounds__(kThreads) void adjoint_gather_kernel(const double* __restrict__ E,
                                                                  double* __restrict__ lam_src, uint32_t n,
                                                                  size_t pitch) {
    const uint32_t node = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t col = blockIdx.y;
    if (node >= n * n * n) return;
    const uint32_t i = node % n, t = node / n, j = t % n, k = t / n;
    double acc = 0.0;
#pragma unroll
    for (int sv = 0; sv < 8; ++sv) {
        const uint32_t ci = (i + n - (sv & 1)) % n, cj = (j + n - ((sv >> 1) & 1)) % n, ck = (k + n - (sv >> 2)) % n;
        acc += E[((size_t)sv * 128 + col) * pitch + ((size_t)ck * n + cj) * n + ci];
    }
    lam_src[(size_t)col * pitch + node] = acc;
}

}  // namespace

size_t adjoint_mfma_operator_doubles() { return (size_t)kAdjOpDoubles; }

void adjoint_mfma_build_operator(const double* K, double* KT) {
    // K: canonical [8][16][128]. A operand of (class p, tile T, K-step ks):
    // lane = i + 16 k, A[i][k] = K_p[4 ks + k][column of logical tile row
    // 4 (i % 4) + i / 4], whose register is i / 4 in quarter i % 4.
    for (int p = 0; p < 8; ++p)
        for (int T = 0; T < 8; ++T)
            for (int ks = 0; ks < 4; ++ks)
                for (int lane = 0; lane < 64; ++lane) {
                    const int i = lane & 15, k = lane >> 4;
                    const int g = i & 3, r = i >> 2;
                    KT[((p * 8 + T) * 4 + ks) * 64 + lane] = K[((size_t)p * 16 + 4 * ks + k) * 128 + adj_col(T, g, r)];
                }
}

hipError_t launch_adjoint_mfma(const double* lam_dst, double* lam_src, double* E, const double* KT, int n,
                               size_t pitch, int off, int grid, hipStream_t st) {
    if (grid < 8 || grid % 8 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(adjoint_mfma_kernel, dim3(grid), dim3(kMfWaves * 64), 0, st, lam_dst, E, KT, (uint32_t)n,
                       pitch, (uint32_t)off);
    const uint32_t ncell = (uint32_t)n * n * n;
    hipLaunchKernelGGL(adjoint_gather_kernel, dim3((ncell + kThreads - 1) / kThreads, 128), dim3(kThreads), 0, st,
                       (const double*)E, lam_src, (uint32_t)n, pitch);
    return hipGetLastError();
}

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
