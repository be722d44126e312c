// Fused Hermite half step for m = 3 on the FP64 matrix cores of gfx950.
//
// Per cell and parity class the half step is a dense 16 x 128 map (16 new
// node values: 2 fields x 2x2x2 derivative orders of that parity; 128 class
// inputs: 2 fields x 64 derivative multi-indices, each the signed 2x2x2
// butterfly of the 8 corner values). Sixteen cells side by side make it a
// 16 x 128 x 16 product per class, i.e. 32 v_mfma_f64_16x16x4f64 steps:
//   A (16 x 4): the class operator, rows = outputs, 4 input columns per step,
//   B (4 x 16): the class inputs of those 4 columns for the 16 cells,
//   D (16 x 16): accumulated outputs; register r of lane l holds row
//      4r + l/16 of column (cell) l%16 (the FP64 16x16x4 output layout).
// The operator rows are stored permuted (row 4r + g of A holds logical row
// 4g + r) so that register r of lane quarter g ends up with logical output
// row 4g + r: the quarter g = (field, o3) and r = (o2, o1).
// Lane l = (quarter q = l/16, cell l%16) loads the 8 corners of input column
// q of the current step for its cell and forms all 8 butterfly outputs, one
// per class. The 4 columns of a step share the parity pattern of d, so the
// butterfly output that feeds each class is fixed at compile time.
// The eight class operators (8 x 32 x 64 doubles = 128 KB) are staged once
// per workgroup in LDS, already permuted to lane order; each MFMA reads its
// A operand with one conflict-free ds_read_b64 per lane.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "mfma_order.h"

namespace hermite {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;                 // waves per workgroup (2 per SIMD)
constexpr int kOpDoubles = 8 * 32 * 64;   // class operators in lane order

struct Cell16 {
    uint32_t corner[8];
    uint32_t out;
};

__device__ __forceinline__ Cell16 cell_nodes(uint32_t cell, uint32_t n, uint32_t off) {
    const uint32_t i = cell % n, t = cell / n, j = t % n, k = t / n;
    const uint32_t i1 = (i + 1 == n) ? 0 : i + 1, j1 = (j + 1 == n) ? 0 : j + 1, k1 = (k + 1 == n) ? 0 : k + 1;
    Cell16 c;
    const uint32_t xs[2] = {i, i1}, ys[2] = {j, j1}, zs[2] = {k, k1};
#pragma unroll
    for (int s = 0; s < 8; ++s) c.corner[s] = (zs[s >> 2] * n + ys[(s >> 1) & 1]) * n + xs[s & 1];
    c.out = ((off ? k1 : k) * n + (off ? j1 : j)) * n + (off ? i1 : i);
    return c;
}

// Butterfly of the 8 corner values v[s1 + 2 s2 + 4 s3] of one derivative
// multi-index: T[t1 + 2 t2 + 4 t3] = sum_s prod_x (t_x ? (s_x ? 1 : -1) : 1) v[s]
// (t_x = 1: right minus left along x, t_x = 0: right plus left).
__device__ __forceinline__ void butterfly8(const double* v, double* T) {
    double a[8], b[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        a[2 * q] = v[2 * q + 1] + v[2 * q];
        a[2 * q + 1] = v[2 * q + 1] - v[2 * q];
    }
    // a index: t1 + 2*(s2 + 2 s3)
#pragma unroll
    for (int s3 = 0; s3 < 2; ++s3)
#pragma unroll
        for (int t1 = 0; t1 < 2; ++t1) {
            const double l = a[t1 + 2 * (0 + 2 * s3)], r = a[t1 + 2 * (1 + 2 * s3)];
            b[t1 + 2 * 0 + 4 * s3] = r + l;
            b[t1 + 2 * 1 + 4 * s3] = r - l;
        }
    // b index: t1 + 2 t2 + 4 s3
#pragma unroll
    for (int t12 = 0; t12 < 4; ++t12) {
        const double l = b[t12], r = b[t12 + 4];
        T[t12] = r + l;
        T[t12 + 4] = r - l;
    }
}

template <int T>
__device__ __forceinline__ void load_step(const double* __restrict__ src, size_t plane, const Cell16& c, int q,
                                          double* v) {
    constexpr MfmaSchedule S{};
    constexpr int c0 = S.col[T][0], c1 = S.col[T][1], c2 = S.col[T][2], c3 = S.col[T][3];
    const int col = (q == 0) ? c0 : (q == 1) ? c1 : (q == 2) ? c2 : c3;
    const double* __restrict__ b = src + (size_t)col * plane;
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = b[c.corner[s]];
}

// One K-step: the corner values of this step (v) were loaded one step ahead;
// the loads of the next step are issued before this step's MFMAs so that
// their latency hides behind the matrix work. The scheduling barrier keeps
// the compiler from hoisting every step's loads (which would spill).
template <int T>
struct Steps {
    __device__ __forceinline__ static void run(const double* __restrict__ src, size_t plane, const Cell16& c, int q,
                                               int lane, const double* sK, d4* acc, double* v) {
        constexpr MfmaSchedule S{};
        constexpr int dp = S.dpar[T];
        double vn[8];
        if constexpr (T + 1 < 32) load_step<T + 1>(src, plane, c, q, vn);
        double Tv[8];
        butterfly8(v, Tv);
        // class p takes the butterfly output t = p xor (d mod 2): a sum along
        // x when p_x and d_x agree, a difference otherwise
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const double a = sK[(p * 32 + T) * 64 + lane];
            acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Tv[p ^ dp], acc[p], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (T + 1 < 32) {
#pragma unroll
            for (int s = 0; s < 8; ++s) v[s] = vn[s];
            Steps<T + 1>::run(src, plane, c, q, lane, sK, acc, v);
        }
    }
};

// Persistent: gridDim.x is a multiple of 8 (one workgroup per CU). Workgroup
// b runs on XCD b % 8; logical block (b % 8) * (G/8) + b/8 gives each XCD one
// contiguous range of the domain, so node rows shared by neighbouring cells
// meet in that XCD's L2.
__global__ __launch_bounds__(kWaves * 64) void fused_mfma_kernel(const double* __restrict__ src,
                                                                 double* __restrict__ dst,
                                                                 const double* __restrict__ Kperm, uint32_t n,
                                                                 uint32_t off, uint32_t nbatch) {
    __shared__ double sK[kOpDoubles];
    for (int i = threadIdx.x; i < kOpDoubles; i += blockDim.x) sK[i] = Kperm[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane & 15, q = lane >> 4;
    const uint32_t ncell = n * n * n;
    const size_t plane = ncell;
    const uint32_t G = gridDim.x;
    const uint32_t lb = (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;
    const uint32_t per = (nbatch + G - 1) / G;
    const uint32_t b0 = lb * per;
    const uint32_t b1 = (b0 + per < nbatch) ? b0 + per : nbatch;
    for (uint32_t bt = b0 + wave; bt < b1; bt += kWaves) {
        const uint32_t cell = bt * 16 + cl;
        const bool valid = cell < ncell;
        const Cell16 c = cell_nodes(valid ? cell : 0u, n, off);
        d4 acc[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) acc[p] = d4{0.0, 0.0, 0.0, 0.0};
        double v[8];
        load_step<0>(src, plane, c, q, v);
        Steps<0>::run(src, plane, c, q, lane, sK, acc, v);
        if (!valid) continue;
        // logical output row 4q + r of class p (register r of quarter q): field q/2,
        // derivative orders j = p + 2 (o1, o2, o3) with o3 = q % 2, o2 = r / 2, o1 = r % 2
        const int fo = q >> 1, o3 = q & 1;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int p1 = p & 1, p2 = (p >> 1) & 1, p3 = p >> 2;
            const int j3 = p3 + 2 * o3;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j1 = p1 + 2 * (r & 1), j2 = p2 + 2 * (r >> 1);
                dst[(size_t)(fo * 64 + (j3 * 4 + j2) * 4 + j1) * plane + c.out] = acc[p][r];
            }
        }
    }
}

}  // namespace

size_t mfma_operator_doubles() { return (size_t)kOpDoubles; }

void mfma_permute_operators(const double* K, double* Kperm) {
    // K: [8][16][128] canonical class operators (rows (fo, o3, o2, o1), columns
    // f*64 + dd). A operand of step t: lane l holds A[l % 16][l / 16]. The
    // MFMA leaves output row i in register i / 4 of lane quarter i % 4, so A
    // row i carries logical row 4 (i % 4) + i / 4: register r of quarter g then
    // holds logical row 4g + r.
    //   Kperm[p][t][lane] = K[p][4 (i % 4) + i / 4][col(t, lane / 16)], i = lane % 16
    constexpr MfmaSchedule S{};
    for (int p = 0; p < 8; ++p)
        for (int t = 0; t < 32; ++t)
            for (int lane = 0; lane < 64; ++lane) {
                const int i = lane & 15, row = 4 * (i & 3) + (i >> 2);
                Kperm[((size_t)p * 32 + t) * 64 + lane] = K[((size_t)p * 16 + row) * 128 + S.col[t][lane >> 4]];
            }
}

hipError_t launch_fused_mfma(const double* src, double* dst, const double* Kperm, int n, int off, int grid,
                             hipStream_t st) {
    const uint32_t ncell = (uint32_t)n * n * n;
    const uint32_t nbatch = (ncell + 15) / 16;
    if (grid < 8 || grid % 8 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fused_mfma_kernel, dim3(grid), dim3(kWaves * 64), 0, st, src, dst, Kperm, (uint32_t)n,
                       (uint32_t)off, nbatch);
    return hipGetLastError();
}

}  // namespace hermite
