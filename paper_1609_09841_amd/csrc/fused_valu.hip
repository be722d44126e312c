// Fused Hermite half steps in FP64 on the vector ALUs: the m = 3 variant of
// the matrix-core kernel, and the m = 1, 2 kernels.
//
// One lane per cell and output field. Per parity class p the half step is
// the dense map y_p = K_p x_p (16 new values x 128 class inputs, the class
// inputs being the 2x2x2 butterflies of the corner data); a lane computes the
// 8 new values of its field for all 8 classes (64 accumulators). The operator
// entries are wave-uniform, so they come from scalar loads and enter the FMAs
// as scalar operands. Each input column is loaded as 8 corner values per lane
// (64 consecutive cells per load instruction, one column, contiguous), formed
// into its 8 butterfly outputs once and used by all 8 classes.
//
// Column order: 16 rounds; round r takes, for each parity pattern of d, the
// r-th column of that pattern in order of decreasing |d| (field v before u),
// so the small high-order inputs are summed first.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch_common.h"
#include "fused_common.h"
#include "kernels.h"

namespace hermite {
namespace {

using fused::butterfly8;
using fused::Cell16;
using fused::cell_writing;

constexpr int kThreads = 256;

__device__ __forceinline__ void load_col(const double* __restrict__ src, size_t pitch, const Cell16& c, int col,
                                         double* v) {
    const double* __restrict__ b = src + (size_t)col * pitch;
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = b[c.corner[s]];
}

struct RoundTable {
    int col[16][8];  // col[r][dpar]
    constexpr RoundTable() : col() {
        int cnt[8] = {};
        for (int s = 9; s >= 0; --s)
            for (int f = 1; f >= 0; --f)
                for (int d3 = 0; d3 < 4; ++d3)
                    for (int d2 = 0; d2 < 4; ++d2) {
                        const int d1 = s - d3 - d2;
                        if (d1 < 0 || d1 > 3) continue;
                        const int par = (d1 & 1) | ((d2 & 1) << 1) | ((d3 & 1) << 2);
                        col[cnt[par]++][par] = f * 64 + (d3 * 4 + d2) * 4 + d1;
                    }
    }
};
__constant__ RoundTable kRounds = RoundTable();

__global__ __launch_bounds__(kThreads) void fused_valu4_kernel(const double* __restrict__ src,
                                                               double* __restrict__ dst,
                                                               const double* __restrict__ Kv, uint32_t n,
                                                               size_t pitch, uint32_t off) {
    const uint32_t ncell = n * n * n;
    const uint32_t fo = blockIdx.x & 1;
    const uint32_t node = (blockIdx.x >> 1) * kThreads + threadIdx.x;  // new node this lane writes
    const bool valid = node < ncell;
    const Cell16 c = cell_writing(valid ? node : 0u, n, off);
    const double* __restrict__ Kf = Kv + (size_t)fo * (128 * 64);
    double acc[8][8];
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int r = 0; r < 8; ++r) acc[p][r] = 0.0;
    for (int rd = 0; rd < 16; ++rd) {
#pragma unroll
        for (int dp = 0; dp < 8; ++dp) {
            double v[8];
            load_col(src, pitch, c, kRounds.col[rd][dp], v);
            double T[8];
            butterfly8(v, T);
            const double* __restrict__ kk = Kf + (rd * 8 + dp) * 64;  // [class][row]
            // class p takes the butterfly output p xor (d mod 2)
#pragma unroll
            for (int p = 0; p < 8; ++p)
#pragma unroll
                for (int r = 0; r < 8; ++r) acc[p][r] = __builtin_fma(kk[p * 8 + r], T[p ^ dp], acc[p][r]);
        }
    }
    if (!valid) return;
    // row r = (o3, o2, o1) of class p: derivative orders j = p + 2 o
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int p1 = p & 1, p2 = (p >> 1) & 1, p3 = p >> 2;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int j1 = p1 + 2 * (r & 1), j2 = p2 + 2 * ((r >> 1) & 1), j3 = p3 + 2 * (r >> 2);
            dst[(size_t)(fo * 64 + (j3 * 4 + j2) * 4 + j1) * pitch + c.out] = acc[p][r];
        }
    }
}

// ---------------------------------------------------------------------------
// m = 1, 2: one lane per cell computes all 2 M^3 new values. Columns (all
// 2 M^3 input columns, small |d| last) are fully unrolled, so the parity
// pattern of each column and the class each accumulator belongs to are
// compile-time constants; the operator is dense per column over all classes'
// outputs (the class inputs differ per class: butterfly output p xor par(d)).
// ---------------------------------------------------------------------------
template <int M>
struct SmallLayout {
    static constexpr int M3 = M * M * M, NC = 2 * M3, NO = 2 * M3;
    int col[NC];          // columns in accumulation order
    int out_class[NO];    // class of output slot o
    int out_j[NO];        // destination row fo * M3 + (j3 M + j2) M + j1 of slot o
    int out_row[NO];      // row of slot o in its class operator (canonical order)
    bool zero[NC][NO];    // entry (column step C, slot o) vanishes for every time step
    constexpr SmallLayout() : col(), out_class(), out_j(), out_row(), zero() {
        int k = 0;
        for (int s = 3 * (M - 1); s >= 0; --s)
            for (int f = 1; f >= 0; --f)
                for (int d3 = 0; d3 < M; ++d3)
                    for (int d2 = 0; d2 < M; ++d2) {
                        const int d1 = s - d3 - d2;
                        if (d1 < 0 || d1 >= M) continue;
                        col[k++] = f * M3 + (d3 * M + d2) * M + d1;
                    }
        int o = 0;
        for (int p = 0; p < 8; ++p) {
            const int p1 = p & 1, p2 = (p >> 1) & 1, p3 = p >> 2;
            const int n1 = (M + 1 - p1) / 2, n2 = (M + 1 - p2) / 2, n3 = (M + 1 - p3) / 2, nof = n1 * n2 * n3;
            for (int fo = 0; fo < 2; ++fo)
                for (int o3 = 0; o3 < n3; ++o3)
                    for (int o2 = 0; o2 < n2; ++o2)
                        for (int o1 = 0; o1 < n1; ++o1) {
                            out_class[o] = p;
                            out_row[o] = fo * nof + (o3 * n2 + o2) * n1 + o1;
                            const int j1 = p1 + 2 * o1, j2 = p2 + 2 * o2, j3 = p3 + 2 * o3;
                            out_j[o] = fo * M3 + (j3 * M + j2) * M + j1;
                            // Along an axis with even class parity, new order
                            // j_x = 2 takes nothing from input order d_x = 0: the
                            // even part of the 1D interpolant has no such term and
                            // the evolution lowers orders in steps of two.
                            for (int c = 0; c < NC; ++c) {
                                const int dd = col[c] % M3;
                                const int d1 = dd % M, d2 = (dd / M) % M, d3 = dd / (M * M);
                                zero[c][o] = (p1 == 0 && o1 == 1 && d1 == 0) || (p2 == 0 && o2 == 1 && d2 == 0) ||
                                             (p3 == 0 && o3 == 1 && d3 == 0);
                            }
                            ++o;
                        }
        }
    }
    static constexpr int parity(int c) {
        const int dd = c % M3;
        const int d1 = dd % M, d2 = (dd / M) % M, d3 = dd / (M * M);
        return (d1 & 1) | ((d2 & 1) << 1) | ((d3 & 1) << 2);
    }
};

template <int M, int C>
struct SmallCols {
    __device__ __forceinline__ static void run(const double* __restrict__ src, size_t pitch, const Cell16& cc,
                                               const double* __restrict__ Kv, double* acc) {
        constexpr SmallLayout<M> L{};
        constexpr int NO = SmallLayout<M>::NO;
        constexpr int col = L.col[C], par = SmallLayout<M>::parity(col);
        double v[8];
        load_col(src, pitch, cc, col, v);
        double T[8];
        butterfly8(v, T);
        const double* __restrict__ kk = Kv + C * NO;
#pragma unroll
        for (int o = 0; o < NO; ++o)
            if (!L.zero[C][o]) acc[o] = __builtin_fma(kk[o], T[L.out_class[o] ^ par], acc[o]);
        if constexpr (C + 1 < SmallLayout<M>::NC) SmallCols<M, C + 1>::run(src, pitch, cc, Kv, acc);
    }
};

template <int M>
__device__ __forceinline__ void small_cell(const double* __restrict__ src, double* __restrict__ dst,
                                           const double* __restrict__ Kv, uint32_t n, size_t pitch, uint32_t off,
                                           uint32_t node) {
    constexpr SmallLayout<M> L{};
    constexpr int NO = SmallLayout<M>::NO;
    const Cell16 c = cell_writing(node, n, off);
    double acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = 0.0;
    SmallCols<M, 0>::run(src, pitch, c, Kv, acc);
#pragma unroll
    for (int o = 0; o < NO; ++o) dst[(size_t)L.out_j[o] * pitch + c.out] = acc[o];
}

template <int M>
__global__ __launch_bounds__(kThreads) void fused_valu_small_kernel(const double* __restrict__ src,
                                                                    double* __restrict__ dst,
                                                                    const double* __restrict__ Kv, uint32_t n,
                                                                    size_t pitch, uint32_t off) {
    const uint32_t node = blockIdx.x * kThreads + threadIdx.x;
    if (node >= n * n * n) return;
    small_cell<M>(src, dst, Kv, n, pitch, off, node);
}

// Batched: work item = a block of BS cells of one shot (batch_common.h).
template <int M, int BS>
__global__ __launch_bounds__(BS) void fused_valu_small_batch_kernel(const batch::ShotGrid* __restrict__ shots,
                                                                    const uint32_t* __restrict__ ids,
                                                                    const uint32_t* __restrict__ prefix, uint32_t ng,
                                                                    uint32_t from, const double* __restrict__ Kv) {
    const uint32_t g = batch::find_entry(prefix, ng, blockIdx.x);
    const batch::ShotGrid& S = shots[ids[g]];
    const uint32_t n = S.n;
    const uint32_t node = (blockIdx.x - prefix[g]) * BS + threadIdx.x;
    if (node >= n * n * n) return;
    small_cell<M>(S.grid[from], S.grid[1 - from], Kv, n, S.pitch, from, node);
}

template <int M>
hipError_t launch_small_batch(int bs, const batch::ShotGrid* shots, const uint32_t* ids, const uint32_t* prefix,
                              uint32_t ng, uint32_t blocks, int from, const double* Kv, hipStream_t st) {
    if (bs == 64)
        hipLaunchKernelGGL((fused_valu_small_batch_kernel<M, 64>), dim3(blocks), dim3(64), 0, st, shots, ids, prefix,
                           ng, (uint32_t)from, Kv);
    else if (bs == 128)
        hipLaunchKernelGGL((fused_valu_small_batch_kernel<M, 128>), dim3(blocks), dim3(128), 0, st, shots, ids,
                           prefix, ng, (uint32_t)from, Kv);
    else if (bs == 256)
        hipLaunchKernelGGL((fused_valu_small_batch_kernel<M, 256>), dim3(blocks), dim3(256), 0, st, shots, ids,
                           prefix, ng, (uint32_t)from, Kv);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int M>
bool small_build(const double* K, double* Kv) {
    constexpr SmallLayout<M> L{};
    constexpr int NO = SmallLayout<M>::NO, NC = SmallLayout<M>::NC;
    const int no0 = (M + 1) / 2, RM = 2 * no0 * no0 * no0;
    bool ok = true;
    for (int c = 0; c < NC; ++c)
        for (int o = 0; o < NO; ++o) {
            const double k = K[((size_t)L.out_class[o] * RM + L.out_row[o]) * NC + L.col[c]];
            Kv[(size_t)c * NO + o] = k;
            ok = ok && (!L.zero[c][o] || k == 0.0);
        }
    return ok;
}

}  // namespace

size_t valu_small_operator_doubles(int m) { return (size_t)(2 * (m + 1) * (m + 1) * (m + 1)) * (2 * (m + 1) * (m + 1) * (m + 1)); }

bool valu_small_build_operators(int m, const double* K, double* Kv) {
    if (m == 1) return small_build<2>(K, Kv);
    if (m == 2) return small_build<3>(K, Kv);
    return false;
}

hipError_t launch_fused_valu_small(int m, const double* src, double* dst, const double* Kv, int n, size_t pitch,
                                   int off, hipStream_t st) {
    const uint32_t ncell = (uint32_t)n * n * n;
    const dim3 grid((ncell + kThreads - 1) / kThreads), block(kThreads);
    if (m == 1)
        hipLaunchKernelGGL(fused_valu_small_kernel<2>, grid, block, 0, st, src, dst, Kv, (uint32_t)n, pitch,
                           (uint32_t)off);
    else if (m == 2)
        hipLaunchKernelGGL(fused_valu_small_kernel<3>, grid, block, 0, st, src, dst, Kv, (uint32_t)n, pitch,
                           (uint32_t)off);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_fused_valu_small_batch(int m, int block, const batch::ShotGrid* shots, const uint32_t* ids,
                                         const uint32_t* prefix, uint32_t ng, uint32_t blocks, int from,
                                         const double* Kv, hipStream_t st) {
    if (blocks == 0) return hipSuccess;
    if (m == 1) return launch_small_batch<2>(block, shots, ids, prefix, ng, blocks, from, Kv, st);
    if (m == 2) return launch_small_batch<3>(block, shots, ids, prefix, ng, blocks, from, Kv, st);
    return hipErrorInvalidValue;
}

size_t valu4_operator_doubles() { return (size_t)2 * 128 * 64; }

void valu4_build_operators(const double* K, double* Kv) {
    // K: [8][16][128] canonical class operators (rows (fo, o3, o2, o1), columns
    // f*64 + dd). Kv[fo][round][dpar][class][row] with row = (o3, o2, o1).
    constexpr RoundTable R{};
    for (int fo = 0; fo < 2; ++fo)
        for (int rd = 0; rd < 16; ++rd)
            for (int dp = 0; dp < 8; ++dp)
                for (int p = 0; p < 8; ++p)
                    for (int r = 0; r < 8; ++r)
                        Kv[((((size_t)fo * 16 + rd) * 8 + dp) * 8 + p) * 8 + r] =
                            K[((size_t)p * 16 + fo * 8 + r) * 128 + R.col[rd][dp]];
}

hipError_t launch_fused_valu4(const double* src, double* dst, const double* Kv, int n, size_t pitch, int off,
                              hipStream_t st) {
    const uint32_t ncell = (uint32_t)n * n * n;
    const uint32_t blocks = 2 * ((ncell + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(fused_valu4_kernel, dim3(blocks), dim3(kThreads), 0, st, src, dst, Kv, (uint32_t)n, pitch,
                       (uint32_t)off);
    return hipGetLastError();
}

}  // namespace hermite
