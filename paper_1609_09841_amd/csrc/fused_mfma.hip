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

#include "batch_common.h"
#include "fused_common.h"
#include "kernels.h"
#include "mfma_order.h"

namespace hermite {
namespace {

using fused::butterfly8;
using fused::Cell16;
using fused::cell_nodes;

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;                 // waves per workgroup (2 per SIMD)
constexpr int kOpDoubles = 8 * 32 * 64;   // class operators in lane order

// Input column of step T for this lane, from the lane's packed column table
// (four 7-bit column numbers per word, filled once per kernel): branch-free,
// so the whole step chain stays one basic block and the loads stay where the
// pipeline puts them.
template <int T>
__device__ __forceinline__ uint32_t step_col(const uint32_t* packed) {
    return (packed[T >> 2] >> (8 * (T & 3))) & 0xFFu;
}

template <int T>
__device__ __forceinline__ void load_step(const double* __restrict__ src, size_t plane, const Cell16& c,
                                          const uint32_t* packed, double* v) {
    const double* __restrict__ b = src + (size_t)step_col<T>(packed) * plane;
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = b[c.corner[s]];
}

// Software pipeline depth: the corner values of step T + kAhead are requested
// while step T runs its butterfly and matrix work.
constexpr int kAhead = 2;
constexpr int kRing = kAhead + 1;

// One K-step. ring[T % kRing] holds this step's corner values (loaded kAhead
// steps earlier). The scheduling barrier keeps the compiler from hoisting
// every step's loads to the top (which would spill).
template <int T>
struct Steps {
    __device__ __forceinline__ static void run(const double* __restrict__ src, size_t plane, const Cell16& c,
                                               const uint32_t* packed, int lane, const double* sK, d4* acc,
                                               double (*ring)[8]) {
        constexpr MfmaSchedule S{};
        constexpr int dp = S.dpar[T];
        if constexpr (T + kAhead < 32) load_step<T + kAhead>(src, plane, c, packed, ring[(T + kAhead) % kRing]);
        double Tv[8];
        butterfly8(ring[T % kRing], Tv);
        double a[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) a[p] = sK[(p * 32 + T) * 64 + lane];
        // class p takes the butterfly output t = p xor (d mod 2): a sum along
        // x when p_x and d_x agree, a difference otherwise
#pragma unroll
        for (int p = 0; p < 8; ++p) acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], Tv[p ^ dp], acc[p], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (T + 1 < 32) Steps<T + 1>::run(src, plane, c, packed, lane, sK, acc, ring);
    }
};

// The same K-step in 4x4 tiles on v_mfma_f64_4x4x4f64 (4 blocks), which runs
// at 1.55x the FP64 rate of the 16x16x4 instruction on gfx950. Block b (lane
// bits 2-3) multiplies A[i][k] (lane 16k + 4b + i) by B[k][j] (lane 16k + 4b +
// j) into D[i][j] (lane 16i + 4b + j). With block b taking cells 4b .. 4b+3,
// B is exactly the 16x16 kernel's operand (lane 16q + cell: the butterfly
// output of column q for that cell), and D row i lands in quarter i at the
// cell's lane. Per class, 4 instructions cover the 16 rows as row tiles ri
// whose row i is class row 4i + ri, so quarter q accumulates class rows
// 4q + ri, ri = 0..3: the 16x16 kernel's accumulator layout.
//
// A 16-cell batch alone would read 4x the operator values from LDS per cell
// that the 16x16 kernel does (each tile's 16 values are the same in all 4
// blocks). So each wave runs two batches at once, the cells (x, y, z) and
// (x, y, z + 1): every operator tile read feeds both, and the lower corner
// plane of the second cell is the upper corner plane of the first, so a step
// loads 12 corner values instead of 16 (ra: the first cell's 8, rb: the
// second cell's upper 4). Per step the wave issues 64 instructions, one class
// after the other, with the next class's tiles already in flight.
constexpr int kAhead4 = 2;
constexpr int kRing4 = kAhead4 + 1;

// Row tiles that are zero for every operator: entry (row, column) of class p
// vanishes whenever on some axis x the class parity p_x is 0, the output's
// o_x is 1 and the input's d_x is 0 (the even part of the 1D interpolant has
// no second-order term from the values, and the evolution lowers orders in
// steps of two). Tile ri of class p at step T holds rows 4 i + ri (i = field
// and o3, ri = o2 and o1) of the step's 4 columns; z[T][p][ri] when all 16
// entries vanish (124 of 1,024 tiles with this schedule). The kernel skips
// them; mfma4_arrange_operators checks that the operator is zero there.
struct ZeroTiles4 {
    bool z[32][8][4];
    static constexpr bool zero_entry(int p, int row, int col) {
        const int d = col & 63;
        const int dx[3] = {d & 3, (d >> 2) & 3, d >> 4};
        for (int x = 0; x < 3; ++x)
            if (((p >> x) & 1) == 0 && ((row >> x) & 1) == 1 && dx[x] == 0) return true;
        return false;
    }
    constexpr ZeroTiles4() : z() {
        constexpr MfmaSchedule S{};
        for (int t = 0; t < 32; ++t)
            for (int p = 0; p < 8; ++p)
                for (int ri = 0; ri < 4; ++ri) {
                    bool all = true;
                    for (int i = 0; i < 4; ++i)
                        for (int k = 0; k < 4; ++k) all = all && zero_entry(p, 4 * i + ri, S.col[t][k]);
                    z[t][p][ri] = all;
                }
    }
};

// Corner values s = 4 .. 7 (the upper z plane) of a cell, input column of step T.
template <int T>
__device__ __forceinline__ void load_upper(const double* __restrict__ src, size_t plane, const Cell16& c,
                                           const uint32_t* packed, double* v) {
    const double* __restrict__ b = src + (size_t)step_col<T>(packed) * plane;
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = b[c.corner[4 + s]];
}

// The first kAhead4 steps' corner values of a batch pair.
template <int T>
struct ProloguePair {
    __device__ __forceinline__ static void run(const double* __restrict__ src, size_t plane, const Cell16& ca,
                                               const Cell16& cb, const uint32_t* packed, double (*ra)[8],
                                               double (*rb)[4]) {
        load_step<T>(src, plane, ca, packed, ra[T]);
        load_upper<T>(src, plane, cb, packed, rb[T]);
        if constexpr (T + 1 < kAhead4) ProloguePair<T + 1>::run(src, plane, ca, cb, packed, ra, rb);
    }
};

template <int T>
struct Steps4Pair {
    __device__ __forceinline__ static void run(const double* __restrict__ src, size_t plane, const Cell16& ca,
                                               const Cell16& cb, const uint32_t* packed, int lane, const double* sK,
                                               double (*acca)[4], double (*accb)[4], double (*ra)[8],
                                               double (*rb)[4]) {
        constexpr MfmaSchedule S{};
        constexpr ZeroTiles4 Z{};
        constexpr int dp = S.dpar[T];
        if constexpr (T + kAhead4 < 32) {
            load_step<T + kAhead4>(src, plane, ca, packed, ra[(T + kAhead4) % kRing4]);
            load_upper<T + kAhead4>(src, plane, cb, packed, rb[(T + kAhead4) % kRing4]);
        }
        double Ta[8], Tb[8], vb[8];
#pragma unroll
        for (int s = 0; s < 4; ++s) vb[s] = ra[T % kRing4][4 + s], vb[4 + s] = rb[T % kRing4][s];
        butterfly8(ra[T % kRing4], Ta);
        butterfly8(vb, Tb);
        // this lane's A[i][k] (k = lane / 16, i = lane % 4) for row tiles
        // 2 rp and 2 rp + 1 of class p: one 16-byte read; a step's 32 tiles
        // are 4 KB, so every read of the step has an immediate offset
        const int at = ((lane >> 4) << 2) | (lane & 3);
        const double2* __restrict__ sT = reinterpret_cast<const double2*>(sK) + (size_t)T * 8 * 2 * 16 + at;
        double2 a[2][2];  // [class parity of the pipeline][rp]
#pragma unroll
        for (int rp = 0; rp < 2; ++rp) a[0][rp] = sT[(0 * 2 + rp) * 16];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            if (p + 1 < 8) {
#pragma unroll
                for (int rp = 0; rp < 2; ++rp) a[(p + 1) & 1][rp] = sT[((p + 1) * 2 + rp) * 16];
            }
#pragma unroll
            for (int ri = 0; ri < 4; ++ri) {
                if (Z.z[T][p][ri]) continue;  // resolved at compile time
                const double2 av = a[p & 1][ri >> 1];
                const double x = (ri & 1) ? av.y : av.x;
                acca[p][ri] = __builtin_amdgcn_mfma_f64_4x4x4f64(x, Ta[p ^ dp], acca[p][ri], 0, 0, 0);
                accb[p][ri] = __builtin_amdgcn_mfma_f64_4x4x4f64(x, Tb[p ^ dp], accb[p][ri], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (T + 1 < 32)
            Steps4Pair<T + 1>::run(src, plane, ca, cb, packed, lane, sK, acca, accb, ra, rb);
    }
};

// The first kAhead steps' corner values, before the step chain starts.
template <int T>
struct Prologue {
    __device__ __forceinline__ static void run(const double* __restrict__ src, size_t plane, const Cell16& c,
                                               const uint32_t* packed, double (*ring)[8]) {
        load_step<T>(src, plane, c, packed, ring[T]);
        if constexpr (T + 1 < kAhead) Prologue<T + 1>::run(src, plane, c, packed, ring);
    }
};

// Column tables: kColTable[q][w] packs the input columns of steps 4w..4w+3
// for lane quarter q.
struct ColTable {
    uint32_t w[4][8];
    constexpr ColTable() : w() {
        constexpr MfmaSchedule S{};
        for (int q = 0; q < 4; ++q)
            for (int t = 0; t < 32; ++t) w[q][t >> 2] |= (uint32_t)S.col[t][q] << (8 * (t & 3));
    }
};
__constant__ ColTable kColTable = ColTable();

// Stores the 32 new values a lane holds for one cell: logical output row 4q + r
// of class p (register r of quarter q) is field q/2, derivative orders
// j = p + 2 (o1, o2, o3) with o3 = q % 2, o2 = r / 2, o1 = r % 2.
template <class Acc>
__device__ __forceinline__ void store_cell(double* __restrict__ dst, size_t plane, uint32_t out, int q,
                                           const Acc& acc) {
    const int fo = q >> 1, o3 = q & 1;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int p1 = p & 1, p2 = (p >> 1) & 1, p3 = p >> 2;
        const int j3 = p3 + 2 * o3;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j1 = p1 + 2 * (r & 1), j2 = p2 + 2 * (r >> 1);
            dst[(size_t)(fo * 64 + (j3 * 4 + j2) * 4 + j1) * plane + out] = acc[p][r];
        }
    }
}

// One batch: the 16 neighbouring cells of row (y, z) whose new nodes are
// x0 .. x0+15 (lower corners x0 - off .., periodic); lanes past the end of
// the row compute a copy of the last cell and store nothing.
// SLAB: z is a buffer plane of a slab (fused::slab_cell_nodes) instead of a
// plane of the periodic cube.
template <bool SLAB = false>
__device__ __forceinline__ void run_batch(const double* __restrict__ src, double* __restrict__ dst, size_t plane,
                                          uint32_t n, uint32_t off, uint32_t x0, uint32_t y, uint32_t z, int lane,
                                          int cl, int q, uint32_t* packed, const double* sK) {
    const uint32_t x = x0 + cl;
    const bool valid = x < n;
    // lane cl produces new node x0 + cl of row (y + off, z + off): the cell's
    // lower corner is x - off, so that the stores of a batch fill whole
    // 128-byte lines also in the dual -> primal half step
    const uint32_t cx = valid ? (x + n - off) % n : n - 1;
    Cell16 c;
    if constexpr (SLAB)
        c = fused::slab_cell_nodes(cx, y, z, n, off);
    else
        c = cell_nodes((z * n + y) * n + cx, n, off);
    // Opaque per batch: without this the 32 per-lane column base addresses
    // are hoisted out of the batch loop and pin 64 registers.
#pragma unroll
    for (int w = 0; w < 8; ++w) asm volatile("" : "+v"(packed[w]));
    d4 acc[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) acc[p] = d4{0.0, 0.0, 0.0, 0.0};
    double ring[kRing][8];
    Prologue<0>::run(src, plane, c, packed, ring);
    Steps<0>::run(src, plane, c, packed, lane, sK, acc, ring);
    if (valid) store_cell(dst, plane, c.out, q, acc);
}

// Two batches on the 4x4-tile instruction: the 16 cells of row (y, z) whose
// new nodes are x0 .. x0+15, as in run_batch, and the 16 cells above them in
// row (y, z + 1) (periodic in the cube), stored only if upper is set.
// SLAB: z is a buffer plane of a slab; without upper, the second batch
// repeats the first (plane z + 1 may lie past the slab's buffer) and is not
// stored.
template <bool SLAB = false>
__device__ __forceinline__ void run_batch_pair(const double* __restrict__ src, double* __restrict__ dst,
                                               size_t plane, uint32_t n, uint32_t off, uint32_t x0, uint32_t y,
                                               uint32_t z, bool upper, int lane, int cl, int q, uint32_t* packed,
                                               const double* sK) {
    const uint32_t x = x0 + cl;
    const bool valid = x < n;
    const uint32_t cx = valid ? (x + n - off) % n : n - 1;
    Cell16 ca, cb;
    if constexpr (SLAB) {
        ca = fused::slab_cell_nodes(cx, y, z, n, off);
        cb = fused::slab_cell_nodes(cx, y, upper ? z + 1 : z, n, off);
    } else {
        const uint32_t zb = (z + 1 == n) ? 0 : z + 1;
        ca = cell_nodes((z * n + y) * n + cx, n, off);
        cb = cell_nodes((zb * n + y) * n + cx, n, off);
    }
#pragma unroll
    for (int w = 0; w < 8; ++w) asm volatile("" : "+v"(packed[w]));
    double acca[8][4], accb[8][4];
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) acca[p][r] = accb[p][r] = 0.0;
    double ra[kRing4][8], rb[kRing4][4];
    ProloguePair<0>::run(src, plane, ca, cb, packed, ra, rb);
    Steps4Pair<0>::run(src, plane, ca, cb, packed, lane, sK, acca, accb, ra, rb);
    if (valid) store_cell(dst, plane, ca.out, q, acca);
    if (valid && upper) store_cell(dst, plane, cb.out, q, accb);
}

// Persistent kernel over the XCD-blocked row sweep (fused::sweep_rows).
__global__ __launch_bounds__(kWaves * 64) void fused_mfma_kernel(const double* __restrict__ src,
                                                                 double* __restrict__ dst,
                                                                 const double* __restrict__ Kperm, uint32_t n,
                                                                 size_t pitch, uint32_t off) {
    __shared__ double sK[kOpDoubles];
    for (int i = threadIdx.x; i < kOpDoubles; i += blockDim.x) sK[i] = Kperm[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane & 15, q = lane >> 4;
    uint32_t packed[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) packed[k] = kColTable.w[q][k];
    fused::sweep_rows(n, wave, kWaves, [&](uint32_t x0, uint32_t y, uint32_t z) {
        run_batch(src, dst, pitch, n, off, x0, y, z, lane, cl, q, packed, sK);
    });
}

// The periodic cube on the 4x4-tile instruction, two z-adjacent batches per
// wave (Steps4Pair); operators from mfma4_arrange_operators. The two
// accumulator sets (128 registers) and the corner ring take more than half a
// SIMD's registers, so the workgroup has one wave per SIMD.
constexpr int kWaves4 = 4;

__global__ __launch_bounds__(kWaves4 * 64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void fused_mfma4_kernel(const double* __restrict__ src, double* __restrict__ dst, const double* __restrict__ K4,
                        uint32_t n, size_t pitch, uint32_t off, uint32_t* __restrict__ queue) {
    __shared__ double sK[kOpDoubles];
    for (int i = threadIdx.x; i < kOpDoubles; i += blockDim.x) sK[i] = K4[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane & 15, q = lane >> 4;
    uint32_t packed[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) packed[k] = kColTable.w[q][k];
    fused::sweep_row_pairs(n, wave, kWaves4, queue, [&](uint32_t x0, uint32_t y, uint32_t z, bool upper) {
        run_batch_pair(src, dst, pitch, n, off, x0, y, z, upper, lane, cl, q, packed, sK);
    });
}

// One z-slab of a periodic grid sharded over GPUs: the cells on buffer planes
// k0 .. k1-1 (fused::slab_cell_nodes), the same per-cell arithmetic.
__global__ __launch_bounds__(kWaves * 64) void fused_mfma_slab_kernel(const double* __restrict__ src,
                                                                      double* __restrict__ dst,
                                                                      const double* __restrict__ Kperm, uint32_t n,
                                                                      uint32_t k0, uint32_t k1, size_t pitch,
                                                                      uint32_t off) {
    __shared__ double sK[kOpDoubles];
    for (int i = threadIdx.x; i < kOpDoubles; i += blockDim.x) sK[i] = Kperm[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane & 15, q = lane >> 4;
    uint32_t packed[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) packed[k] = kColTable.w[q][k];
    fused::sweep_rows_slab(n, k0, k1, wave, kWaves, [&](uint32_t x0, uint32_t y, uint32_t z) {
        run_batch<true>(src, dst, pitch, n, off, x0, y, z, lane, cl, q, packed, sK);
    });
}

// The cell planes k0 .. k1-1 of a slab on the 4x4-tile instruction, two
// z-adjacent batches per wave (fused::sweep_row_pairs_slab).
__global__ __launch_bounds__(kWaves4 * 64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void fused_mfma4_slab_kernel(const double* __restrict__ src, double* __restrict__ dst, const double* __restrict__ K4,
                             uint32_t n, uint32_t k0, uint32_t k1, size_t pitch, uint32_t off,
                             uint32_t* __restrict__ queue) {
    __shared__ double sK[kOpDoubles];
    for (int i = threadIdx.x; i < kOpDoubles; i += blockDim.x) sK[i] = K4[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane & 15, q = lane >> 4;
    uint32_t packed[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) packed[k] = kColTable.w[q][k];
    fused::sweep_row_pairs_slab(n, k0, k1, wave, kWaves4, queue,
                                [&](uint32_t x0, uint32_t y, uint32_t z, bool upper) {
                                    run_batch_pair<true>(src, dst, pitch, n, off, x0, y, z, upper, lane, cl, q,
                                                         packed, sK);
                                });
}

// Batched: the batch pairs of every shot of the group (batch_common.h) on the
// 4x4-tile instruction. A shot of n cells per side has n ceil(n/2) ceil(n/16)
// items: item (bx, y, zp), bx fastest, is the pair of rows (y, 2 zp) and
// (y, 2 zp + 1) at x-batch bx (the second row absent when n is odd and
// 2 zp + 1 = n).
__global__ __launch_bounds__(kWaves4 * 64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void fused_mfma_batch_kernel(const batch::ShotGrid* __restrict__ shots, const uint32_t* __restrict__ ids,
                             const uint32_t* __restrict__ prefix, uint32_t ng, uint32_t from,
                             const double* __restrict__ K4, uint32_t chunk, uint32_t interleaved) {
    __shared__ double sK[kOpDoubles];
    for (int i = threadIdx.x; i < kOpDoubles; i += blockDim.x) sK[i] = K4[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane & 15, q = lane >> 4;
    uint32_t packed[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) packed[k] = kColTable.w[q][k];
    batch::sweep_items(prefix[ng], wave, kWaves4, chunk, interleaved, [&](uint32_t it) {
        const uint32_t g = batch::find_entry(prefix, ng, it);
        const batch::ShotGrid& S = shots[ids[g]];
        const uint32_t n = S.n, nbx = (n + 15) >> 4, local = it - prefix[g];
        const uint32_t bx = local % nbx, rest = local / nbx, y = rest % n, z = 2 * (rest / n);
        run_batch_pair(S.grid[from], S.grid[1 - from], S.pitch, n, from, bx * 16, y, z, z + 1 < n, lane, cl, q,
                       packed, sK);
    });
}

}  // namespace

size_t mfma_operator_doubles() { return (size_t)kOpDoubles; }

hipError_t launch_fused_mfma_batch(const batch::ShotGrid* shots, const uint32_t* ids, const uint32_t* prefix,
                                   uint32_t ng, int from, const double* K4, int grid, uint32_t chunk,
                                   uint32_t interleaved, hipStream_t st) {
    if (grid < 8 || grid % 8 != 0 || chunk < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fused_mfma_batch_kernel, dim3(grid), dim3(kWaves4 * 64), 0, st, shots, ids, prefix, ng,
                       (uint32_t)from, K4, chunk, interleaved);
    return hipGetLastError();
}

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

hipError_t launch_fused_mfma_slab(const double* src, double* dst, const double* Kperm, int n, int k0, int k1,
                                  size_t pitch, int off, int grid, hipStream_t st) {
    if (grid < 8 || grid % 8 != 0 || k0 < 0 || k1 < k0) return hipErrorInvalidValue;
    if (k1 == k0) return hipSuccess;
    hipLaunchKernelGGL(fused_mfma_slab_kernel, dim3(grid), dim3(kWaves * 64), 0, st, src, dst, Kperm, (uint32_t)n,
                       (uint32_t)k0, (uint32_t)k1, pitch, (uint32_t)off);
    return hipGetLastError();
}

bool mfma4_arrange_operators(const double* K, double* K4) {
    // K: [8][16][128] canonical class operators. Tile ri = 2 rp + h of class p
    // at step t: A[i][k] = K[p][4 i + ri][col(t, k)], stored at
    // ((((t 8 + p) 2 + rp) 16 + 4 k + i) 2 + h: a lane reads its two tiles of
    // a row-tile pair as one 16-byte value. Returns false if a tile that the
    // kernels skip (ZeroTiles4) holds a nonzero entry.
    constexpr MfmaSchedule S{};
    constexpr ZeroTiles4 Z{};
    bool ok = true;
    for (int t = 0; t < 32; ++t)
        for (int p = 0; p < 8; ++p)
            for (int ri = 0; ri < 4; ++ri)
                for (int k = 0; k < 4; ++k)
                    for (int i = 0; i < 4; ++i) {
                        const double v = K[((size_t)p * 16 + 4 * i + ri) * 128 + S.col[t][k]];
                        K4[((((size_t)t * 8 + p) * 2 + (ri >> 1)) * 16 + 4 * k + i) * 2 + (ri & 1)] = v;
                        if (Z.z[t][p][ri] && v != 0.0) ok = false;
                    }
    return ok;
}

hipError_t launch_fused_mfma4_slab(const double* src, double* dst, const double* K4, int n, int k0, int k1,
                                   size_t pitch, int off, int grid, uint32_t* queue, hipStream_t st) {
    if (grid < 8 || grid % 8 != 0 || k0 < 0 || k1 < k0 || queue == nullptr) return hipErrorInvalidValue;
    if (k1 == k0) return hipSuccess;
    hipLaunchKernelGGL(fused_mfma4_slab_kernel, dim3(grid), dim3(kWaves4 * 64), 0, st, src, dst, K4, (uint32_t)n,
                       (uint32_t)k0, (uint32_t)k1, pitch, (uint32_t)off, queue);
    return hipGetLastError();
}

hipError_t launch_fused_mfma4(const double* src, double* dst, const double* K4, int n, size_t pitch, int off, int grid,
                              uint32_t* queue, hipStream_t st) {
    if (grid < 8 || grid % 8 != 0 || queue == nullptr) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fused_mfma4_kernel, dim3(grid), dim3(kWaves4 * 64), 0, st, src, dst, K4, (uint32_t)n, pitch,
                       (uint32_t)off, queue);
    return hipGetLastError();
}

hipError_t launch_fused_mfma(const double* src, double* dst, const double* Kperm, int n, size_t pitch, int off,
                             int grid, hipStream_t st) {
    if (grid < 8 || grid % 8 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fused_mfma_kernel, dim3(grid), dim3(kWaves * 64), 0, st, src, dst, Kperm, (uint32_t)n, pitch,
                       (uint32_t)off);
    return hipGetLastError();
}

}  // namespace hermite
