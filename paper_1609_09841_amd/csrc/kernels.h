// Launch wrappers of the Hermite half-step kernels (gfx950). Internal to the
// library; the public interface is include/hermite.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hermite {

// Grids: a two-field grid holds 2 M^3 columns (field-major, then the
// derivative multi-index d), column c starting at c * pitch doubles; within a
// column node (i,j,k) sits at (k n + j) n + i. pitch >= n^3 is padded so that
// the columns of one node do not all fall into the same cache set.
//
// Fused half step (interpolation + evolution + truncation per cell) with the
// per-parity-class operators K of constants.h ([8][rows_max][2 M^3], FP64),
// laid out for the kernel in use: src/dst are two-field grids; the cell with
// lower corner (i,j,k) of src writes node (i+off, j+off, k+off) mod n of dst
// (off = 0 primal->dual, off = 1 dual->primal).
//
// m = 3 on the FP64 matrix cores. Kperm: the
// class operators permuted by mfma_permute_operators (mfma_operator_doubles()
// doubles). grid: workgroups, a multiple of 8 (one per CU is enough).
hipError_t launch_fused_mfma(const double* src, double* dst, const double* Kperm, int n, size_t pitch, int off,
                             int grid, hipStream_t st);
void mfma_permute_operators(const double* K, double* Kperm);
size_t mfma_operator_doubles();
// The same half step in 4x4 tiles (v_mfma_f64_4x4x4f64), two z-adjacent
// batches per wave; K4 from mfma4_arrange_operators (mfma_operator_doubles()
// doubles). queue: kMfma4QueueWords words of device memory, zero before the
// first launch and left zero by every completed launch; launches that may
// run at the same time need queues of their own.
constexpr size_t kMfma4QueueWords = 8 * 64;
hipError_t launch_fused_mfma4(const double* src, double* dst, const double* K4, int n, size_t pitch, int off, int grid,
                              uint32_t* queue, hipStream_t st);
// false if a tile the 4x4 kernels skip as structurally zero is not zero in K
bool mfma4_arrange_operators(const double* K, double* K4);
// Cell planes k0 .. k1-1 (no launch if empty) of a z-slab on the 4x4-tile
// instruction, two z-adjacent batches per wave; K4 and queue as for
// launch_fused_mfma4.
hipError_t launch_fused_mfma4_slab(const double* src, double* dst, const double* K4, int n, int k0, int k1,
                                   size_t pitch, int off, int grid, uint32_t* queue, hipStream_t st);
// Cell planes k0 .. k1-1 (no launch if empty) of one z-slab of nz cell
// planes of a periodic n x n x (shards * nz) grid: src and dst hold nz + 1
// node planes of n^2 nodes per column (the slab layout of
// fused::slab_cell_nodes); off as launch_fused_mfma.
hipError_t launch_fused_mfma_slab(const double* src, double* dst, const double* Kperm, int n, int k0, int k1,
                                  size_t pitch, int off, int grid, hipStream_t st);

// Same fused FP64 half step for m = 3 on the vector ALUs: one lane per cell
// and output field, operator entries as scalar operands. Kv:
// valu4_build_operators output (valu4_operator_doubles() doubles).
hipError_t launch_fused_valu4(const double* src, double* dst, const double* Kv, int n, size_t pitch, int off,
                              hipStream_t st);
size_t valu4_operator_doubles();
void valu4_build_operators(const double* K, double* Kv);

// Fused FP64 half step for m = 1, 2 on the vector ALUs: one lane per cell,
// all 2 (m+1)^3 new values. Kv: valu_small_build_operators output
// (valu_small_operator_doubles(m) doubles). The kernels skip the operator
// entries that vanish for every time step (at m = 2, 868 of 2,916); the
// builder returns false if one of them is not zero in K.
hipError_t launch_fused_valu_small(int m, const double* src, double* dst, const double* Kv, int n, size_t pitch,
                                   int off, hipStream_t st);
size_t valu_small_operator_doubles(int m);
bool valu_small_build_operators(int m, const double* K, double* Kv);

// Mixed-precision fused half step (m = 3): precision 1 = FP32 matrix cores,
// 2 = split BF16 (three products), both with FP32 accumulation; FP64 state,
// FP64 corner-mean part and FP64 update. Aops: mixed_build_operators output
// (mixed_operator_bytes(precision) bytes). grid as for launch_fused_mfma.
// FP32 runs two z-adjacent batches per wave and needs a queue as
// launch_fused_mfma4 does (kMfma4QueueWords words); BF16x3 ignores it.
hipError_t launch_fused_mixed(int precision, const double* src, double* dst, const void* Aops, int n, size_t pitch,
                              int off, int grid, uint32_t* queue, hipStream_t st);
size_t mixed_operator_bytes(int precision);
void mixed_build_operators(int precision, const double* K, void* out);

// Point source (one entry per forced grid, device-resident). The source
// kernel adds the particular solution of the forced cell system to the new
// nodes of the cells of box[from] (stream-ordered after the half step that
// wrote grid[1 - from]).
struct SourceDesc {
    double* grid[2];     // primal, dual
    uint64_t pitch;      // doubles between columns
    uint32_t n, m, q;    // cells per side, order, Taylor stages
    uint32_t box[2][6];  // per half step (from = 0, 1): first cell x, y, z
                         // (periodic) and counts nx, ny, nz of the source-grid
                         // cells whose centres may lie within 6 sigma
    double x[3];         // source point in [0, 1)^3
    double sigma, amp, f0, t0;
    double h, tau, dt, lam, pre;  // pre = tau h / c
    int64_t steps;       // full steps taken: the device-side clock
    const double* series;  // NULL, or the amplitude of half step 2 steps + from
};
// Blocks the source kernel needs for entry s in half step `from`.
uint32_t source_blocks(const SourceDesc& s, int from);
// srcs: ns device entries, all of order m; prefix: ns + 1 device block
// offsets for this half step (prefix[ns] = blocks). host_steps >= 0 replaces
// every entry's clock. scal: device scratch of 20 ns doubles (the half
// step's scalars, written and read within the call's two launches).
hipError_t launch_source(const SourceDesc* srcs, const uint32_t* prefix, uint32_t ns, uint32_t blocks, int m, int from,
                         long long host_steps, double* scal, hipStream_t st);
// Gradient of an amplitude series entry: *grad = <lam, P> over the
// destination grid grid[1 - from] (which holds the adjoint lam) for one
// source entry, P its source term of the half step with unit amplitude
// series (times the entry's amp). partial: device scratch of `blocks`
// doubles; the sum runs in a fixed order.
hipError_t launch_source_dot(const SourceDesc* src, const uint32_t* prefix, uint32_t blocks, int m, int from,
                             long long host_steps, double* scal, double* partial, double* grad, hipStream_t st);

// Transposed fused half step (FP64, m = 1, 2): lam_src (adjoint of the grid the half
// step reads) from lam_dst (adjoint of the grid it writes); K: canonical
// class operators ([8][rows_max][2 M^3], fused_class_operators), device.
hipError_t launch_adjoint(int m, const double* lam_dst, double* lam_src, const double* K, int n, size_t pitch, int off,
                          hipStream_t st);
// m = 3 on the matrix cores: KT = adjoint_mfma_build_operator(K)
// (adjoint_mfma_operator_doubles() doubles); grid as for launch_fused_mfma,
// queue as for launch_fused_mfma4 (the context's own). One launch, no
// scratch.
hipError_t launch_adjoint_mfma(const double* lam_dst, double* lam_src, const double* KT, int n, size_t pitch, int off,
                               int grid, uint32_t* queue, hipStream_t st);
size_t adjoint_mfma_operator_doubles();
void adjoint_mfma_build_operator(const double* K, double* KT);
// Receivers: traces[r] = grid[nodes[r]] (u, d = 0 of the primal grid);
// inject: lam[nodes[r]] += res[r] in receiver order.
hipError_t launch_record(const double* grid, const uint32_t* nodes, uint32_t nr, double* traces, hipStream_t st);
hipError_t launch_inject(double* lam, const uint32_t* nodes, uint32_t nr, const double* res, hipStream_t st);
// steps += 1 for every entry (end of a full step of a batch).
hipError_t launch_advance_clock(SourceDesc* srcs, uint32_t ns, hipStream_t st);

// Batched fused half steps (batch_common.h): one launch over the shots of one
// order. ids/prefix: group entries and their first work item (ng + 1
// entries, device); from: 0 primal -> dual, 1 dual -> primal. Operators as
// for the single-grid launches (they depend on m and lam only).
//   m = 1, 2: work item = `block` cells (64, 128 or 256); blocks = prefix[ng].
//   m = 3 FP64 and mixed: 16-cell batches; persistent grid (multiple of 8);
//   chunk/interleaved select the item order (batch::sweep_items).
namespace batch {
struct ShotGrid;
}
hipError_t launch_fused_valu_small_batch(int m, int block, const batch::ShotGrid* shots, const uint32_t* ids,
                                         const uint32_t* prefix, uint32_t ng, uint32_t blocks, int from,
                                         const double* Kv, hipStream_t st);
// FP64 m = 3 batches run two z-adjacent batches per wave on the 4x4-tile
// instruction: K4 from mfma4_arrange_operators, and prefix counts
// n ceil(n/2) ceil(n/16) items per shot.
hipError_t launch_fused_mfma_batch(const batch::ShotGrid* shots, const uint32_t* ids, const uint32_t* prefix,
                                   uint32_t ng, int from, const double* K4, int grid, uint32_t chunk,
                                   uint32_t interleaved, hipStream_t st);
// Both precisions work on z-adjacent row pairs (items counted as for
// launch_fused_mfma_batch).
hipError_t launch_fused_mixed_batch(int precision, const batch::ShotGrid* shots, const uint32_t* ids,
                                    const uint32_t* prefix, uint32_t ng, int from, const void* Aops, int grid,
                                    uint32_t chunk, uint32_t interleaved, hipStream_t st);

// Fused advection half step (m = 1..3, FP64): one field of M^3 columns per
// grid; K1: advection_axis_operator (M x 2M doubles, host memory, passed by
// value to the kernel).
hipError_t launch_advect(int m, const double* src, double* dst, const double* K1, int n, size_t pitch, int off,
                         hipStream_t st);

// Interpolation half of the two-kernel variant: writes the monomial
// coefficients R[nf][P^3][n^3] (P = 2m+2) of every cell of src (nf fields:
// 2 for the wave system, 1 for advection). Hp: parity blocks of H, [2][M][M].
hipError_t launch_interp(int m, const double* src, double* R, const double* Hp, int n, size_t pitch, int nf,
                         hipStream_t st);

// Advection evolution half of the two-kernel variant: reads R[P^3][n^3],
// translates each cell polynomial by lam (1,1,1) (the exact Taylor series,
// q >= 3(2m+1)) and writes the coefficients with every index <= m to node
// cell + off of dst. E1: M x P row-major, E1[j][k] = C(k, j) lam^(k-j) (host
// memory, passed by value).
hipError_t launch_advect_evolve(int m, const double* R, double* dst, const double* E1, int n, size_t pitch, int off,
                                hipStream_t st);

// Evolution half: reads R, runs the Taylor stage loop (evolution 0, q stages)
// or 4-stage Runge-Kutta (evolution 1, S substeps) with lam = c*tau/h, and
// writes the coefficients with every index <= m to node cell+off of dst.
hipError_t launch_evolve(int m, const double* R, double* dst, int n, size_t pitch, int off, int evolution,
                         int q, int S, double lam, hipStream_t st);

// *flag |= 1 if any entry g[r * pitch + c], r < rows, c < cols, is NaN or Inf.
hipError_t launch_nonfinite(const double* g, size_t pitch, size_t cols, int rows, int* flag, hipStream_t st);

// dst[r * dpitch + c] = s * src[r * spitch + c], r < rows, c < cols (dst may equal src).
hipError_t launch_scale(double* dst, size_t dpitch, const double* src, size_t spitch, double s, size_t cols,
                        int rows, hipStream_t st);

}  // namespace hermite
