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

// Same fused FP64 half step for m = 3 on the vector ALUs: one lane per cell
// and output field, operator entries as scalar operands. Kv:
// valu4_build_operators output (valu4_operator_doubles() doubles).
hipError_t launch_fused_valu4(const double* src, double* dst, const double* Kv, int n, size_t pitch, int off,
                              hipStream_t st);
size_t valu4_operator_doubles();
void valu4_build_operators(const double* K, double* Kv);

// Fused FP64 half step for m = 1, 2 on the vector ALUs: one lane per cell,
// all 2 (m+1)^3 new values. Kv: valu_small_build_operators output
// (valu_small_operator_doubles(m) doubles).
hipError_t launch_fused_valu_small(int m, const double* src, double* dst, const double* Kv, int n, size_t pitch,
                                   int off, hipStream_t st);
size_t valu_small_operator_doubles(int m);
void valu_small_build_operators(int m, const double* K, double* Kv);

// Mixed-precision fused half step (m = 3): precision 1 = FP32 matrix cores,
// 2 = split BF16 (three products), both with FP32 accumulation; FP64 state,
// FP64 corner-mean part and FP64 update. Aops: mixed_build_operators output
// (mixed_operator_bytes(precision) bytes). grid as for launch_fused_mfma.
hipError_t launch_fused_mixed(int precision, const double* src, double* dst, const void* Aops, int n, size_t pitch,
                              int off, int grid, hipStream_t st);
size_t mixed_operator_bytes(int precision);
void mixed_build_operators(int precision, const double* K, void* out);

// Point source: per-half-step scalars (A_i i!, B_i i!, i <= 3m) and the box
// of source-grid cells (lower corners x0.., periodic, nx x ny x nz) whose
// centres lie within 6 sigma of the source along every axis.
struct SourceScalars {
    double Ai[10];
    double Bi[10];
};
struct SourceBox {
    uint32_t x0, y0, z0, nx, ny, nz;
};
// Adds the particular solution of the forced cell system to the new nodes of
// the box's cells (stream-ordered after the half step that wrote dst).
hipError_t launch_source(double* dst, int n, size_t pitch, int m, const SourceBox& box, const double* centre,
                         double h, double sigma, double amp, int to_dual, const SourceScalars& sc,
                         hipStream_t st);

// Interpolation half of the two-kernel variant: writes the monomial
// coefficients R[2][P^3][n^3] (P = 2m+2) of every cell of src. Hp: parity
// blocks of H, [2][M][M].
hipError_t launch_interp(int m, const double* src, double* R, const double* Hp, int n, size_t pitch,
                         hipStream_t st);

// Evolution half: reads R, runs the Taylor stage loop (evolution 0, q stages)
// or 4-stage Runge-Kutta (evolution 1, S substeps) with lam = c*tau/h, and
// writes the coefficients with every index <= m to node cell+off of dst.
hipError_t launch_evolve(int m, const double* R, double* dst, int n, size_t pitch, int off, int evolution,
                         int q, int S, double lam, hipStream_t st);

// dst[r * dpitch + c] = s * src[r * spitch + c], r < rows, c < cols (dst may equal src).
hipError_t launch_scale(double* dst, size_t dpitch, const double* src, size_t spitch, double s, size_t cols,
                        int rows, hipStream_t st);

}  // namespace hermite
