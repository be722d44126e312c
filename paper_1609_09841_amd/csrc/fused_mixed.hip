// Mixed-precision fused Hermite half step for m = 3 (FP32 or split-BF16
// contractions on the matrix cores, FP64 state and FP64 update).
//
// The half step of a cell is, per parity class p, y = K_p x with x the 128
// class inputs (the 2x2x2 butterfly of the corner data, formed in FP64) and
// y the 16 new values of that class. Most of each new value is the mean of
// its own scaled derivative over the 8 corners: for the new value j of field
// f, P0 = (1/8) x[(f, d = j)], the all-sums butterfly output of column
// (f, j). So the kernel keeps P0 in FP64 and runs only the remainder
// (K_p - P0) x in low precision:
//   y = P0 (FP64) + [(K_p - P0) x] (FP32 accumulation) -> FP64 store.
// Which lane computes which P0: lane quarter q reads exactly the 32 columns
// whose new values its accumulators hold (fused::OwnSchedule), so P0 is a
// register of the lane that holds the output.
//
// FP32: v_mfma_f32_16x16x4f32, one K-step per input column chunk, the same
// shape as the FP64 kernel (A = operator rows x 4 columns, B = 4 columns x 16
// cells; register r of lane quarter q holds row 4q + r).
// BF16x3: v_mfma_f32_16x16x16_bf16 over 8 K-steps of 16 columns (lane
// quarter q supplies k = 4q .. 4q+3). Operator and inputs are split into a
// high and a low BF16 part (x = x_hi + x_lo, each round-to-nearest-even) and
// the three products lo*hi, hi*lo, hi*hi are accumulated in FP32; the lo*lo
// term is dropped (relative weight 2^-16 and below).
// Both run two z-adjacent batches per wave (StepsF32Pair, StepsBf16Pair), on
// a single grid and in batches of shots.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "batch_common.h"
#include "fused_common.h"
#include "kernels.h"

namespace hermite {
namespace {

using fused::butterfly8;
using fused::Cell16;
using fused::cell_nodes;
using fused::OwnSchedule;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));  // 4 BF16 bit patterns

constexpr int kF32Floats = 8 * 32 * 64;      // [class][step][lane]
constexpr int kBf16Vecs = 8 * 8 * 2 * 64;    // [class][K-step][hi/lo][lane] of 4 BF16

// Corner values of step T: column 32 q + u[T]; `base` is src + 32 q pitch.
template <int T>
__device__ __forceinline__ void load_own(const double* __restrict__ base, size_t pitch, const Cell16& c, double* v) {
    constexpr OwnSchedule S{};
    const double* __restrict__ b = base + (size_t)S.u[T] * pitch;
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = b[c.corner[s]];
}

// ---------------------------------------------------------------- FP32
// Two batches per wave, the cells (x, y, z) and (x, y, z + 1), as in the FP64
// 4x4-tile kernel: every operator value read from LDS feeds both, and the
// lower corner plane of the second cell is the upper plane of the first, so
// a step loads 12 corner values (ra: the first cell's 8, rb: the second
// cell's upper 4) instead of 16. A step's matrix work is short in FP32, and
// with one wave per SIMD only the prefetch hides the gathers: kAheadPair
// steps are in flight.
constexpr int kAheadPair = 4;
constexpr int kRingPair = kAheadPair + 1;
template <int T>
__device__ __forceinline__ void load_own_upper(const double* __restrict__ base, size_t pitch, const Cell16& c,
                                               double* v) {
    constexpr OwnSchedule S{};
    const double* __restrict__ b = base + (size_t)S.u[T] * pitch;
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = b[c.corner[4 + s]];
}

template <int T>
struct PrologueF32Pair {
    __device__ __forceinline__ static void run(const double* __restrict__ base, size_t pitch, const Cell16& ca,
                                               const Cell16& cb, double (*ra)[8], double (*rb)[4]) {
        load_own<T>(base, pitch, ca, ra[T]);
        load_own_upper<T>(base, pitch, cb, rb[T]);
        if constexpr (T + 1 < kAheadPair) PrologueF32Pair<T + 1>::run(base, pitch, ca, cb, ra, rb);
    }
};

template <int T>
struct StepsF32Pair {
    __device__ __forceinline__ static void run(const double* __restrict__ base, size_t pitch, const Cell16& ca,
                                               const Cell16& cb, int lane, const float* sA, f4* acca, f4* accb,
                                               double (*P0a)[4], double (*P0b)[4], double (*ra)[8],
                                               double (*rb)[4]) {
        constexpr OwnSchedule S{};
        constexpr int u = S.u[T], dp = OwnSchedule::parity(u), rg = OwnSchedule::reg(u);
        constexpr int AH = kAheadPair;
        if constexpr (T + AH < 32) {
            load_own<T + AH>(base, pitch, ca, ra[(T + AH) % kRingPair]);
            load_own_upper<T + AH>(base, pitch, cb, rb[(T + AH) % kRingPair]);
        }
        double Ta[8], Tb[8], vb[8];
#pragma unroll
        for (int s = 0; s < 4; ++s) vb[s] = ra[T % kRingPair][4 + s], vb[4 + s] = rb[T % kRingPair][s];
        butterfly8(ra[T % kRingPair], Ta);
        butterfly8(vb, Tb);
        P0a[dp][rg] = 0.125 * Ta[0];
        P0b[dp][rg] = 0.125 * Tb[0];
        float a[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) a[p] = sA[(p * 32 + T) * 64 + lane];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            acca[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[p], (float)Ta[p ^ dp], acca[p], 0, 0, 0);
            accb[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[p], (float)Tb[p ^ dp], accb[p], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (T + 1 < 32)
            StepsF32Pair<T + 1>::run(base, pitch, ca, cb, lane, sA, acca, accb, P0a, P0b, ra, rb);
    }
};

// ---------------------------------------------------------------- BF16x3
// BF16x3, two z-adjacent batches per wave (as StepsF32Pair): the split
// operator tiles read from LDS feed both batches' three products.
constexpr int kAheadBf16Pair = 3;
constexpr int kRingBf16Pair = kAheadBf16Pair + 1;

template <int T>
struct PrologueBf16Pair {
    __device__ __forceinline__ static void run(const double* __restrict__ base, size_t pitch, const Cell16& ca,
                                               const Cell16& cb, double (*ra)[8], double (*rb)[4]) {
        load_own<T>(base, pitch, ca, ra[T]);
        load_own_upper<T>(base, pitch, cb, rb[T]);
        if constexpr (T + 1 < kAheadBf16Pair) PrologueBf16Pair<T + 1>::run(base, pitch, ca, cb, ra, rb);
    }
};

template <int T>
struct StepsBf16Pair {
    __device__ __forceinline__ static void run(const double* __restrict__ base, size_t pitch, const Cell16& ca,
                                               const Cell16& cb, int lane, const s4* sA, f4* acca, f4* accb,
                                               double (*P0a)[4], double (*P0b)[4], double (*ra)[8], double (*rb)[4],
                                               s4* Bhia, s4* Bloa, s4* Bhib, s4* Blob) {
        constexpr OwnSchedule S{};
        constexpr int u = S.u[T], dp = OwnSchedule::parity(u), rg = OwnSchedule::reg(u);
        constexpr int ks = T / 4, e = T % 4;
        constexpr int AH = kAheadBf16Pair, R = kRingBf16Pair;
        if constexpr (T + AH < 32) {
            load_own<T + AH>(base, pitch, ca, ra[(T + AH) % R]);
            load_own_upper<T + AH>(base, pitch, cb, rb[(T + AH) % R]);
        }
        double Ta[8], Tb[8], vb[8];
#pragma unroll
        for (int s = 0; s < 4; ++s) vb[s] = ra[T % R][4 + s], vb[4 + s] = rb[T % R][s];
        butterfly8(ra[T % R], Ta);
        butterfly8(vb, Tb);
        P0a[dp][rg] = 0.125 * Ta[0];
        P0b[dp][rg] = 0.125 * Tb[0];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const float xa = (float)Ta[p ^ dp], xb = (float)Tb[p ^ dp];
            const __bf16 ha = (__bf16)xa, hb = (__bf16)xb;  // round to nearest even
            Bhia[p][e] = __builtin_bit_cast(short, ha);
            Bloa[p][e] = __builtin_bit_cast(short, (__bf16)(xa - (float)ha));
            Bhib[p][e] = __builtin_bit_cast(short, hb);
            Blob[p][e] = __builtin_bit_cast(short, (__bf16)(xb - (float)hb));
        }
        if constexpr (e == 3) {
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                const s4 ahi = sA[((p * 8 + ks) * 2 + 0) * 64 + lane];
                const s4 alo = sA[((p * 8 + ks) * 2 + 1) * 64 + lane];
                acca[p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, Bhia[p], acca[p], 0, 0, 0);
                accb[p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, Bhib[p], accb[p], 0, 0, 0);
                acca[p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, Bloa[p], acca[p], 0, 0, 0);
                accb[p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, Blob[p], accb[p], 0, 0, 0);
                acca[p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, Bhia[p], acca[p], 0, 0, 0);
                accb[p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, Bhib[p], accb[p], 0, 0, 0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (T + 1 < 32)
            StepsBf16Pair<T + 1>::run(base, pitch, ca, cb, lane, sA, acca, accb, P0a, P0b, ra, rb, Bhia, Bloa, Bhib,
                                      Blob);
    }
};

// y = P0 + (double) acc; register r of quarter q of class p is the new value
// of field q/2 with derivative orders j = p + 2 (r % 2, r / 2, q % 2).
__device__ __forceinline__ void store_batch(double* __restrict__ dst, size_t plane, const Cell16& c, int q,
                                            const f4* acc, double (*P0)[4]) {
    const int fo = q >> 1, o3 = q & 1;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int p1 = p & 1, p2 = (p >> 1) & 1, p3 = p >> 2;
        const int j3 = p3 + 2 * o3;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j1 = p1 + 2 * (r & 1), j2 = p2 + 2 * (r >> 1);
            dst[(size_t)(fo * 64 + (j3 * 4 + j2) * 4 + j1) * plane + c.out] = P0[p][r] + (double)acc[p][r];
        }
    }
}

// The batch of row (y, z) and the one above it, row (y, z + 1) (periodic),
// stored only if upper is set; PREC 1 = FP32, 2 = BF16x3.
template <int PREC>
__device__ __forceinline__ void run_batch_pair_mixed(const double* __restrict__ src, double* __restrict__ dst,
                                                     size_t pitch, uint32_t n, uint32_t off, uint32_t x0, uint32_t y,
                                                     uint32_t z, bool upper, int lane, int cl, int q,
                                                     const unsigned char* sbuf) {
    const uint32_t x = x0 + cl;
    const bool valid = x < n;
    const uint32_t cx = valid ? (x + n - off) % n : n - 1;
    const uint32_t zb = (z + 1 == n) ? 0 : z + 1;
    const Cell16 ca = cell_nodes((z * n + y) * n + cx, n, off);
    const Cell16 cb = cell_nodes((zb * n + y) * n + cx, n, off);
    const double* base = src + (size_t)(32 * q) * pitch;
    asm volatile("" : "+v"(base));
    f4 acca[8], accb[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) acca[p] = accb[p] = f4{0.f, 0.f, 0.f, 0.f};
    double P0a[8][4], P0b[8][4];
    if constexpr (PREC == 1) {
        double ra[kRingPair][8], rb[kRingPair][4];
        PrologueF32Pair<0>::run(base, pitch, ca, cb, ra, rb);
        StepsF32Pair<0>::run(base, pitch, ca, cb, lane, (const float*)sbuf, acca, accb, P0a, P0b, ra, rb);
    } else {
        double ra[kRingBf16Pair][8], rb[kRingBf16Pair][4];
        s4 Bhia[8], Bloa[8], Bhib[8], Blob[8];
        PrologueBf16Pair<0>::run(base, pitch, ca, cb, ra, rb);
        StepsBf16Pair<0>::run(base, pitch, ca, cb, lane, (const s4*)sbuf, acca, accb, P0a, P0b, ra, rb, Bhia, Bloa,
                              Bhib, Blob);
    }
    if (valid) store_batch(dst, pitch, ca, q, acca, P0a);
    if (valid && upper) store_batch(dst, pitch, cb, q, accb, P0b);
}

template <int PREC>
__device__ __forceinline__ void load_operator(const void* __restrict__ Aops, unsigned char* sbuf) {
    constexpr int kBytes = (PREC == 1) ? kF32Floats * 4 : kBf16Vecs * 8;
    const uint4* g = (const uint4*)Aops;
    uint4* l = (uint4*)sbuf;
    for (int i = threadIdx.x; i < kBytes / 16; i += blockDim.x) l[i] = g[i];
    __syncthreads();
}

template <int PREC>
constexpr int kOpBytes = (PREC == 1) ? kF32Floats * 4 : kBf16Vecs * 8;

// A single grid in FP32 (PREC 1) or BF16x3 (PREC 2): two z-adjacent batches
// per wave over the queue-fed row-pair sweep (fused::sweep_row_pairs). The
// second set of accumulators and P0 values takes the registers of a second
// wave: one wave per SIMD, four per workgroup.
constexpr int kWavesPair = 4;

template <int PREC>
__global__ __launch_bounds__(kWavesPair * 64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void fused_mixed_pair_kernel(const double* __restrict__ src, double* __restrict__ dst, const void* __restrict__ Aops,
                             uint32_t n, size_t pitch, uint32_t off, uint32_t* __restrict__ queue) {
    __shared__ __attribute__((aligned(16))) unsigned char sbuf[kOpBytes<PREC>];
    load_operator<PREC>(Aops, sbuf);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane & 15, q = lane >> 4;
    fused::sweep_row_pairs(n, wave, kWavesPair, queue, [&](uint32_t x0, uint32_t y, uint32_t z, bool upper) {
        run_batch_pair_mixed<PREC>(src, dst, pitch, n, off, x0, y, z, upper, lane, cl, q, sbuf);
    });
}

// Batches of shots: item (bx, y, zp) of a shot, bx fastest, is the pair of
// rows (y, 2 zp) and (y, 2 zp + 1) at x-batch bx (n ceil(n/2) ceil(n/16)
// items per shot, the FP64 batch kernel's numbering).
template <int PREC>
__global__ __launch_bounds__(kWavesPair * 64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void fused_mixed_pair_batch_kernel(const batch::ShotGrid* __restrict__ shots, const uint32_t* __restrict__ ids,
                                   const uint32_t* __restrict__ prefix, uint32_t ng, uint32_t from,
                                   const void* __restrict__ Aops, uint32_t chunk, uint32_t interleaved) {
    __shared__ __attribute__((aligned(16))) unsigned char sbuf[kOpBytes<PREC>];
    load_operator<PREC>(Aops, sbuf);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane & 15, q = lane >> 4;
    batch::sweep_items(prefix[ng], wave, kWavesPair, chunk, interleaved, [&](uint32_t it) {
        const uint32_t g = batch::find_entry(prefix, ng, it);
        const batch::ShotGrid& S = shots[ids[g]];
        const uint32_t n = S.n, nbx = (n + 15) >> 4, local = it - prefix[g];
        const uint32_t bx = local % nbx, rest = local / nbx, y = rest % n, z = 2 * (rest / n);
        run_batch_pair_mixed<PREC>(S.grid[from], S.grid[1 - from], S.pitch, n, from, bx * 16, y, z, z + 1 < n, lane,
                                   cl, q, sbuf);
    });
}

uint16_t bf16_rne(float f) {
    uint32_t b;
    std::memcpy(&b, &f, 4);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

float bf16_to_float(uint16_t h) {
    const uint32_t b = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

}  // namespace

size_t mixed_operator_bytes(int precision) {
    return precision == 1 ? (size_t)kF32Floats * 4 : precision == 2 ? (size_t)kBf16Vecs * 8 : 0;
}

void mixed_build_operators(int precision, const double* K, void* out) {
    // K: [8][16][128] canonical class operators (rows (fo, o3, o2, o1), columns
    // f*64 + dd). Remainder operator K' = K - P0: the new value j of field fo
    // (row (fo, o), j = p + 2o) loses 1/8 on its own column (fo, d = j).
    constexpr OwnSchedule S{};
    auto kr = [&](int p, int row, int col) {
        const int fo = row >> 3, o3 = (row >> 2) & 1, o2 = (row >> 1) & 1, o1 = row & 1;
        const int j1 = (p & 1) + 2 * o1, j2 = ((p >> 1) & 1) + 2 * o2, j3 = (p >> 2) + 2 * o3;
        const int own = fo * 64 + (j3 * 4 + j2) * 4 + j1;
        return K[((size_t)p * 16 + row) * 128 + col] - (col == own ? 0.125 : 0.0);
    };
    if (precision == 1) {
        float* A = (float*)out;
        for (int p = 0; p < 8; ++p)
            for (int t = 0; t < 32; ++t)
                for (int lane = 0; lane < 64; ++lane)
                    A[((size_t)p * 32 + t) * 64 + lane] = (float)kr(p, lane & 15, 32 * (lane >> 4) + S.u[t]);
    } else {
        uint16_t* A = (uint16_t*)out;
        for (int p = 0; p < 8; ++p)
            for (int ks = 0; ks < 8; ++ks)
                for (int lane = 0; lane < 64; ++lane)
                    for (int e = 0; e < 4; ++e) {
                        const double v = kr(p, lane & 15, 32 * (lane >> 4) + S.u[4 * ks + e]);
                        const uint16_t hi = bf16_rne((float)v);
                        const uint16_t lo = bf16_rne((float)(v - (double)bf16_to_float(hi)));
                        A[((((size_t)p * 8 + ks) * 2 + 0) * 64 + lane) * 4 + e] = hi;
                        A[((((size_t)p * 8 + ks) * 2 + 1) * 64 + lane) * 4 + e] = lo;
                    }
    }
}

hipError_t launch_fused_mixed_batch(int precision, const batch::ShotGrid* shots, const uint32_t* ids,
                                    const uint32_t* prefix, uint32_t ng, int from, const void* Aops, int grid,
                                    uint32_t chunk, uint32_t interleaved, hipStream_t st) {
    if (grid < 8 || grid % 8 != 0 || chunk < 1) return hipErrorInvalidValue;
    if (precision == 1)
        hipLaunchKernelGGL(fused_mixed_pair_batch_kernel<1>, dim3(grid), dim3(kWavesPair * 64), 0, st, shots, ids,
                           prefix, ng, (uint32_t)from, Aops, chunk, interleaved);
    else if (precision == 2)
        hipLaunchKernelGGL(fused_mixed_pair_batch_kernel<2>, dim3(grid), dim3(kWavesPair * 64), 0, st, shots, ids,
                           prefix, ng, (uint32_t)from, Aops, chunk, interleaved);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_fused_mixed(int precision, const double* src, double* dst, const void* Aops, int n, size_t pitch,
                              int off, int grid, uint32_t* queue, hipStream_t st) {
    if (grid < 8 || grid % 8 != 0) return hipErrorInvalidValue;
    if (queue == nullptr) return hipErrorInvalidValue;
    if (precision == 1)
        hipLaunchKernelGGL(fused_mixed_pair_kernel<1>, dim3(grid), dim3(kWavesPair * 64), 0, st, src, dst, Aops,
                           (uint32_t)n, pitch, (uint32_t)off, queue);
    else if (precision == 2)
        hipLaunchKernelGGL(fused_mixed_pair_kernel<2>, dim3(grid), dim3(kWavesPair * 64), 0, st, src, dst, Aops,
                           (uint32_t)n, pitch, (uint32_t)off, queue);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace hermite
