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
// Both kernels gather at each node: they butterfly the adjoint values of the
// 8 neighbouring new nodes first and then run the transposed class products,
// as many as the forward half step (m = 3 on the matrix cores, m = 1, 2 on
// the vector ALUs).
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
// m = 3 on the FP64 matrix cores, gather form. With U_{p,r}[t] the butterfly
// of lam_y[p, r] over a node's 8 neighbours (node - s + off, s in {0,1}^3),
//   U_{p,r}[t] = sum_s sg(t, s) lam_y[p, r](node - s + off),
// the adjoint at the node is
//   g[c] = sum_p sum_r K_p[r][c] U_{p,r}[p xor par(c)],
// the forward kernel's contraction with the roles exchanged: the input
// columns are the 128 (class p, class row r) pairs of lam (32 K-steps of 4,
// step T holding class p = T / 4), the accumulators are the 8 parity groups
// pi of the output columns c (16 columns each: 2 fields x 2x2x2 orders), and
// group pi takes butterfly output p xor pi. The forward kernel's data flow
// on the 4x4-tile instruction (v_mfma_f64_4x4x4f64, 4 blocks): per group and
// K-step 4 row tiles, tile ri holding output rows (quarter i, register ri);
// each wave computes two batches of 16 nodes, rows (y, z) and (y, z + 1),
// which share every operator read and a plane of neighbours: the neighbours
// s3 = 1 of the upper node are the neighbours s3 = 0 of the lower one, so a
// step loads 12 values per lane instead of 16. Work comes from the
// context's queue (fused::sweep_row_pairs); no scratch.
// ---------------------------------------------------------------------------
constexpr int kAdjWaves = 4;                 // one wave per SIMD (two accumulator sets)
constexpr int kAdjOpDoubles = 8 * 32 * 64;  // [K-step][group][row-tile pair][4k + i][2]
constexpr int kAdjAhead = 2;
constexpr int kAdjRing = kAdjAhead + 1;

// Packed per-lane column table: step T, quarter q reads the lam column of
// class T / 4, class row 4 (T % 4) + q (7 bits, four steps per word).
struct AdjColTable {
    uint32_t w[4][8];
    constexpr AdjColTable() : w() {
        constexpr AdjLayout<4> L{};
        for (int q = 0; q < 4; ++q)
            for (int T = 0; T < 32; ++T) w[q][T >> 2] |= (uint32_t)L.row_col[T >> 2][4 * (T & 3) + q] << (8 * (T & 3));
    }
};
__constant__ AdjColTable kAdjColTable = AdjColTable();

// Column c of logical output row l = 4 g + r of parity group pi (register r of
// lane quarter g): field g / 2, d_x = pi_x + 2 b_x with b3 = g % 2, b2 = r / 2,
// b1 = r % 2.
__host__ __device__ constexpr int adj_out_col(int pi, int g, int r) {
    const int d1 = (pi & 1) + 2 * (r & 1), d2 = ((pi >> 1) & 1) + 2 * (r >> 1), d3 = (pi >> 2) + 2 * (g & 1);
    return (g >> 1) * 64 + (d3 * 4 + d2) * 4 + d1;
}

// The 8 neighbours node - s + off of a node (per axis, periodic), as corners.
__device__ __forceinline__ fused::Cell16 node_neighbours(uint32_t node, uint32_t n, uint32_t off) {
    const uint32_t i = node % n, t = node / n, j = t % n, k = t / n;
    uint32_t xs[2], ys[2], zs[2];
    if (off) {
        xs[0] = (i + 1 == n) ? 0 : i + 1, xs[1] = i;
        ys[0] = (j + 1 == n) ? 0 : j + 1, ys[1] = j;
        zs[0] = (k + 1 == n) ? 0 : k + 1, zs[1] = k;
    } else {
        xs[0] = i, xs[1] = i ? i - 1 : n - 1;
        ys[0] = j, ys[1] = j ? j - 1 : n - 1;
        zs[0] = k, zs[1] = k ? k - 1 : n - 1;
    }
    fused::Cell16 c;
#pragma unroll
    for (int s = 0; s < 8; ++s) c.corner[s] = (zs[s >> 2] * n + ys[(s >> 1) & 1]) * n + xs[s & 1];
    c.out = node;
    return c;
}

template <int T>
__device__ __forceinline__ void adj_load_step(const double* __restrict__ lam, size_t plane, const fused::Cell16& c,
                                              const uint32_t* packed, double* v) {
    const double* __restrict__ b = lam + (size_t)((packed[T >> 2] >> (8 * (T & 3))) & 0xFFu) * plane;
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = b[c.corner[s]];
}

// Neighbours s = 0 .. 3 (the s3 = 0 plane) of a node, lam column of step T.
template <int T>
__device__ __forceinline__ void adj_load_lower(const double* __restrict__ lam, size_t plane, const fused::Cell16& c,
                                               const uint32_t* packed, double* v) {
    const double* __restrict__ b = lam + (size_t)((packed[T >> 2] >> (8 * (T & 3))) & 0xFFu) * plane;
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = b[c.corner[s]];
}

// ra: the lower node's 8 neighbour values; rb: the upper node's s3 = 0 four.
template <int T>
struct AdjStepsPair {
    __device__ __forceinline__ static void run(const double* __restrict__ lam, size_t plane, const fused::Cell16& ca,
                                               const fused::Cell16& cb, const uint32_t* packed, int lane,
                                               const double* sK, double (*acca)[4], double (*accb)[4],
                                               double (*ra)[8], double (*rb)[4]) {
        constexpr int p = T >> 2;  // class of this step's lam rows
        if constexpr (T + kAdjAhead < 32) {
            adj_load_step<T + kAdjAhead>(lam, plane, ca, packed, ra[(T + kAdjAhead) % kAdjRing]);
            adj_load_lower<T + kAdjAhead>(lam, plane, cb, packed, rb[(T + kAdjAhead) % kAdjRing]);
        }
        double Ua[8], Ub[8], vb[8];
#pragma unroll
        for (int s = 0; s < 4; ++s) vb[s] = rb[T % kAdjRing][s], vb[4 + s] = ra[T % kAdjRing][s];
        fused::butterfly8(ra[T % kAdjRing], Ua);
        fused::butterfly8(vb, Ub);
        // this lane's A[i][k] (k = lane / 16, i = lane % 4) for row tiles
        // 2 rp and 2 rp + 1 of group pi: one 16-byte read
        const int at = ((lane >> 4) << 2) | (lane & 3);
        const double2* __restrict__ sT = reinterpret_cast<const double2*>(sK) + (size_t)T * 8 * 2 * 16 + at;
        double2 a[2][2];  // [group parity of the pipeline][rp]
#pragma unroll
        for (int rp = 0; rp < 2; ++rp) a[0][rp] = sT[(0 * 2 + rp) * 16];
#pragma unroll
        for (int pi = 0; pi < 8; ++pi) {
            if (pi + 1 < 8) {
#pragma unroll
                for (int rp = 0; rp < 2; ++rp) a[(pi + 1) & 1][rp] = sT[((pi + 1) * 2 + rp) * 16];
            }
#pragma unroll
            for (int ri = 0; ri < 4; ++ri) {
                const double2 av = a[pi & 1][ri >> 1];
                const double x = (ri & 1) ? av.y : av.x;
                acca[pi][ri] = __builtin_amdgcn_mfma_f64_4x4x4f64(x, Ua[pi ^ p], acca[pi][ri], 0, 0, 0);
                accb[pi][ri] = __builtin_amdgcn_mfma_f64_4x4x4f64(x, Ub[pi ^ p], accb[pi][ri], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (T + 1 < 32) AdjStepsPair<T + 1>::run(lam, plane, ca, cb, packed, lane, sK, acca, accb, ra, rb);
    }
};

template <int T>
struct AdjProloguePair {
    __device__ __forceinline__ static void run(const double* __restrict__ lam, size_t plane, const fused::Cell16& ca,
                                               const fused::Cell16& cb, const uint32_t* packed, double (*ra)[8],
                                               double (*rb)[4]) {
        adj_load_step<T>(lam, plane, ca, packed, ra[T]);
        adj_load_lower<T>(lam, plane, cb, packed, rb[T]);
        if constexpr (T + 1 < kAdjAhead) AdjProloguePair<T + 1>::run(lam, plane, ca, cb, packed, ra, rb);
    }
};

__device__ __forceinline__ void adj_store(double* __restrict__ lam_src, size_t pitch, uint32_t node, int q,
                                          const double (*acc)[4]) {
#pragma unroll
    for (int pi = 0; pi < 8; ++pi)
#pragma unroll
        for (int r = 0; r < 4; ++r) lam_src[(size_t)adj_out_col(pi, q, r) * pitch + node] = acc[pi][r];
}

// Persistent kernel over the queue-fed row-pair sweep: one pair of 16-node
// batches per wave and item, nodes x0 .. x0+15 of rows (y, z) and (y, z + 1)
// (periodic; the second stored only if upper is set).
__global__ __launch_bounds__(kAdjWaves * 64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void adjoint_mfma_kernel(const double* __restrict__ lam_dst, double* __restrict__ lam_src,
                         const double* __restrict__ KT, uint32_t n, size_t pitch, uint32_t off,
                         uint32_t* __restrict__ queue) {
    __shared__ double sK[kAdjOpDoubles];
    for (int i = threadIdx.x; i < kAdjOpDoubles; i += blockDim.x) sK[i] = KT[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane & 15, q = lane >> 4;
    uint32_t packed[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) packed[k] = kAdjColTable.w[q][k];
    fused::sweep_row_pairs(n, wave, kAdjWaves, queue, [&](uint32_t x0, uint32_t y, uint32_t z, bool upper) {
        const uint32_t x = x0 + cl;
        const bool valid = x < n;
        const uint32_t xx = valid ? x : n - 1, zb = (z + 1 == n) ? 0 : z + 1;
        const uint32_t na = (z * n + y) * n + xx, nb = (zb * n + y) * n + xx;
        const fused::Cell16 ca = node_neighbours(na, n, off);
        const fused::Cell16 cb = node_neighbours(nb, n, off);
        // opaque per item (keeps the per-lane column bases from being hoisted
        // out of the sweep, which would pin 64 registers)
#pragma unroll
        for (int w = 0; w < 8; ++w) asm volatile("" : "+v"(packed[w]));
        double acca[8][4], accb[8][4];
#pragma unroll
        for (int pi = 0; pi < 8; ++pi)
#pragma unroll
            for (int r = 0; r < 4; ++r) acca[pi][r] = accb[pi][r] = 0.0;
        double ra[kAdjRing][8], rb[kAdjRing][4];
        AdjProloguePair<0>::run(lam_dst, pitch, ca, cb, packed, ra, rb);
        AdjStepsPair<0>::run(lam_dst, pitch, ca, cb, packed, lane, sK, acca, accb, ra, rb);
        if (valid) adj_store(lam_src, pitch, na, q, acca);
        if (valid && upper) adj_store(lam_src, pitch, nb, q, accb);
    });
}

// ---------------------------------------------------------------------------
// m = 1, 2 on the vector ALUs, the same gather form: one lane per node, all
// 2 M^3 adjoint values. The 2 M^3 (class p, row r) columns of lam are
// unrolled at compile time: the 8 neighbour values of column (p, r) are
// butterflied once, and output c takes butterfly output p xor par(c) times
// K_p[r][c], a wave-uniform scalar operand of the canonical operator.
// Entries that vanish for every time step (even class parity along an axis,
// row order 2 there, column order 0 there) are skipped.
// ---------------------------------------------------------------------------
template <int M>
struct AdjSmall {
    static constexpr int M3 = M * M * M, NC = 2 * M3;
    int p[NC], r[NC];     // column step -> (class, class row)
    bool zero[NC][NC];    // (column step, output c): structural zero
    constexpr AdjSmall() : p(), r(), zero() {
        constexpr AdjLayout<M> L{};
        int k = 0;
        for (int q = 0; q < 8; ++q)
            for (int rr = 0; rr < L.nrows[q]; ++rr, ++k) {
                p[k] = q;
                r[k] = rr;
                const int n1 = (M + 1 - (q & 1)) / 2, n2 = (M + 1 - ((q >> 1) & 1)) / 2;
                const int nof = n1 * n2 * ((M + 1 - (q >> 2)) / 2), w = rr % nof;
                const int o1 = w % n1, o2 = (w / n1) % n2, o3 = w / (n1 * n2);
                for (int c = 0; c < NC; ++c) {
                    const int d = c % M3, d1 = d % M, d2 = (d / M) % M, d3 = d / (M * M);
                    zero[k][c] = ((q & 1) == 0 && o1 == 1 && d1 == 0) || (((q >> 1) & 1) == 0 && o2 == 1 && d2 == 0) ||
                                 ((q >> 2) == 0 && o3 == 1 && d3 == 0);
                }
            }
    }
};

template <int M, int S>
struct AdjSmallSteps {
    __device__ __forceinline__ static void run(const double* __restrict__ lam, size_t pitch, const fused::Cell16& nb,
                                               const double* __restrict__ K, double* acc) {
        constexpr AdjLayout<M> L{};
        constexpr AdjSmall<M> A{};
        constexpr int NC = AdjSmall<M>::NC, M3 = AdjSmall<M>::M3, RM = AdjLayout<M>::RM;
        constexpr int p = A.p[S], r = A.r[S];
        const double* __restrict__ b = lam + (size_t)L.row_col[p][r] * pitch;
        double v[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = b[nb.corner[s]];
        double U[8];
        fused::butterfly8(v, U);
        const double* __restrict__ kk = K + ((size_t)p * RM + r) * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (!A.zero[S][c]) acc[c] = __builtin_fma(kk[c], U[p ^ AdjLayout<M>::par(c % M3)], acc[c]);
        if constexpr (S + 1 < NC) AdjSmallSteps<M, S + 1>::run(lam, pitch, nb, K, acc);
    }
};

template <int M>
__global__ __launch_bounds__(kThreads) void adjoint_kernel(const double* __restrict__ lam_dst,
                                                           double* __restrict__ lam_src,
                                                           const double* __restrict__ K, uint32_t n, size_t pitch,
                                                           uint32_t off) {
    constexpr int NC = AdjSmall<M>::NC;
    const uint32_t node = blockIdx.x * kThreads + threadIdx.x;
    if (node >= n * n * n) return;
    const fused::Cell16 nb = node_neighbours(node, n, off);
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    AdjSmallSteps<M, 0>::run(lam_dst, pitch, nb, K, acc);
#pragma unroll
    for (int c = 0; c < NC; ++c) lam_src[(size_t)c * pitch + node] = acc[c];
}

}  // namespace

size_t adjoint_mfma_operator_doubles() { return (size_t)kAdjOpDoubles; }

void adjoint_mfma_build_operator(const double* K, double* KT) {
    // K: canonical [8][16][128]. Row tile ri of group pi at step T (p = T / 4):
    // A[i][k] = K_p[4 (T % 4) + k][column of the output row held in register ri
    // of lane quarter i], stored at ((((T 8 + pi) 2 + ri / 2) 16 + 4 k + i) 2 +
    // ri % 2: a lane reads the two tiles of a row-tile pair as one 16-byte value.
    for (int T = 0; T < 32; ++T)
        for (int pi = 0; pi < 8; ++pi)
            for (int ri = 0; ri < 4; ++ri)
                for (int k = 0; k < 4; ++k)
                    for (int i = 0; i < 4; ++i)
                        KT[((((size_t)T * 8 + pi) * 2 + (ri >> 1)) * 16 + 4 * k + i) * 2 + (ri & 1)] =
                            K[((size_t)(T >> 2) * 16 + 4 * (T & 3) + k) * 128 + adj_out_col(pi, i, ri)];
}

hipError_t launch_adjoint_mfma(const double* lam_dst, double* lam_src, const double* KT, int n, size_t pitch, int off,
                               int grid, uint32_t* queue, hipStream_t st) {
    if (grid < 8 || grid % 8 != 0 || queue == nullptr) return hipErrorInvalidValue;
    hipLaunchKernelGGL(adjoint_mfma_kernel, dim3(grid), dim3(kAdjWaves * 64), 0, st, lam_dst, lam_src, KT,
                       (uint32_t)n, pitch, (uint32_t)off, queue);
    return hipGetLastError();
}

hipError_t launch_adjoint(int m, const double* lam_dst, double* lam_src, const double* K, int n, size_t pitch, int off,
                          hipStream_t st) {
    const uint32_t ncell = (uint32_t)n * n * n;
    const dim3 grid((ncell + kThreads - 1) / kThreads), block(kThreads);
    switch (m) {
        case 1: hipLaunchKernelGGL(adjoint_kernel<2>, grid, block, 0, st, lam_dst, lam_src, K, (uint32_t)n, pitch, (uint32_t)off); break;
        case 2: hipLaunchKernelGGL(adjoint_kernel<3>, grid, block, 0, st, lam_dst, lam_src, K, (uint32_t)n, pitch, (uint32_t)off); break;
        default: return hipErrorInvalidValue;  // m = 3: launch_adjoint_mfma
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
