// Device building blocks shared by the matrix-core fused half-step kernels
// (m = 3): cell corner addressing, the 2x2x2 parity butterfly of the corner
// data and the XCD-blocked sweep over the grid.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hermite {
namespace fused {

// The 8 corner nodes of one cell, s = s1 + 2 s2 + 4 s3, and the node of the
// other grid that the cell writes.
struct Cell16 {
    uint32_t corner[8];
    uint32_t out;
};

// Cell with lower corner (i, j, k) = flat index (k n + j) n + i, periodic in
// every axis; off = 0 writes node (i, j, k) (primal -> dual), off = 1 writes
// (i+1, j+1, k+1) mod n (dual -> primal).
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

// The same cell, enumerated by the node it writes: node (i, j, k) of the new
// grid comes from the cell with lower corner (i - off, j - off, k - off) mod
// n. Kernels that give consecutive lanes consecutive nodes this way store
// whole cache lines in both half steps (off = 1 would otherwise shift every
// store of a wave by one node).
__device__ __forceinline__ Cell16 cell_writing(uint32_t node, uint32_t n, uint32_t off) {
    const uint32_t i = node % n, t = node / n, j = t % n, k = t / n;
    uint32_t xs[2], ys[2], zs[2];
    if (off) {
        xs[0] = i ? i - 1 : n - 1, xs[1] = i;
        ys[0] = j ? j - 1 : n - 1, ys[1] = j;
        zs[0] = k ? k - 1 : n - 1, zs[1] = k;
    } else {
        xs[0] = i, xs[1] = (i + 1 == n) ? 0 : i + 1;
        ys[0] = j, ys[1] = (j + 1 == n) ? 0 : j + 1;
        zs[0] = k, zs[1] = (k + 1 == n) ? 0 : k + 1;
    }
    Cell16 c;
#pragma unroll
    for (int s = 0; s < 8; ++s) c.corner[s] = (zs[s >> 2] * n + ys[(s >> 1) & 1]) * n + xs[s & 1];
    c.out = node;
    return c;
}

// Cell of a z-slab of a periodic grid (x and y periodic, buffer planes k and
// k + 1 in z, no wrap): lower corner (i, j, k); it writes node (i + off,
// j + off) mod n on buffer plane k + 1 - off. A slab holds nz + 1 node planes
// per grid: the primal grid its own planes 0 .. nz-1 and, as plane nz, the
// first primal plane of the slab above; the dual grid, as plane 0, the last
// dual plane of the slab below and its own planes as 1 .. nz. Both half steps
// then update the cells on buffer planes 0 .. nz-1.
__device__ __forceinline__ Cell16 slab_cell_nodes(uint32_t i, uint32_t j, uint32_t k, uint32_t n, uint32_t off) {
    const uint32_t i1 = (i + 1 == n) ? 0 : i + 1, j1 = (j + 1 == n) ? 0 : j + 1;
    Cell16 c;
    const uint32_t xs[2] = {i, i1}, ys[2] = {j, j1}, zs[2] = {k, k + 1};
#pragma unroll
    for (int s = 0; s < 8; ++s) c.corner[s] = (zs[s >> 2] * n + ys[(s >> 1) & 1]) * n + xs[s & 1];
    c.out = ((k + 1 - off) * n + (off ? j1 : j)) * n + (off ? i1 : i);
    return c;
}

// Butterfly of the 8 corner values v[s1 + 2 s2 + 4 s3] of one derivative
// multi-index: T[t1 + 2 t2 + 4 t3] = sum_s prod_x (t_x ? (s_x ? 1 : -1) : 1) v[s]
// (t_x = 1: right minus left along x, t_x = 0: right plus left). Parity class
// p takes output t = p xor (d mod 2) of the butterfly of index d.
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

// Persistent sweep: one workgroup per CU, gridDim.x a multiple of 8, and
// workgroup b runs on XCD b % 8. Each XCD owns a slab of z-planes; its G/8
// workgroups form a block of BY rows (y) x BZ planes (z) that sweeps the
// slab, one x-row segment per workgroup per iteration, the waves of the
// workgroup taking its 16-cell batches (one each: a segment is 16 * waves
// cells, and rows longer than that are swept one segment after the other,
// so the block's working set does not grow with n). A node row is read by
// the cells on both sides of it in y and z; in this order those cells run at
// the same time on the same XCD, so the second read hits L2 instead of coming
// back from memory one iteration later. f(x0, y, z) runs the batch of cells
// x0 .. x0+15 of row (y, z).
template <class F>
__device__ __forceinline__ void sweep_rows(uint32_t n, int wave, int waves, F&& f) {
    const uint32_t wpx = gridDim.x / 8;  // workgroups per XCD
    const uint32_t BZ = (wpx % 4 == 0) ? 4 : (wpx % 2 == 0) ? 2 : 1, BY = wpx / BZ;
    const uint32_t xcd = blockIdx.x % 8, w = blockIdx.x / 8;
    const uint32_t yy = w % BY, zz = w / BY;
    const uint32_t z0 = xcd * n / 8, z1 = (xcd + 1) * n / 8;
    const uint32_t nyb = (n + BY - 1) / BY, ngr = (z1 - z0 + BZ - 1) / BZ;
    const uint32_t nbx = (n + 15) / 16, nseg = (nbx + waves - 1) / waves;
    for (uint32_t sg = 0; sg < nseg; ++sg) {
        const uint32_t bx = sg * waves + wave;
        for (uint32_t it = 0; it < nyb * ngr; ++it) {
            const uint32_t y = (it % nyb) * BY + yy, z = z0 + (it / nyb) * BZ + zz;
            if (y >= n || z >= z1 || bx >= nbx) continue;
            f(bx * 16, y, z);
        }
    }
}

// The sweep of the two-batch kernels, whose waves each take the cells of
// rows (y, z) and (y, z + 1) (a row pair; f's last argument says whether the
// second row belongs to this XCD's planes and is to be stored). Each XCD owns
// its slab of z-planes as in sweep_rows, cut into nzp row-pair planes. The
// batch positions (y, bx) of a plane, bx fastest, are dealt out in groups of
// one per wave, so that rows whose batch count is not a multiple of the wave
// count leave no wave idle. Items (row-pair plane, group) are numbered in
// tiles of BZ planes (BZ dividing nzp) x consecutive groups, and the XCD's
// workgroups take them from a counter in that order: the items in flight on
// an XCD are always a window of consecutive ones, whose rows share node rows
// in L2, however far the workgroups have drifted apart (a static round-robin
// assignment let them drift and read 1.4x more). The workgroup's first wave
// takes the next item while the current one runs.
//
// queue: 8 x 64 words, zero before the first launch; words 64 x and 64 x + 32
// are XCD x's item counter and finished-workgroup counter. The last workgroup
// of an XCD to finish sets both back to zero, so consecutive launches on one
// stream need no reset; launches that run at the same time need queues of
// their own. This XCD's rows are y0 .. y1-1 of planes z0 .. z1-1; f(x0, y, z,
// upper) runs the pair at x0 .. x0+15.
template <class F>
__device__ __forceinline__ void sweep_row_pairs_in(uint32_t n, uint32_t y0, uint32_t y1, uint32_t z0, uint32_t z1,
                                                   int wave, int waves, uint32_t* queue, F&& f) {
    const uint32_t wpx = gridDim.x / 8;
    const uint32_t xcd = blockIdx.x % 8;
    const uint32_t nzp = (z1 - z0 + 1) / 2;
    const uint32_t nbx = (n + 15) / 16, npos = (y1 - y0) * nbx, NG = (npos + waves - 1) / waves;
    const uint32_t BZ = (nzp % 4 == 0) ? 4 : (nzp % 2 == 0) ? 2 : 1;
    const uint32_t NI = nzp * NG;
    uint32_t* ctr = queue + 64 * xcd;
    uint32_t* done = ctr + 32;
    // item numbers handed to the waves; the two slots alternate, so a slot is
    // written only after every wave has passed the barrier that follows its read
    __shared__ uint32_t s_item[2];
    if (threadIdx.x == 0) s_item[0] = atomicAdd(ctr, 1u);
    __syncthreads();
    uint32_t i = s_item[0];
    int slot = 0;
    while (i < NI) {
        uint32_t next = 0;
        if (threadIdx.x == 0) next = atomicAdd(ctr, 1u);
        const uint32_t zz = i % BZ, rest = i / BZ, g = rest % NG, zp = (rest / NG) * BZ + zz;
        const uint32_t pos = g * waves + wave;
        if (pos < npos) {
            const uint32_t z = z0 + 2 * zp;
            f((pos % nbx) * 16, y0 + pos / nbx, z, z + 1 < z1);
        }
        if (threadIdx.x == 0) s_item[slot ^ 1] = next;
        __syncthreads();
        slot ^= 1;
        i = s_item[slot];
    }
    // every workgroup's last atomicAdd on ctr has returned before it counts
    // itself here, so the last one to arrive can reset both
    if (threadIdx.x == 0 && atomicAdd(done, 1u) == wpx - 1) {
        atomicExch(ctr, 0u);
        atomicExch(done, 0u);
    }
}

// The periodic cube: XCD x owns planes x n / 8 .. (x + 1) n / 8 - 1.
template <class F>
__device__ __forceinline__ void sweep_row_pairs(uint32_t n, int wave, int waves, uint32_t* queue, F&& f) {
    const uint32_t xcd = blockIdx.x % 8;
    sweep_row_pairs_in(n, 0, n, xcd * n / 8, (xcd + 1) * n / 8, wave, waves, queue, f);
}

// The cell planes k0 .. k1-1 of a slab, split among the XCDs as in
// sweep_rows_slab: along z when deep, along y when thin.
template <class F>
__device__ __forceinline__ void sweep_row_pairs_slab(uint32_t n, uint32_t k0, uint32_t k1, int wave, int waves,
                                                     uint32_t* queue, F&& f) {
    const uint32_t xcd = blockIdx.x % 8, nz = k1 - k0;
    if (nz >= 32)
        sweep_row_pairs_in(n, 0, n, k0 + xcd * nz / 8, k0 + (xcd + 1) * nz / 8, wave, waves, queue, f);
    else
        sweep_row_pairs_in(n, xcd * n / 8, (xcd + 1) * n / 8, k0, k1, wave, waves, queue, f);
}

// The same sweep over the rows (y, k) of the cell planes k0 .. k1-1 of a
// slab. A deep range is split among the XCDs along z as the cube is; a thin
// one (fewer than 4 planes per XCD) along y, so that each XCD still sweeps a
// block of rows several planes deep and the second read of a node row hits
// its L2.
template <class F>
__device__ __forceinline__ void sweep_rows_slab(uint32_t n, uint32_t k0, uint32_t k1, int wave, int waves, F&& f) {
    const uint32_t wpx = gridDim.x / 8;
    const uint32_t xcd = blockIdx.x % 8, w = blockIdx.x / 8;
    const uint32_t nz = k1 - k0;
    const bool by_z = nz >= 32;
    const uint32_t z0 = k0 + (by_z ? xcd * nz / 8 : 0), z1 = k0 + (by_z ? (xcd + 1) * nz / 8 : nz);
    const uint32_t y0 = by_z ? 0 : xcd * n / 8, y1 = by_z ? n : (xcd + 1) * n / 8;
    const uint32_t pz = z1 - z0, py = y1 - y0;
    const uint32_t BZ = (wpx % 4 == 0 && pz >= 4) ? 4 : (wpx % 2 == 0 && pz >= 2) ? 2 : 1, BY = wpx / BZ;
    const uint32_t yy = w % BY, zz = w / BY;
    const uint32_t nyb = (py + BY - 1) / BY, ngr = (pz + BZ - 1) / BZ;
    const uint32_t nbx = (n + 15) / 16, nseg = (nbx + waves - 1) / waves;
    for (uint32_t sg = 0; sg < nseg; ++sg) {
        const uint32_t bx = sg * waves + wave;
        for (uint32_t it = 0; it < nyb * ngr; ++it) {
            const uint32_t y = y0 + (it % nyb) * BY + yy, z = z0 + (it / nyb) * BZ + zz;
            if (y >= y1 || z >= z1 || bx >= nbx) continue;
            f(bx * 16, y, z);
        }
    }
}

// Input-column schedule of the mixed-precision kernels: lane quarter q reads
// the columns of field q/2 with d3 in {2 (q%2), 2 (q%2) + 1}, which are exactly
// the 32 new values (of field q/2 and o3 = q%2) that its accumulators hold.
// Step t reads column 32 q + u[t], u = 16 b3 + 4 d2 + d1 (d3 = 2 (q%2) + b3),
// in order of decreasing b3 + d2 + d1. The parity pattern of d, and so the
// butterfly output that feeds each class, depends on t only.
struct OwnSchedule {
    int u[32];
    constexpr OwnSchedule() : u() {
        int t = 0;
        for (int s = 7; s >= 0; --s)
            for (int b3 = 0; b3 < 2; ++b3)
                for (int d2 = 0; d2 < 4; ++d2)
                    for (int d1 = 0; d1 < 4; ++d1)
                        if (b3 + d2 + d1 == s) u[t++] = 16 * b3 + 4 * d2 + d1;
    }
    static constexpr int parity(int u) { return (u & 1) | (((u >> 2) & 1) << 1) | ((u >> 4) << 2); }
    // accumulator register (o2, o1) of the new value j = d read at u
    static constexpr int reg(int u) { return ((u >> 3) & 1) * 2 + ((u >> 1) & 1); }
};

}  // namespace fused
}  // namespace hermite
