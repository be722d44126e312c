// Batches of independent grids (shots) in one launch: the shot table and the
// mapping of a launch's work items onto shots.
//
// A batched launch covers the shots of one order m. Its work is a list of
// items (a 16-cell batch of one x-row for the matrix-core kernels, a block of
// cells for the vector kernels), numbered shot after shot; prefix[g] is the
// first item of group entry g and prefix[ng] the total. Group entry g is shot
// ids[g] of the shot table. Both half steps use the same tables: the source
// grid is grid[from], the destination grid[1 - from].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hermite {
namespace batch {

struct ShotGrid {
    double* grid[2];  // primal, dual: 2 M^3 columns of `pitch` doubles each
    uint64_t pitch;   // doubles between consecutive columns (>= n^3)
    uint32_t n;       // cells per side
    uint32_t m;       // derivatives per dimension
};

// Group entry holding work item `item` (prefix[0] = 0 <= item < prefix[ng]).
// `item` must be wave-uniform; the search then runs on scalar registers.
__device__ __forceinline__ uint32_t find_entry(const uint32_t* __restrict__ prefix, uint32_t ng, uint32_t item) {
    uint32_t lo = 0, hi = ng;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Item order of the persistent matrix-core kernels: the item list is cut into
// 8 contiguous slabs, one per XCD (workgroup b runs on XCD b mod 8), so cells
// that share nodes run under the same L2; within a slab the waves of the
// XCD's workgroups take runs of `chunk` consecutive items in turn
// (interleaved = 1 deals runs round-robin over the whole list instead).
// f(item) is called with wave-uniform items.
template <class F>
__device__ __forceinline__ void sweep_items(uint32_t total, int wave, int waves, uint32_t chunk, uint32_t interleaved,
                                            F&& f) {
    uint32_t lo, hi, first, stride;
    if (interleaved) {
        lo = 0;
        hi = total;
        first = (blockIdx.x * (uint32_t)waves + (uint32_t)wave) * chunk;
        stride = gridDim.x * (uint32_t)waves * chunk;
    } else {
        const uint32_t xcd = blockIdx.x & 7, wpx = gridDim.x >> 3, w = blockIdx.x >> 3;
        lo = (uint32_t)(((uint64_t)total * xcd) >> 3);
        hi = (uint32_t)(((uint64_t)total * (xcd + 1)) >> 3);
        first = lo + (w * (uint32_t)waves + (uint32_t)wave) * chunk;
        stride = wpx * (uint32_t)waves * chunk;
    }
    for (uint32_t b = __builtin_amdgcn_readfirstlane(first); b < hi; b += stride) {
        const uint32_t e = (b + chunk < hi) ? b + chunk : hi;
        for (uint32_t it = b; it < e; ++it) f(it);
    }
}

}  // namespace batch
}  // namespace hermite
