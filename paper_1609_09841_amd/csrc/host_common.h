// Host-side helpers shared by the single-grid context and the batch.
#pragma once

#include <cstddef>
#include <string>

#include "hermite.h"
#include "kernels.h"

namespace hermite {

// Column pitch of the device grids: n^3 rounded up to whole 256-byte blocks,
// plus 5 cache lines (640 bytes). With the unpadded power-of-two strides of
// the common grid sizes, the 2 M^3 columns of one node (and of its
// neighbours) all map to the same L2 set and channel, and the cache holds
// almost none of the data that the 8 cells around a node share.
inline size_t column_pitch(size_t ncell) { return ((ncell + 31) / 32) * 32 + 80; }

// Empty string if src is a valid source, else the reason.
std::string check_source(const hermite_source& src);

// Source entry for a grid of n cells per side and order m (the caller fills
// grid[], pitch and steps); x reduced modulo 1, boxes for both half steps.
SourceDesc make_source_desc(const hermite_source& src, int n, int m, int q, double cfl, double c);

}  // namespace hermite
