// Host-side helpers shared by the single-grid context and the batch.
#include "host_common.h"

#include <cmath>
#include <cstdio>

namespace hermite {

std::string check_source(const hermite_source& src) {
    char buf[160];
    for (int x = 0; x < 3; ++x)
        if (!std::isfinite(src.x[x])) {
            std::snprintf(buf, sizeof(buf), "source x[%d] not finite", x);
            return buf;
        }
    if (!std::isfinite(src.sigma) || !(src.sigma > 0.0)) {
        std::snprintf(buf, sizeof(buf), "source sigma=%g must be finite and > 0", src.sigma);
        return buf;
    }
    if (!std::isfinite(src.freq) || src.freq < 0.0) {
        std::snprintf(buf, sizeof(buf), "source freq=%g must be finite and >= 0", src.freq);
        return buf;
    }
    if (!std::isfinite(src.t0) || !std::isfinite(src.amplitude)) return "source t0 and amplitude must be finite";
    return "";
}

SourceDesc make_source_desc(const hermite_source& src, int n, int m, int q, double cfl, double c) {
    SourceDesc d{};
    d.n = (uint32_t)n;
    d.m = (uint32_t)m;
    d.q = (uint32_t)q;
    for (int x = 0; x < 3; ++x) d.x[x] = src.x[x] - std::floor(src.x[x]);
    d.sigma = src.sigma;
    d.amp = src.amplitude;
    d.f0 = src.freq;
    d.t0 = src.t0;
    d.h = 1.0 / n;
    d.dt = cfl * d.h / c;
    d.tau = 0.5 * d.dt;
    d.lam = c * d.tau / d.h;
    d.pre = d.tau * d.h / c;
    // Cells (per axis, a periodic run of indices) whose centres may lie within
    // 6 sigma of the source; the kernel applies the exact cut-off per cell.
    // Centre of cell i: (i + 1/2) h on the primal grid, (i + 1) h on the dual.
    const double R = 6.0 * src.sigma * n;
    for (int from = 0; from < 2; ++from) {
        const double off = from ? 1.0 : 0.5;
        for (int x = 0; x < 3; ++x) {
            const double S = d.x[x] * n;
            const double a = std::floor(S - R - off) - 1.0, b = std::ceil(S + R - off) + 1.0;
            if (b - a + 1.0 >= (double)n) {
                d.box[from][x] = 0;
                d.box[from][3 + x] = (uint32_t)n;
            } else {
                long long i0 = (long long)a % n;
                if (i0 < 0) i0 += n;
                d.box[from][x] = (uint32_t)i0;
                d.box[from][3 + x] = (uint32_t)(b - a + 1.0);
            }
        }
    }
    return d;
}

}  // namespace hermite
