// Input-column schedule of the matrix-core (MFMA FP64 16x16x4) fused half
// step for m = 3. Shared by the kernel and the host code that lays out the
// operator tables for it.
#pragma once

namespace hermite {

// 128 inputs per parity class (2 fields x 64 derivative multi-indices d) are
// fed as 32 chunks of 4 (one MFMA K-step each). Every chunk holds 4 columns
// with the same parity pattern of d (bit x = d_x mod 2), so which butterfly
// output feeds which class is fixed per chunk. Chunks follow the small-first
// accumulation order (|d| descending, field v before u, flat index ascending),
// each chunk filled greedily with the next columns of its group: the same
// parity pattern and the same answers to d1 = 0 and d2 = 0. The last two keep
// the columns with d_x = 0 together, so that more 4x4 row tiles of the class
// operators are zero for every operator (124 of 1,024 rather than 36: an
// entry vanishes when on some axis p_x = 0, o_x = 1 and d_x = 0, and a row
// tile fixes o1 and o2); every group has a multiple of 4 columns.
struct MfmaSchedule {
    static constexpr int M = 4, M3 = 64, NC = 128, NSTEP = 32;
    int col[NSTEP][4];  // column f*64 + (d3*4 + d2)*4 + d1
    int dpar[NSTEP];    // parity pattern of the chunk's d
    constexpr MfmaSchedule() : col(), dpar() {
        int order[NC] = {};
        int k = 0;
        for (int s = 3 * (M - 1); s >= 0; --s)
            for (int f = 1; f >= 0; --f)
                for (int d3 = 0; d3 < M; ++d3)
                    for (int d2 = 0; d2 < M; ++d2) {
                        const int d1 = s - d3 - d2;
                        if (d1 < 0 || d1 >= M) continue;
                        order[k++] = f * M3 + (d3 * M + d2) * M + d1;
                    }
        bool used[NC] = {};
        int t = 0;
        for (int a = 0; a < NC; ++a) {
            const int c0 = order[a];
            if (used[c0]) continue;
            const int grp = group(c0);
            int got = 0;
            for (int b = a; b < NC && got < 4; ++b) {
                const int cb = order[b];
                if (!used[cb] && group(cb) == grp) {
                    col[t][got++] = cb;
                    used[cb] = true;
                }
            }
            dpar[t] = parity(c0);
            ++t;
        }
    }
    static constexpr int parity(int column) {
        const int dd = column % M3;
        const int d1 = dd % M, d2 = (dd / M) % M, d3 = dd / (M * M);
        return (d1 & 1) | ((d2 & 1) << 1) | ((d3 & 1) << 2);
    }
    static constexpr int group(int column) {
        const int dd = column % M3;
        return parity(column) | ((dd % M == 0) << 3) | (((dd / M) % M == 0) << 4);
    }
};

}  // namespace hermite
