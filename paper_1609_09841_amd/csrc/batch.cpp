// Batches of independent shots (declared in include/hermite.h).
//
// Every shot owns a primal and a dual grid (layout of the single-grid
// context). Shots of one order m form a group that one batched kernel
// launch covers per half step (batch_common.h); the operator of a group
// depends on m and lam = cfl/2 only, so one table serves all its shots. The
// point sources of all shots are one more launch per half step, after the
// groups, and one clock-advance launch per full step.
//
// A full step is captured once into a HIP graph: the groups of each half
// step on parallel branches (forked from and joined to the capture stream),
// then the sources, then the clock. hermite_batch_step replays it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "batch_common.h"
#include "constants.h"
#include "hermite.h"
#include "host_common.h"
#include "kernels.h"

namespace {

constexpr int kMaxShots = 4096;

struct Group {
    int m = 0;
    std::vector<uint32_t> ids;     // shot indices
    std::vector<uint32_t> prefix;  // work items before each entry, per candidate-independent unit
    uint32_t* d_ids = nullptr;
    uint32_t* d_prefix[3] = {nullptr, nullptr, nullptr};  // m < 3: per block size candidate; m = 3: [0]
    uint32_t blocks[3] = {0, 0, 0};                       // m < 3: total blocks per candidate
    void* K = nullptr;                                    // operator in the kernel's layout
    int choice = 0;                                       // tuned candidate
    double ms = 0.0;                                      // its half-step time
};

constexpr int kSmallBlocks[3] = {64, 128, 256};
constexpr uint32_t kChunk[4] = {1, 4, 1, 4};
constexpr uint32_t kInterleaved[4] = {0, 0, 1, 1};

}  // namespace

struct hermite_batch {
    int n_shots = 0;
    double cfl = 0, c = 0;
    hermite_batch_options opt{};
    int q[4] = {0, 0, 0, 0};  // Taylor stages per m
    int substeps = 1;
    int device = 0, cus = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap[3] = {nullptr, nullptr, nullptr};  // capture streams (main + 2 branches)
    hipEvent_t ev[8] = {};
    std::vector<hermite_shot> shots;
    std::vector<hermite::batch::ShotGrid> grids;  // host copy of the shot table
    std::vector<long long> steps;                 // full steps per shot (host mirror)
    hermite::batch::ShotGrid* d_grids = nullptr;
    Group groups[3];                              // m = 1, 2, 3
    // sources
    std::vector<int> src_entry;                   // entry of each shot, -1 without
    std::vector<hermite::SourceDesc> srcs;        // sorted by order m
    hermite::SourceDesc* d_srcs = nullptr;
    uint32_t* d_src_prefix = nullptr;             // per order and half step: ns_m + 1 block offsets
    double* d_src_scal = nullptr;                 // 20 doubles per source: the half step's scalars
    uint32_t src_first[3] = {0, 0, 0}, src_count[3] = {0, 0, 0};  // entries of order m = 1, 2, 3
    size_t src_prefix_off[3][2] = {};
    uint32_t src_blocks[3][2] = {};
    // graph of one full step
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string err;
};

namespace {

thread_local std::string g_batch_err;

int bfail(hermite_batch* b, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    else g_batch_err = buf;
    return code;
}

int bhip(hermite_batch* b, hipError_t e, const char* what) {
    (void)hipGetLastError();  // clear the thread's last error (see capi.cpp)
    return bfail(b, (e == hipErrorOutOfMemory) ? HERMITE_ENOMEM : HERMITE_EDEVICE, "%s: %s (%d)", what,
                 hipGetErrorString(e), (int)e);
}

#define BCHECK(b, expr, what)                               \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return bhip(b, e_, what);     \
    } while (0)

void free_batch(hermite_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto& g : b->grids)
        for (double*& p : g.grid)
            if (p) { (void)hipFree(p); p = nullptr; }
    if (b->d_grids) (void)hipFree(b->d_grids);
    for (Group& g : b->groups) {
        if (g.d_ids) (void)hipFree(g.d_ids);
        for (uint32_t*& p : g.d_prefix)
            if (p) { (void)hipFree(p); p = nullptr; }
        if (g.K) (void)hipFree(g.K);
    }
    if (b->d_srcs) (void)hipFree(b->d_srcs);
    if (b->d_src_prefix) (void)hipFree(b->d_src_prefix);
    if (b->d_src_scal) (void)hipFree(b->d_src_scal);
    for (hipEvent_t& e : b->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t& s : b->cap)
        if (s) (void)hipStreamDestroy(s);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

int persistent_grid(const hermite_batch* b) { return b->cus >= 8 ? (b->cus / 8) * 8 : 8; }

// One half step of group g with candidate `choice`.
hipError_t launch_group(const hermite_batch* b, const Group& g, int choice, int from, hipStream_t st) {
    const uint32_t ng = (uint32_t)g.ids.size();
    if (g.m < 3)
        return hermite::launch_fused_valu_small_batch(g.m, kSmallBlocks[choice], b->d_grids, g.d_ids,
                                                      g.d_prefix[choice], ng, g.blocks[choice], from,
                                                      (const double*)g.K, st);
    if (b->opt.precision != HERMITE_PREC_FP64)
        return hermite::launch_fused_mixed_batch(b->opt.precision, b->d_grids, g.d_ids, g.d_prefix[0], ng, from, g.K,
                                                 persistent_grid(b), kChunk[choice], kInterleaved[choice], st);
    return hermite::launch_fused_mfma_batch(b->d_grids, g.d_ids, g.d_prefix[0], ng, from, (const double*)g.K,
                                            persistent_grid(b), kChunk[choice], kInterleaved[choice], st);
}

int n_candidates(int m) { return m < 3 ? 3 : 4; }

// Enqueues one full step. With `branches`, groups of a half step run on the
// capture streams forked from st (graph capture); otherwise in order on st.
int enqueue_full_step(hermite_batch* b, hipStream_t st, bool branches) {
    const uint32_t ns = (uint32_t)b->srcs.size();
    for (int from = 0; from < 2; ++from) {
        std::vector<const Group*> act;
        for (const Group& g : b->groups)
            if (!g.ids.empty()) act.push_back(&g);
        if (branches && act.size() > 1) {
            hipEvent_t* ev = b->ev + 3 * from;  // fork, then one join per branch
            BCHECK(b, hipEventRecord(ev[0], st), "fork");
            for (size_t i = 1; i < act.size(); ++i) BCHECK(b, hipStreamWaitEvent(b->cap[i], ev[0], 0), "fork");
            for (size_t i = 0; i < act.size(); ++i) {
                hipStream_t s = i ? b->cap[i] : st;
                BCHECK(b, launch_group(b, *act[i], act[i]->choice, from, s), "batched half step");
            }
            for (size_t i = 1; i < act.size(); ++i) {
                BCHECK(b, hipEventRecord(ev[i], b->cap[i]), "join");
                BCHECK(b, hipStreamWaitEvent(st, ev[i], 0), "join");
            }
        } else {
            for (const Group* g : act) BCHECK(b, launch_group(b, *g, g->choice, from, st), "batched half step");
        }
        for (int g = 0; g < 3; ++g)
            if (b->src_count[g])
                BCHECK(b, hermite::launch_source(b->d_srcs + b->src_first[g], b->d_src_prefix + b->src_prefix_off[g][from],
                                                 b->src_count[g], b->src_blocks[g][from], g + 1, from, -1,
                                                 b->d_src_scal + 20 * (size_t)b->src_first[g], st),
                       "source launch");
    }
    if (ns) BCHECK(b, hermite::launch_advance_clock(b->d_srcs, ns, st), "clock launch");
    return HERMITE_OK;
}

int capture_graph(hermite_batch* b) {
    hipStream_t st = b->cap[0];
    BCHECK(b, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    const int rc = enqueue_full_step(b, st, true);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != HERMITE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return bhip(b, e, "hipStreamEndCapture");
    b->graph = g;
    BCHECK(b, hipGraphInstantiateWithFlags(&b->exec, g, 0), "hipGraphInstantiate");
    return HERMITE_OK;
}

// Times every candidate of every group on half steps primal -> dual (they
// write only the dual grids, which hold no state between full steps).
int autotune(hermite_batch* b) {
    hipEvent_t t0 = b->ev[6], t1 = b->ev[7];
    for (Group& g : b->groups) {
        if (g.ids.empty()) continue;
        double best = 1e300;
        for (int cnd = 0; cnd < n_candidates(g.m); ++cnd) {
            BCHECK(b, launch_group(b, g, cnd, 0, b->stream), "autotune warm-up");
            constexpr int kReps = 3;
            BCHECK(b, hipEventRecord(t0, b->stream), "autotune");
            for (int r = 0; r < kReps; ++r) BCHECK(b, launch_group(b, g, cnd, 0, b->stream), "autotune");
            BCHECK(b, hipEventRecord(t1, b->stream), "autotune");
            BCHECK(b, hipEventSynchronize(t1), "autotune");
            float ms = 0.f;
            BCHECK(b, hipEventElapsedTime(&ms, t0, t1), "autotune");
            const double per = ms / kReps;
            if (per < best) {
                best = per;
                g.choice = cnd;
            }
        }
        g.ms = best;
    }
    return HERMITE_OK;
}

template <class T>
int upload(hermite_batch* b, T** dptr, const std::vector<T>& v, const char* what) {
    BCHECK(b, hipMalloc((void**)dptr, std::max<size_t>(1, v.size()) * sizeof(T)), what);
    if (!v.empty()) BCHECK(b, hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), what);
    return HERMITE_OK;
}

int check_shot(hermite_batch* b, int shot) {
    if (!b) return bfail(nullptr, HERMITE_EINVAL, "batch is NULL");
    if (shot < 0 || shot >= b->n_shots) return bfail(b, HERMITE_EINVAL, "shot=%d outside [0, %d)", shot, b->n_shots);
    (void)hipGetLastError();
    BCHECK(b, hipSetDevice(b->device), "hipSetDevice");
    return HERMITE_OK;
}

}  // namespace

extern "C" {

void hermite_batch_default_options(hermite_batch_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = HERMITE_PREC_FP64;
    opt->evolution = HERMITE_EVOLVE_TAYLOR;
    opt->rk_substeps = 1;
    opt->graph = 1;
    opt->autotune = 1;
}

int hermite_batch_create(int n_shots, const hermite_shot* shots, double cfl, double c,
                         const hermite_batch_options* opt, hermite_batch** out) {
    g_batch_err.clear();
    if (!out) return bfail(nullptr, HERMITE_EINVAL, "out is NULL");
    if (!shots) return bfail(nullptr, HERMITE_EINVAL, "shots is NULL");
    if (n_shots < 1 || n_shots > kMaxShots)
        return bfail(nullptr, HERMITE_EINVAL, "n_shots=%d outside [1, %d]", n_shots, kMaxShots);
    if (!std::isfinite(cfl) || !(cfl > 0.0) || cfl > 1.0)
        return bfail(nullptr, HERMITE_EINVAL, "cfl=%g outside (0, 1]", cfl);
    if (!std::isfinite(c) || !(c > 0.0)) return bfail(nullptr, HERMITE_EINVAL, "c=%g must be finite and > 0", c);
    hermite_batch_options o;
    hermite_batch_default_options(&o);
    if (opt) o = *opt;
    if (o.precision < 0 || o.precision > 2) return bfail(nullptr, HERMITE_EINVAL, "precision=%d", o.precision);
    if (o.evolution != 0 && o.evolution != 1) return bfail(nullptr, HERMITE_EINVAL, "evolution=%d", o.evolution);
    if (o.rk_substeps < 0 || o.rk_substeps > 64)
        return bfail(nullptr, HERMITE_EINVAL, "rk_substeps=%d", o.rk_substeps);
    if (o.q < 0 || o.q > 64) return bfail(nullptr, HERMITE_EINVAL, "q=%d outside [0, 64]", o.q);
    if (o.graph != 0 && o.graph != 1) return bfail(nullptr, HERMITE_EINVAL, "graph=%d", o.graph);
    if (o.autotune != 0 && o.autotune != 1) return bfail(nullptr, HERMITE_EINVAL, "autotune=%d", o.autotune);
    for (int s = 0; s < n_shots; ++s) {
        const hermite_shot& sh = shots[s];
        if (sh.n_cells < 2 || sh.n_cells > 1290)
            return bfail(nullptr, HERMITE_EINVAL, "shot %d: n_cells=%d outside [2, 1290]", s, sh.n_cells);
        if (sh.m < 1 || sh.m > 3) return bfail(nullptr, HERMITE_EINVAL, "shot %d: m=%d outside [1, 3]", s, sh.m);
        if (sh.has_source != 0 && sh.has_source != 1)
            return bfail(nullptr, HERMITE_EINVAL, "shot %d: has_source=%d", s, sh.has_source);
        if (sh.has_source) {
            const std::string why = hermite::check_source(sh.source);
            if (!why.empty()) return bfail(nullptr, HERMITE_EINVAL, "shot %d: %s", s, why.c_str());
            if (o.evolution != HERMITE_EVOLVE_TAYLOR)
                return bfail(nullptr, HERMITE_EUNSUPPORTED, "shot %d: the point source needs Taylor evolution", s);
        }
    }

    hermite_batch* b = new (std::nothrow) hermite_batch();
    if (!b) return bfail(nullptr, HERMITE_ENOMEM, "host allocation failed");
    b->n_shots = n_shots;
    b->cfl = cfl;
    b->c = c;
    b->opt = o;
    b->substeps = o.rk_substeps ? o.rk_substeps : 1;
    for (int m = 1; m <= 3; ++m) b->q[m] = o.q ? o.q : 6 * m + 1;
    b->shots.assign(shots, shots + n_shots);
    b->steps.assign(n_shots, 0);
    auto bail = [&](int code) {
        g_batch_err = b->err;
        free_batch(b);
        delete b;
        return code;
    };
    (void)hipGetLastError();  // start from a clean last-error state
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) return bail(bhip(b, e, "hipGetDevice"));
    if ((e = hipSetDevice(b->device)) != hipSuccess) return bail(bhip(b, e, "hipSetDevice"));
    if ((e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device)) != hipSuccess)
        return bail(bhip(b, e, "hipDeviceGetAttribute"));
    if (o.stream) {
        b->stream = (hipStream_t)o.stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess)
            return bail(bhip(b, e, "hipStreamCreate"));
        b->own_stream = true;
    }
    for (hipStream_t& s : b->cap)
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
            return bail(bhip(b, e, "hipStreamCreate"));
    for (int i = 0; i < 8; ++i) {
        const unsigned flags = (i < 6) ? hipEventDisableTiming : hipEventDefault;
        if ((e = hipEventCreateWithFlags(&b->ev[i], flags)) != hipSuccess) return bail(bhip(b, e, "hipEventCreate"));
    }

    // grids (zero data at t = 0)
    const double lam = cfl / 2.0;
    b->grids.resize(n_shots);
    for (int s = 0; s < n_shots; ++s) {
        const int n = shots[s].n_cells, M = shots[s].m + 1;
        hermite::batch::ShotGrid& g = b->grids[s];
        g.n = (uint32_t)n;
        g.m = (uint32_t)shots[s].m;
        g.pitch = hermite::column_pitch((size_t)n * n * n);
        const size_t bytes = (size_t)2 * M * M * M * g.pitch * sizeof(double);
        for (double*& p : g.grid) {
            if ((e = hipMalloc(&p, bytes)) != hipSuccess) return bail(bhip(b, e, "hipMalloc(grid)"));
            if ((e = hipMemsetAsync(p, 0, bytes, b->stream)) != hipSuccess) return bail(bhip(b, e, "zero grid"));
        }
    }
    if (upload(b, &b->d_grids, b->grids, "upload shot table") != HERMITE_OK) return bail(HERMITE_EDEVICE);

    // order groups and their operators
    for (int m = 1; m <= 3; ++m) {
        Group& g = b->groups[m - 1];
        g.m = m;
        for (int s = 0; s < n_shots; ++s)
            if (shots[s].m == m) g.ids.push_back((uint32_t)s);
        if (g.ids.empty()) continue;
        int rc = upload(b, &g.d_ids, g.ids, "upload group");
        if (rc) return bail(rc);
        const int ncand = (m < 3) ? 3 : 1;
        for (int cnd = 0; cnd < ncand; ++cnd) {
            std::vector<uint32_t> pre(1, 0);
            for (uint32_t s : g.ids) {
                const uint64_t n = shots[s].n_cells;
                // m = 3: the 16-cell batches of a z-adjacent row pair per
                // work item, in every precision (the kernels decode item
                // numbers below n ceil(n/2) ceil(n/16) only)
                const uint64_t items = (m < 3) ? (n * n * n + kSmallBlocks[cnd] - 1) / kSmallBlocks[cnd]
                                               : n * ((n + 1) / 2) * ((n + 15) / 16);
                if (pre.back() + items > 0xFFFFFFFFull)
                    return bail(bfail(b, HERMITE_EINVAL, "order-%d shots exceed 2^32 work items", m));
                pre.push_back(pre.back() + (uint32_t)items);
            }
            g.blocks[cnd] = pre.back();
            if (cnd == 0) g.prefix = pre;
            if ((rc = upload(b, &g.d_prefix[cnd], pre, "upload group")) != HERMITE_OK) return bail(rc);
        }
        const std::vector<double> cpoly = hermite::evolution_poly(m, o.evolution, b->q[m], b->substeps);
        const std::vector<double> K = hermite::fused_class_operators(m, lam, cpoly);
        std::vector<unsigned char> Kdev;
        if (m < 3) {
            Kdev.resize(hermite::valu_small_operator_doubles(m) * sizeof(double));
            if (!hermite::valu_small_build_operators(m, K.data(), (double*)Kdev.data()))
                return bail(bfail(b, HERMITE_EUNSUPPORTED, "class operator has a nonzero entry the kernel skips"));
        } else if (o.precision != HERMITE_PREC_FP64) {
            Kdev.resize(hermite::mixed_operator_bytes(o.precision));
            hermite::mixed_build_operators(o.precision, K.data(), Kdev.data());
        } else {
            Kdev.resize(hermite::mfma_operator_doubles() * sizeof(double));
            if (!hermite::mfma4_arrange_operators(K.data(), (double*)Kdev.data()))
                return bail(bfail(b, HERMITE_EUNSUPPORTED, "class operator has a nonzero entry the kernel skips"));
        }
        if ((rc = upload(b, (unsigned char**)&g.K, Kdev, "upload operator")) != HERMITE_OK) return bail(rc);
    }

    // sources, grouped by order (one source launch per order present)
    b->src_entry.assign(n_shots, -1);
    for (int m = 1; m <= 3; ++m) {
        b->src_first[m - 1] = (uint32_t)b->srcs.size();
        for (int s = 0; s < n_shots; ++s) {
            if (shots[s].m != m || !shots[s].has_source || shots[s].source.amplitude == 0.0) continue;
            hermite::SourceDesc d = hermite::make_source_desc(shots[s].source, shots[s].n_cells, m, b->q[m], cfl, c);
            d.grid[0] = b->grids[s].grid[0];
            d.grid[1] = b->grids[s].grid[1];
            d.pitch = b->grids[s].pitch;
            d.steps = 0;
            b->src_entry[s] = (int)b->srcs.size();
            b->srcs.push_back(d);
        }
        b->src_count[m - 1] = (uint32_t)b->srcs.size() - b->src_first[m - 1];
    }
    if (!b->srcs.empty()) {
        std::vector<uint32_t> pre;
        for (int g = 0; g < 3; ++g)
            for (int from = 0; from < 2; ++from) {
                b->src_prefix_off[g][from] = pre.size();
                pre.push_back(0);
                for (uint32_t i = 0; i < b->src_count[g]; ++i) {
                    const uint64_t next =
                        (uint64_t)pre.back() + hermite::source_blocks(b->srcs[b->src_first[g] + i], from);
                    if (next > 0x7FFFFFFFull) return bail(bfail(b, HERMITE_EINVAL, "sources exceed 2^31 blocks"));
                    pre.push_back((uint32_t)next);
                }
                b->src_blocks[g][from] = pre.back();
            }
        int rc = upload(b, &b->d_srcs, b->srcs, "upload sources");
        if (rc == HERMITE_OK) rc = upload(b, &b->d_src_prefix, pre, "upload sources");
        if (rc == HERMITE_OK) rc = upload(b, &b->d_src_scal, std::vector<double>(20 * b->srcs.size(), 0.0),
                                          "allocate source scalars");
        if (rc) return bail(rc);
    }

    if (o.autotune) {
        const int rc = autotune(b);
        if (rc) return bail(rc);
    }
    if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return bail(bhip(b, e, "create"));
    *out = b;
    return HERMITE_OK;
}

int hermite_batch_set_initial(hermite_batch* b, int shot, const double* u, const double* ut) {
    int rc = check_shot(b, shot);
    if (rc) return rc;
    if ((u == nullptr) != (ut == nullptr)) return bfail(b, HERMITE_EINVAL, "u and ut must both be given or both NULL");
    const hermite::batch::ShotGrid& g = b->grids[shot];
    const size_t M3 = (size_t)(g.m + 1) * (g.m + 1) * (g.m + 1), ncell = (size_t)g.n * g.n * g.n;
    const size_t w = ncell * sizeof(double), dp = g.pitch * sizeof(double);
    const double h = 1.0 / g.n;
    BCHECK(b, hipStreamSynchronize(b->stream), "sync before set_initial");
    double* gu = g.grid[0];
    double* gv = gu + M3 * g.pitch;
    if (u) {
        BCHECK(b, hipMemcpy2D(gu, dp, u, w, w, M3, hipMemcpyHostToDevice), "copy u");
        BCHECK(b, hipMemcpy2D(gv, dp, ut, w, w, M3, hipMemcpyHostToDevice), "copy ut");
        BCHECK(b, hermite::launch_scale(gv, g.pitch, gv, g.pitch, h / b->c, ncell, (int)M3, b->stream), "scale ut");
    } else {
        BCHECK(b, hipMemsetAsync(gu, 0, 2 * M3 * g.pitch * sizeof(double), b->stream), "zero grid");
    }
    const int e = b->src_entry[shot];
    if (e >= 0) {
        const int64_t zero = 0;
        BCHECK(b, hipMemcpyAsync((char*)(b->d_srcs + e) + offsetof(hermite::SourceDesc, steps), &zero, sizeof(zero),
                                 hipMemcpyHostToDevice, b->stream),
               "reset clock");
    }
    BCHECK(b, hipStreamSynchronize(b->stream), "set_initial");
    b->steps[shot] = 0;
    return HERMITE_OK;
}

int hermite_batch_step(hermite_batch* b, int n_full_steps) {
    if (!b) return bfail(nullptr, HERMITE_EINVAL, "batch is NULL");
    if (n_full_steps < 0) return bfail(b, HERMITE_EINVAL, "n_full_steps=%d < 0", n_full_steps);
    (void)hipGetLastError();
    BCHECK(b, hipSetDevice(b->device), "hipSetDevice");
    if (n_full_steps == 0) return HERMITE_OK;
    if (b->opt.graph) {
        if (!b->exec) {
            const int rc = capture_graph(b);
            if (rc) return rc;
        }
        for (int s = 0; s < n_full_steps; ++s) BCHECK(b, hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
    } else {
        for (int s = 0; s < n_full_steps; ++s) {
            const int rc = enqueue_full_step(b, b->stream, false);
            if (rc) return rc;
        }
    }
    for (long long& st : b->steps) st += n_full_steps;
    return HERMITE_OK;
}

int hermite_batch_gather(hermite_batch* b, int shot, double* u, double* ut, double* t_out) {
    int rc = check_shot(b, shot);
    if (rc) return rc;
    const hermite::batch::ShotGrid& g = b->grids[shot];
    const size_t M3 = (size_t)(g.m + 1) * (g.m + 1) * (g.m + 1), ncell = (size_t)g.n * g.n * g.n;
    const size_t w = ncell * sizeof(double), sp = g.pitch * sizeof(double);
    const double h = 1.0 / g.n;
    BCHECK(b, hipStreamSynchronize(b->stream), "sync before gather (an earlier kernel failed)");
    if (u) BCHECK(b, hipMemcpy2D(u, w, g.grid[0], sp, w, M3, hipMemcpyDeviceToHost), "copy u");
    if (ut) {
        // the dual grid holds no state between full steps: staging for c/h
        double* tmp = g.grid[1];
        BCHECK(b, hermite::launch_scale(tmp, g.pitch, g.grid[0] + M3 * g.pitch, g.pitch, b->c / h, ncell, (int)M3,
                                        b->stream),
               "scale ut");
        BCHECK(b, hipStreamSynchronize(b->stream), "gather scale");
        BCHECK(b, hipMemcpy2D(ut, w, tmp, sp, w, M3, hipMemcpyDeviceToHost), "copy ut");
    }
    if (t_out) *t_out = (double)b->steps[shot] * (b->cfl * h / b->c);
    return HERMITE_OK;
}

int hermite_batch_sync(hermite_batch* b) {
    if (!b) return bfail(nullptr, HERMITE_EINVAL, "batch is NULL");
    BCHECK(b, hipSetDevice(b->device), "hipSetDevice");
    BCHECK(b, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    return HERMITE_OK;
}

int hermite_batch_tuning(const hermite_batch* b, int m, int* choice, double* ms) {
    if (!b) return bfail(nullptr, HERMITE_EINVAL, "batch is NULL");
    if (m < 1 || m > 3 || b->groups[m - 1].ids.empty())
        return bfail(const_cast<hermite_batch*>(b), HERMITE_EINVAL, "the batch has no shot of order m=%d", m);
    if (choice) *choice = b->groups[m - 1].choice;
    if (ms) *ms = b->groups[m - 1].ms;
    return HERMITE_OK;
}

void hermite_batch_destroy(hermite_batch* b) {
    if (!b) return;
    if (hipSetDevice(b->device) == hipSuccess && b->stream) (void)hipStreamSynchronize(b->stream);
    free_batch(b);
    delete b;
}

const char* hermite_batch_last_error(const hermite_batch* b) { return b ? b->err.c_str() : g_batch_err.c_str(); }

}  // extern "C"
