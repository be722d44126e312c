// One z-slab of a periodic grid sharded over devices (hermite_slab_*): the
// fused m = 3 FP64 half step (Sec. 3.3) on the matrix cores, over the slab's
// own cell planes, with the one plane each half step reads from a neighbour
// held as a halo plane that the caller fills. A half step can run in two
// parts: the cells that do not read the halo (all but one cell plane), which
// may overlap the halo's exchange, then the one plane that does.
//
// Buffers: each grid holds nz + 1 node planes per column (column pitch as the
// cube's grids). Primal: planes 0 .. nz-1 = own planes z0 .. z0+nz-1, plane nz
// = halo z0+nz. Dual: plane 0 = halo z0-1, planes 1 .. nz = own planes z0 ..
// z0+nz-1. The primal -> dual half step (cell lower corners on primal planes
// k, corners k and k+1) writes dual plane k+1; the dual -> primal one (lower
// corners on dual buffer planes k, that is global planes z0-1+k) writes
// primal plane k with the x, y shift of Sec. 2's alternation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "hermite.h"
#include "constants.h"
#include "host_common.h"
#include "kernels.h"

struct hermite_slab {
    int n = 0, nz = 0, m = 3, M3 = 64;
    double cfl = 0, c = 0, h = 0, dt = 0, lam = 0;
    int q = 0, substeps = 1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0, grid_blocks = 8;
    double* grid[2] = {nullptr, nullptr};  // primal, dual: 2 M^3 columns of `pitch` doubles
    size_t plane = 0;                      // n^2 nodes per plane
    size_t pitch = 0;
    void* K = nullptr;                     // class operators, 16x16-tile layout (the boundary plane)
    void* K4 = nullptr;                    // the same, 4x4-tile layout (interior and whole half steps)
    uint32_t* queue = nullptr;             // item counters of the 4x4-tile kernel (zero between launches)
    bool has_state = false;
    long long half_steps = 0;
    bool interior_done = false;            // the current half step's interior cells are enqueued
    std::string err;
};

namespace {

thread_local std::string g_slab_err;

int sfail(hermite_slab* s, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    else g_slab_err = buf;
    return code;
}

int shipfail(hermite_slab* s, hipError_t e, const char* what) {
    (void)hipGetLastError();  // do not let the runtime report it again
    return sfail(s, (e == hipErrorOutOfMemory) ? HERMITE_ENOMEM : HERMITE_EDEVICE, "%s: %s (%d)", what,
                 hipGetErrorString(e), (int)e);
}

#define SCHECK(s, expr, what)                                \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return shipfail(s, e_, what);  \
    } while (0)

void free_slab(hermite_slab* s) {
    for (double*& g : s->grid)
        if (g) { (void)hipFree(g); g = nullptr; }
    if (s->K) { (void)hipFree(s->K); s->K = nullptr; }
    if (s->K4) { (void)hipFree(s->K4); s->K4 = nullptr; }
    if (s->queue) { (void)hipFree(s->queue); s->queue = nullptr; }
    if (s->own_stream && s->stream) { (void)hipStreamDestroy(s->stream); s->stream = nullptr; }
}

int slab_device(hermite_slab* s) {
    (void)hipGetLastError();
    SCHECK(s, hipSetDevice(s->device), "hipSetDevice");
    return HERMITE_OK;
}

}  // namespace

extern "C" {

int hermite_slab_create(int n_cells, int nz, int m, double cfl, double c, const hermite_options* opt,
                        hermite_slab** out) {
    g_slab_err.clear();
    if (!out) return sfail(nullptr, HERMITE_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_cells < 2 || n_cells > 1290) return sfail(nullptr, HERMITE_EINVAL, "n_cells=%d outside [2, 1290]", n_cells);
    if (nz < 1 || (double)n_cells * n_cells * ((double)nz + 1) >= 2147483648.0)
        return sfail(nullptr, HERMITE_EINVAL, "nz=%d: need 1 <= nz and n_cells^2 (nz+1) < 2^31", nz);
    if (m < 1 || m > 3) return sfail(nullptr, HERMITE_EINVAL, "m=%d outside [1, 3]", m);
    if (!std::isfinite(cfl) || !(cfl > 0.0) || cfl > 1.0)
        return sfail(nullptr, HERMITE_EINVAL, "cfl=%g outside (0, 1]", cfl);
    if (!std::isfinite(c) || !(c > 0.0)) return sfail(nullptr, HERMITE_EINVAL, "c=%g must be finite and > 0", c);
    hermite_options o;
    hermite_default_options(&o);
    if (opt) o = *opt;
    if (o.evolution != HERMITE_EVOLVE_TAYLOR && o.evolution != HERMITE_EVOLVE_RK4)
        return sfail(nullptr, HERMITE_EINVAL, "evolution=%d", o.evolution);
    if (o.rk_substeps < 0 || o.rk_substeps > 64) return sfail(nullptr, HERMITE_EINVAL, "rk_substeps=%d", o.rk_substeps);
    if (o.q < 0 || o.q > 64) return sfail(nullptr, HERMITE_EINVAL, "q=%d outside [0, 64]", o.q);
    if (m != 3 || o.precision != HERMITE_PREC_FP64 || o.fused != 1 || o.equation != HERMITE_EQ_WAVE ||
        o.kernel == HERMITE_KERNEL_VALU || o.poison)
        return sfail(nullptr, HERMITE_EUNSUPPORTED,
                     "slabs run the fused m = 3 FP64 wave half step on the matrix cores only "
                     "(m=%d precision=%d fused=%d equation=%d kernel=%d poison=%d)",
                     m, o.precision, o.fused, o.equation, o.kernel, o.poison);

    hermite_slab* s = new (std::nothrow) hermite_slab();
    if (!s) return sfail(nullptr, HERMITE_ENOMEM, "host allocation failed");
    s->n = n_cells;
    s->nz = nz;
    s->m = m;
    s->M3 = (m + 1) * (m + 1) * (m + 1);
    s->cfl = cfl;
    s->c = c;
    s->h = 1.0 / n_cells;
    s->dt = cfl * s->h / c;
    s->lam = c * 0.5 * s->dt / s->h;
    s->q = o.q ? o.q : 6 * m + 1;
    s->substeps = o.rk_substeps ? o.rk_substeps : 1;
    s->plane = (size_t)n_cells * n_cells;
    s->pitch = hermite::column_pitch(s->plane * (nz + 1));
    auto bail = [&](int code) {
        g_slab_err = s->err;
        free_slab(s);
        delete s;
        return code;
    };
    (void)hipGetLastError();
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) return bail(shipfail(s, e, "hipGetDevice"));
    int rc = slab_device(s);
    if (rc) return bail(rc);
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device);
    if (e != hipSuccess) return bail(shipfail(s, e, "hipDeviceGetAttribute"));
    s->grid_blocks = cus >= 8 ? (cus / 8) * 8 : 8;
    if (o.stream) {
        s->stream = (hipStream_t)o.stream;
    } else {
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(shipfail(s, e, "hipStreamCreate"));
        s->own_stream = true;
    }
    const size_t grid_bytes = (size_t)2 * s->M3 * s->pitch * sizeof(double);
    for (double*& g : s->grid) {
        e = hipMalloc(&g, grid_bytes);
        if (e != hipSuccess) return bail(shipfail(s, e, "hipMalloc(slab grid)"));
        e = hipMemset(g, 0, grid_bytes);
        if (e != hipSuccess) return bail(shipfail(s, e, "hipMemset(slab grid)"));
    }
    const std::vector<double> cpoly = hermite::evolution_poly(m, o.evolution, s->q, s->substeps);
    const std::vector<double> K = hermite::fused_class_operators(m, s->lam, cpoly);
    std::vector<double> Kperm(hermite::mfma_operator_doubles());
    hermite::mfma_permute_operators(K.data(), Kperm.data());
    e = hipMalloc(&s->K, Kperm.size() * sizeof(double));
    if (e != hipSuccess) return bail(shipfail(s, e, "hipMalloc(K)"));
    e = hipMemcpy(s->K, Kperm.data(), Kperm.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(shipfail(s, e, "upload K"));
    std::vector<double> K4(hermite::mfma_operator_doubles());
    if (!hermite::mfma4_arrange_operators(K.data(), K4.data()))
        return bail(sfail(s, HERMITE_EUNSUPPORTED, "class operator has a nonzero entry the kernel skips"));
    e = hipMalloc(&s->K4, K4.size() * sizeof(double));
    if (e != hipSuccess) return bail(shipfail(s, e, "hipMalloc(K4)"));
    e = hipMemcpy(s->K4, K4.data(), K4.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(shipfail(s, e, "upload K4"));
    const std::vector<uint32_t> zero(hermite::kMfma4QueueWords, 0u);
    e = hipMalloc(&s->queue, zero.size() * sizeof(uint32_t));
    if (e != hipSuccess) return bail(shipfail(s, e, "hipMalloc(queue)"));
    e = hipMemcpy(s->queue, zero.data(), zero.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(shipfail(s, e, "clear queue"));
    *out = s;
    return HERMITE_OK;
}

int hermite_slab_set_initial(hermite_slab* s, const double* u, const double* ut) {
    if (!s) return sfail(nullptr, HERMITE_EINVAL, "slab is NULL");
    if (!u || !ut) return sfail(s, HERMITE_EINVAL, "u or ut is NULL");
    int rc = slab_device(s);
    if (rc) return rc;
    const size_t rows = (size_t)s->M3, own = s->plane * s->nz, w = own * sizeof(double), dp = s->pitch * sizeof(double);
    double* g = s->grid[0];
    double* gv = g + rows * s->pitch;
    SCHECK(s, hipStreamSynchronize(s->stream), "sync before set_initial");
    SCHECK(s, hipMemcpy2D(g, dp, u, w, w, rows, hipMemcpyHostToDevice), "copy u");
    SCHECK(s, hipMemcpy2D(gv, dp, ut, w, w, rows, hipMemcpyHostToDevice), "copy ut");
    // internal velocity variable (h/c) u_t
    SCHECK(s, hermite::launch_scale(gv, s->pitch, gv, s->pitch, s->h / s->c, own, s->M3, s->stream), "scale ut");
    SCHECK(s, hipStreamSynchronize(s->stream), "set_initial");
    s->has_state = true;
    s->half_steps = 0;
    s->interior_done = false;
    return HERMITE_OK;
}

int hermite_slab_plane(hermite_slab* s, int which, void** dev, size_t* pitch_bytes) {
    if (!s) return sfail(nullptr, HERMITE_EINVAL, "slab is NULL");
    if (!dev) return sfail(s, HERMITE_EINVAL, "dev is NULL");
    double* p = nullptr;
    switch (which) {
        case HERMITE_SLAB_PRIMAL_FIRST: p = s->grid[0]; break;
        case HERMITE_SLAB_PRIMAL_HALO: p = s->grid[0] + s->plane * s->nz; break;
        case HERMITE_SLAB_DUAL_LAST: p = s->grid[1] + s->plane * s->nz; break;
        case HERMITE_SLAB_DUAL_HALO: p = s->grid[1]; break;
        default: return sfail(s, HERMITE_EINVAL, "which=%d is not a HERMITE_SLAB_* plane", which);
    }
    *dev = p;
    if (pitch_bytes) *pitch_bytes = s->pitch * sizeof(double);
    return HERMITE_OK;
}

int hermite_slab_half_step_part(hermite_slab* s, int part, int* next_halo) {
    if (!s) return sfail(nullptr, HERMITE_EINVAL, "slab is NULL");
    if (part != HERMITE_SLAB_INTERIOR && part != HERMITE_SLAB_BOUNDARY && part != HERMITE_SLAB_ALL)
        return sfail(s, HERMITE_EINVAL, "part=%d is not HERMITE_SLAB_INTERIOR, _BOUNDARY or _ALL", part);
    if (!s->has_state) return sfail(s, HERMITE_ESTATE, "slab half step before hermite_slab_set_initial");
    if (part == HERMITE_SLAB_BOUNDARY && !s->interior_done)
        return sfail(s, HERMITE_ESTATE, "HERMITE_SLAB_BOUNDARY before the half step's HERMITE_SLAB_INTERIOR");
    if (part != HERMITE_SLAB_BOUNDARY && s->interior_done)
        return sfail(s, HERMITE_ESTATE, "the half step's interior is enqueued: HERMITE_SLAB_BOUNDARY comes next");
    int rc = slab_device(s);
    if (rc) return rc;
    const int from = (int)(s->half_steps & 1);  // 0: primal -> dual
    // the one cell plane that reads the halo: the top one (primal halo above)
    // in the primal -> dual half step, the bottom one (dual halo below) after
    const int kb = from ? 0 : s->nz - 1;
    int k0 = 0, k1 = s->nz;
    if (part == HERMITE_SLAB_INTERIOR) {
        k0 = from ? 1 : 0;
        k1 = from ? s->nz : s->nz - 1;
    } else if (part == HERMITE_SLAB_BOUNDARY) {
        k0 = kb;
        k1 = kb + 1;
    }
    // several planes: two z-adjacent batches per wave (4x4 tiles); the single
    // boundary plane: one batch per wave (16x16 tiles), which a plane without
    // a partner does not leave half idle. Both give bit-identical results.
    if (part == HERMITE_SLAB_BOUNDARY)
        SCHECK(s,
               hermite::launch_fused_mfma_slab(s->grid[from], s->grid[1 - from], (const double*)s->K, s->n, k0, k1,
                                               s->pitch, from, s->grid_blocks, s->stream),
               "slab boundary-plane launch");
    else
        SCHECK(s,
               hermite::launch_fused_mfma4_slab(s->grid[from], s->grid[1 - from], (const double*)s->K4, s->n, k0,
                                                k1, s->pitch, from, s->grid_blocks, s->queue, s->stream),
               "slab half-step launch");
    if (part == HERMITE_SLAB_INTERIOR) {
        s->interior_done = true;
    } else {
        s->interior_done = false;
        ++s->half_steps;
    }
    if (next_halo)
        *next_halo = (part == HERMITE_SLAB_INTERIOR) ? (from ? HERMITE_SLAB_DUAL_HALO : HERMITE_SLAB_PRIMAL_HALO)
                     : (s->half_steps & 1)            ? HERMITE_SLAB_DUAL_HALO
                                                      : HERMITE_SLAB_PRIMAL_HALO;
    return HERMITE_OK;
}

int hermite_slab_half_step(hermite_slab* s, int* next_halo) {
    return hermite_slab_half_step_part(s, HERMITE_SLAB_ALL, next_halo);
}

int hermite_slab_gather(hermite_slab* s, double* u, double* ut, double* t_out) {
    if (!s) return sfail(nullptr, HERMITE_EINVAL, "slab is NULL");
    if (!s->has_state) return sfail(s, HERMITE_ESTATE, "hermite_slab_gather before hermite_slab_set_initial");
    if ((s->half_steps & 1) || s->interior_done)
        return sfail(s, HERMITE_ESTATE, "hermite_slab_gather inside a half step or after an odd number (%lld)",
                     s->half_steps);
    int rc = slab_device(s);
    if (rc) return rc;
    const size_t rows = (size_t)s->M3, own = s->plane * s->nz, w = own * sizeof(double), sp = s->pitch * sizeof(double);
    const double* g = s->grid[0];
    const double* gv = g + rows * s->pitch;
    SCHECK(s, hipStreamSynchronize(s->stream), "sync before gather (an earlier kernel failed)");
    if (u) SCHECK(s, hipMemcpy2D(u, w, g, sp, w, rows, hipMemcpyDeviceToHost), "copy u");
    if (ut) {
        // between full steps the dual grid is dead: stage the scaled velocity there
        double* tmp = s->grid[1];
        SCHECK(s, hermite::launch_scale(tmp, s->pitch, gv, s->pitch, s->c / s->h, own, s->M3, s->stream), "scale ut");
        SCHECK(s, hipStreamSynchronize(s->stream), "gather scale");
        SCHECK(s, hipMemcpy2D(ut, w, tmp, sp, w, rows, hipMemcpyDeviceToHost), "copy ut");
    }
    if (t_out) *t_out = (double)(s->half_steps / 2) * s->dt;
    return HERMITE_OK;
}

int hermite_slab_copy_plane(hermite_slab* dst, int dst_which, hermite_slab* src, int src_which, void* stream) {
    if (!dst || !src) return sfail(dst, HERMITE_EINVAL, "dst or src is NULL");
    if (dst->n != src->n || dst->M3 != src->M3)
        return sfail(dst, HERMITE_EINVAL, "slabs of different grids (n %d/%d, m %d/%d)", dst->n, src->n, dst->m, src->m);
    void *d = nullptr, *s = nullptr;
    size_t dp = 0, sp = 0;
    int rc = hermite_slab_plane(dst, dst_which, &d, &dp);
    if (rc) return rc;
    if ((rc = hermite_slab_plane(src, src_which, &s, &sp)) != HERMITE_OK) return sfail(dst, rc, "%s", src->err.c_str());
    if ((rc = slab_device(dst)) != HERMITE_OK) return rc;
    SCHECK(dst,
           hipMemcpy2DAsync(d, dp, s, sp, dst->plane * sizeof(double), (size_t)2 * dst->M3, hipMemcpyDefault,
                            stream ? (hipStream_t)stream : dst->stream),
           "plane copy");
    return HERMITE_OK;
}

int hermite_slab_sync(hermite_slab* s) {
    if (!s) return sfail(nullptr, HERMITE_EINVAL, "slab is NULL");
    int rc = slab_device(s);
    if (rc) return rc;
    SCHECK(s, hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    return HERMITE_OK;
}

void hermite_slab_destroy(hermite_slab* s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    free_slab(s);
    delete s;
}

const char* hermite_slab_last_error(const hermite_slab* s) { return s ? s->err.c_str() : g_slab_err.c_str(); }

}  // extern "C"
