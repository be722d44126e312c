// C ABI of the Hermite wave solver (declared in include/hermite.h).
//
// A context owns two FP64 two-field grids (primal, dual), the operator tables
// and, for the two-kernel variant, the reconstructed-coefficient scratch. One
// full step enqueues two half steps, primal -> dual and dual -> primal
// (Sec. 2), on the context's stream; nothing waits on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hermite.h"
#include "constants.h"
#include "host_common.h"
#include "kernels.h"

struct hermite_ctx {
    int n = 0, m = 0, M3 = 0;
    double cfl = 0, c = 0, h = 0, dt = 0, tau = 0, lam = 0;
    hermite_options opt{};
    int q = 0, substeps = 1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    int cus = 0;             // compute units of the device (persistent grids)
    int m3_kernel = 0;       // m = 3 fused FP64: 0 vector ALUs, 1 matrix cores (16x16), 2 matrix cores (4x4 tiles)
    int precision = 0;       // HERMITE_PREC_*: contraction arithmetic
    int nf = 2;              // fields per node: 2 (wave: u, u_t) or 1 (advection)
    std::vector<double> K1;  // advection: per-axis operator (M x 2M)
    std::vector<double> E1;  // advection, two kernels: per-axis translation (M x P)
    double* grid[2] = {nullptr, nullptr};  // primal, dual: 2 M^3 columns of `pitch` doubles each
    double* R = nullptr;                   // two-kernel scratch: 2 P^3 columns of `pitch` doubles
    size_t ncell = 0;                      // n^3 nodes per column
    size_t pitch = 0;                      // doubles between consecutive columns (>= ncell)
    void* K = nullptr;                     // fused class operators (layout of the kernel in use)
    uint32_t* queue = nullptr;             // item counters of the 4x4-tile kernel (zero between launches)
    double* Hp = nullptr;                  // parity blocks of H
    size_t grid_doubles = 0;
    bool has_state = false;
    long long steps = 0;
    bool has_source = false;
    hermite::SourceDesc* d_source = nullptr;  // one device entry
    uint32_t* d_source_prefix = nullptr;      // [from][2] block offsets
    double* d_source_scal = nullptr;          // the half step's source scalars
    uint32_t source_blocks[2] = {0, 0};
    hermite::SourceDesc source_desc{};        // host copy of the device entry
    long long series_len = 0;                 // amplitude series length (half steps), 0 = none
    uint32_t* d_rec = nullptr;                // receiver nodes (flat primal indices)
    uint32_t nrec = 0;
    void* Kadj = nullptr;                     // adjoint operator (canonical, or the m = 3 matrix-core layout)
    double* d_partial = nullptr;              // source-gradient block partials
    uint32_t partial_cap = 0;                 // doubles in d_partial
    bool adjoint = false;                     // grids hold an adjoint state
    long long adj_steps = 0;                  // the adjoint sweep's time, in full steps
    std::string err;
};

namespace {

thread_local std::string g_err;

int fail(hermite_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_err = buf;
    return code;
}

int hip_fail(hermite_ctx* ctx, hipError_t e, const char* what) {
    // the runtime keeps the error as the thread's last error: clear it, so
    // that a later launch check does not report it again
    (void)hipGetLastError();
    return fail(ctx, (e == hipErrorOutOfMemory) ? HERMITE_ENOMEM : HERMITE_EDEVICE, "%s: %s (%d)", what,
                hipGetErrorString(e), (int)e);
}

#define HCHECK(ctx, expr, what)                          \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

void free_all(hermite_ctx* ctx) {
    for (double*& g : ctx->grid)
        if (g) { (void)hipFree(g); g = nullptr; }
    if (ctx->R) { (void)hipFree(ctx->R); ctx->R = nullptr; }
    if (ctx->K) { (void)hipFree(ctx->K); ctx->K = nullptr; }
    if (ctx->queue) { (void)hipFree(ctx->queue); ctx->queue = nullptr; }
    if (ctx->Hp) { (void)hipFree(ctx->Hp); ctx->Hp = nullptr; }
    if (ctx->d_source) { (void)hipFree(ctx->d_source); ctx->d_source = nullptr; }
    if (ctx->d_source_prefix) { (void)hipFree(ctx->d_source_prefix); ctx->d_source_prefix = nullptr; }
    if (ctx->d_source_scal) { (void)hipFree(ctx->d_source_scal); ctx->d_source_scal = nullptr; }
    if (ctx->d_rec) { (void)hipFree(ctx->d_rec); ctx->d_rec = nullptr; }
    if (ctx->Kadj) { (void)hipFree(ctx->Kadj); ctx->Kadj = nullptr; }
    if (ctx->d_partial) { (void)hipFree(ctx->d_partial); ctx->d_partial = nullptr; }
    if (ctx->own_stream && ctx->stream) { (void)hipStreamDestroy(ctx->stream); ctx->stream = nullptr; }
}

int select_device(hermite_ctx* ctx) {
    // a failed runtime call elsewhere in this thread leaves its error as the
    // last error; start from a clean state so launch checks see our own
    (void)hipGetLastError();
    HCHECK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    return HERMITE_OK;
}

int half_step(hermite_ctx* ctx, int from) {
    const double* src = ctx->grid[from];
    double* dst = ctx->grid[1 - from];
    const int off = from;  // primal -> dual keeps the index, dual -> primal adds one
    if (ctx->opt.poison)
        HCHECK(ctx, hipMemsetAsync(dst, 0xFF, ctx->grid_doubles * sizeof(double), ctx->stream), "poison");
    hipError_t e;
    if (ctx->nf == 1 && ctx->opt.fused) {
        e = hermite::launch_advect(ctx->m, src, dst, ctx->K1.data(), ctx->n, ctx->pitch, off, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "advection half-step launch");
    } else if (ctx->nf == 1) {
        e = hermite::launch_interp(ctx->m, src, ctx->R, ctx->Hp, ctx->n, ctx->pitch, 1, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "interpolation launch");
        e = hermite::launch_advect_evolve(ctx->m, ctx->R, dst, ctx->E1.data(), ctx->n, ctx->pitch, off, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "advection evolution launch");
    } else if (ctx->opt.fused) {
        const int grid = ctx->cus >= 8 ? (ctx->cus / 8) * 8 : 8;
        if (ctx->precision != HERMITE_PREC_FP64) {
            e = hermite::launch_fused_mixed(ctx->precision, src, dst, ctx->K, ctx->n, ctx->pitch, off, grid, ctx->queue,
                                            ctx->stream);
        } else if (ctx->m == 3 && ctx->m3_kernel == 1) {
            e = hermite::launch_fused_mfma(src, dst, (const double*)ctx->K, ctx->n, ctx->pitch, off, grid, ctx->stream);
        } else if (ctx->m == 3 && ctx->m3_kernel == 2) {
            e = hermite::launch_fused_mfma4(src, dst, (const double*)ctx->K, ctx->n, ctx->pitch, off, grid, ctx->queue,
                                            ctx->stream);
        } else if (ctx->m == 3) {
            e = hermite::launch_fused_valu4(src, dst, (const double*)ctx->K, ctx->n, ctx->pitch, off, ctx->stream);
        } else {
            e = hermite::launch_fused_valu_small(ctx->m, src, dst, (const double*)ctx->K, ctx->n, ctx->pitch, off,
                                                 ctx->stream);
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "fused half-step launch");
    } else {
        e = hermite::launch_interp(ctx->m, src, ctx->R, ctx->Hp, ctx->n, ctx->pitch, 2, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "interpolation launch");
        e = hermite::launch_evolve(ctx->m, ctx->R, dst, ctx->n, ctx->pitch, off, ctx->opt.evolution, ctx->q,
                                   ctx->substeps, ctx->lam, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "evolution launch");
    }
    if (ctx->has_source) {
        e = hermite::launch_source(ctx->d_source, ctx->d_source_prefix + 2 * from, 1, ctx->source_blocks[from], ctx->m,
                                   from, ctx->steps, ctx->d_source_scal, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "source launch");
    }
    return HERMITE_OK;
}

}  // namespace

extern "C" {

void hermite_default_options(hermite_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = HERMITE_PREC_FP64;
    opt->evolution = HERMITE_EVOLVE_TAYLOR;
    opt->rk_substeps = 1;
    opt->q = 0;
    opt->fused = 1;
    opt->poison = 0;
    opt->kernel = HERMITE_KERNEL_AUTO;
    opt->stream = nullptr;
}

int hermite_create(int n_cells, int m, double cfl, double c, const hermite_options* opt, hermite_ctx** out) {
    g_err.clear();
    if (!out) return fail(nullptr, HERMITE_EINVAL, "out is NULL");
    if (n_cells < 2 || n_cells > 1290) return fail(nullptr, HERMITE_EINVAL, "n_cells=%d outside [2, 1290]", n_cells);
    if (m < 1 || m > 3) return fail(nullptr, HERMITE_EINVAL, "m=%d outside [1, 3]", m);
    if (!std::isfinite(cfl) || !(cfl > 0.0) || cfl > 1.0)
        return fail(nullptr, HERMITE_EINVAL, "cfl=%g outside (0, 1]", cfl);
    if (!std::isfinite(c) || !(c > 0.0)) return fail(nullptr, HERMITE_EINVAL, "c=%g must be finite and > 0", c);
    hermite_options o;
    hermite_default_options(&o);
    if (opt) o = *opt;
    if (o.precision < 0 || o.precision > 2) return fail(nullptr, HERMITE_EINVAL, "precision=%d", o.precision);
    if (o.evolution != 0 && o.evolution != 1) return fail(nullptr, HERMITE_EINVAL, "evolution=%d", o.evolution);
    if (o.rk_substeps < 0 || o.rk_substeps > 64) return fail(nullptr, HERMITE_EINVAL, "rk_substeps=%d", o.rk_substeps);
    if (o.q < 0 || o.q > 64) return fail(nullptr, HERMITE_EINVAL, "q=%d outside [0, 64]", o.q);
    if (o.fused != 0 && o.fused != 1) return fail(nullptr, HERMITE_EINVAL, "fused=%d", o.fused);
    if (o.poison != 0 && o.poison != 1) return fail(nullptr, HERMITE_EINVAL, "poison=%d", o.poison);
    if (o.kernel < HERMITE_KERNEL_AUTO || o.kernel > HERMITE_KERNEL_MFMA4)
        return fail(nullptr, HERMITE_EINVAL, "kernel=%d", o.kernel);
    if (o.equation != HERMITE_EQ_WAVE && o.equation != HERMITE_EQ_ADVECTION)
        return fail(nullptr, HERMITE_EINVAL, "equation=%d", o.equation);
    if (o.equation == HERMITE_EQ_ADVECTION) {
        if (o.precision != HERMITE_PREC_FP64 || o.evolution != HERMITE_EVOLVE_TAYLOR)
            return fail(nullptr, HERMITE_EUNSUPPORTED,
                        "advection needs FP64 and Taylor evolution (precision=%d, evolution=%d)", o.precision,
                        o.evolution);
        if (o.q != 0 && o.q < 3 * (2 * m + 1))
            return fail(nullptr, HERMITE_EUNSUPPORTED, "advection needs q = 0 or q >= 3(2m+1) = %d (q=%d)",
                        3 * (2 * m + 1), o.q);
    }
    if (o.precision != HERMITE_PREC_FP64 && (m != 3 || !o.fused))
        return fail(nullptr, HERMITE_EUNSUPPORTED,
                    "precision=%d needs m = 3 and the fused kernel (m=%d, fused=%d)", o.precision, m, o.fused);

    const int M = m + 1, P = 2 * m + 2;
    const int nf = (o.equation == HERMITE_EQ_ADVECTION) ? 1 : 2;
    const size_t nn = (size_t)n_cells * n_cells * n_cells;
    const size_t pitch = hermite::column_pitch(nn);
    const size_t grid_doubles = (size_t)nf * M * M * M * pitch;
    const size_t r_doubles = o.fused ? 0 : (size_t)nf * P * P * P * pitch;

    hermite_ctx* ctx = new (std::nothrow) hermite_ctx();
    if (!ctx) return fail(nullptr, HERMITE_ENOMEM, "host allocation failed");
    ctx->n = n_cells;
    ctx->m = m;
    ctx->M3 = M * M * M;
    ctx->cfl = cfl;
    ctx->c = c;
    ctx->h = 1.0 / n_cells;
    ctx->dt = cfl * ctx->h / c;
    ctx->tau = 0.5 * ctx->dt;
    ctx->lam = c * ctx->tau / ctx->h;
    ctx->opt = o;
    ctx->nf = nf;
    ctx->q = o.q ? o.q : (nf == 1 ? 3 * (2 * m + 1) : 6 * m + 1);
    ctx->substeps = o.rk_substeps ? o.rk_substeps : 1;
    ctx->grid_doubles = grid_doubles;
    ctx->ncell = nn;
    ctx->pitch = pitch;

    auto bail = [&](int code) {
        g_err = ctx->err;
        free_all(ctx);
        delete ctx;
        return code;
    };
    int rc = HERMITE_OK;
    (void)hipGetLastError();  // start from a clean last-error state
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipGetDevice"));
    if ((rc = select_device(ctx)) != HERMITE_OK) return bail(rc);
    if (o.stream) {
        ctx->stream = (hipStream_t)o.stream;
    } else {
        e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipStreamCreate"));
        ctx->own_stream = true;
    }
    for (double*& g : ctx->grid) {
        e = hipMalloc(&g, grid_doubles * sizeof(double));
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipMalloc(grid)"));
    }
    if (r_doubles) {
        e = hipMalloc(&ctx->R, r_doubles * sizeof(double));
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipMalloc(R scratch)"));
    }
    // operator tables (host FP64, uploaded once)
    const std::vector<double> Hp = hermite::hermite_parity_blocks(m);
    const std::vector<double> cpoly = hermite::evolution_poly(m, o.evolution, ctx->q, ctx->substeps);
    const std::vector<double> K = hermite::fused_class_operators(m, ctx->lam, cpoly);
    e = hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipDeviceGetAttribute"));
    ctx->precision = o.precision;
    ctx->m3_kernel = (o.kernel == HERMITE_KERNEL_VALU) ? 0 : (o.kernel == HERMITE_KERNEL_MFMA) ? 1 : 2;
    std::vector<unsigned char> Kdev;
    if (nf == 1) {
        ctx->K1 = hermite::advection_axis_operator(m, ctx->lam);
        ctx->E1 = hermite::advection_translation(m, ctx->lam);
    } else if (o.precision != HERMITE_PREC_FP64) {
        Kdev.resize(hermite::mixed_operator_bytes(o.precision));
        hermite::mixed_build_operators(o.precision, K.data(), Kdev.data());
    } else if (m == 3 && o.fused && ctx->m3_kernel == 1) {
        Kdev.resize(hermite::mfma_operator_doubles() * sizeof(double));
        hermite::mfma_permute_operators(K.data(), (double*)Kdev.data());
    } else if (m == 3 && o.fused && ctx->m3_kernel == 2) {
        Kdev.resize(hermite::mfma_operator_doubles() * sizeof(double));
        if (!hermite::mfma4_arrange_operators(K.data(), (double*)Kdev.data()))
            return bail(fail(ctx, HERMITE_EUNSUPPORTED, "class operator has a nonzero entry the kernel skips"));
    } else if (m == 3) {
        Kdev.resize(hermite::valu4_operator_doubles() * sizeof(double));
        hermite::valu4_build_operators(K.data(), (double*)Kdev.data());
    } else {
        Kdev.resize(hermite::valu_small_operator_doubles(m) * sizeof(double));
        if (!hermite::valu_small_build_operators(m, K.data(), (double*)Kdev.data()))
            return bail(fail(ctx, HERMITE_EUNSUPPORTED, "class operator has a nonzero entry the kernel skips"));
    }
    if (!Kdev.empty()) {
        e = hipMalloc(&ctx->K, Kdev.size());
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipMalloc(K)"));
        e = hipMemcpy(ctx->K, Kdev.data(), Kdev.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "upload K"));
    }
    if (nf == 2 && m == 3 && o.fused && (o.precision != HERMITE_PREC_FP64 || ctx->m3_kernel == 2)) {
        // the context's own work queue: contexts on different streams may run at once
        const std::vector<uint32_t> zero(hermite::kMfma4QueueWords, 0u);
        e = hipMalloc(&ctx->queue, zero.size() * sizeof(uint32_t));
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipMalloc(queue)"));
        e = hipMemcpy(ctx->queue, zero.data(), zero.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "clear queue"));
    }
    e = hipMalloc(&ctx->Hp, Hp.size() * sizeof(double));
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipMalloc(Hp)"));
    e = hipMemcpy(ctx->Hp, Hp.data(), Hp.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "upload Hp"));
    *out = ctx;
    return HERMITE_OK;
}

int hermite_set_initial(hermite_ctx* ctx, const double* u, const double* ut) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (!u || (!ut && ctx->nf == 2)) return fail(ctx, HERMITE_EINVAL, "u or ut is NULL");
    int rc = select_device(ctx);
    if (rc) return rc;
    const size_t rows = (size_t)ctx->M3, w = ctx->ncell * sizeof(double), dp = ctx->pitch * sizeof(double);
    double* g = ctx->grid[0];
    double* gv = g + rows * ctx->pitch;
    HCHECK(ctx, hipStreamSynchronize(ctx->stream), "sync before set_initial");
    HCHECK(ctx, hipMemcpy2D(g, dp, u, w, w, rows, hipMemcpyHostToDevice), "copy u");
    if (ctx->nf == 2) {
        HCHECK(ctx, hipMemcpy2D(gv, dp, ut, w, w, rows, hipMemcpyHostToDevice), "copy ut");
        HCHECK(ctx,
               hermite::launch_scale(gv, ctx->pitch, gv, ctx->pitch, ctx->h / ctx->c, ctx->ncell, ctx->M3, ctx->stream),
               "scale ut");
    }
    HCHECK(ctx, hipStreamSynchronize(ctx->stream), "set_initial");
    ctx->has_state = true;
    ctx->steps = 0;
    ctx->adjoint = false;
    return HERMITE_OK;
}

int hermite_set_initial_device(hermite_ctx* ctx, const void* u_dev, const void* ut_dev) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (!u_dev || (!ut_dev && ctx->nf == 2)) return fail(ctx, HERMITE_EINVAL, "u_dev or ut_dev is NULL");
    int rc = select_device(ctx);
    if (rc) return rc;
    const size_t rows = (size_t)ctx->M3, w = ctx->ncell * sizeof(double), dp = ctx->pitch * sizeof(double);
    double* g = ctx->grid[0];
    double* gv = g + rows * ctx->pitch;
    HCHECK(ctx, hipMemcpy2DAsync(g, dp, u_dev, w, w, rows, hipMemcpyDeviceToDevice, ctx->stream), "copy u");
    if (ctx->nf == 2)
        HCHECK(ctx, hermite::launch_scale(gv, ctx->pitch, (const double*)ut_dev, ctx->ncell, ctx->h / ctx->c,
                                          ctx->ncell, ctx->M3, ctx->stream),
               "scale ut");
    ctx->has_state = true;
    ctx->steps = 0;
    ctx->adjoint = false;
    return HERMITE_OK;
}

int hermite_step(hermite_ctx* ctx, int n_full_steps) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (n_full_steps < 0) return fail(ctx, HERMITE_EINVAL, "n_full_steps=%d < 0", n_full_steps);
    if (!ctx->has_state) return fail(ctx, HERMITE_ESTATE, "hermite_step before hermite_set_initial");
    if (ctx->has_source && ctx->source_desc.series && 2 * (ctx->steps + n_full_steps) > ctx->series_len)
        return fail(ctx, HERMITE_EINVAL, "the source amplitude series (%lld half steps) ends before step %lld",
                    ctx->series_len, ctx->steps + n_full_steps);
    int rc = select_device(ctx);
    if (rc) return rc;
    for (int s = 0; s < n_full_steps; ++s) {
        if ((rc = half_step(ctx, 0)) != HERMITE_OK) return rc;
        if ((rc = half_step(ctx, 1)) != HERMITE_OK) return rc;
        ++ctx->steps;
    }
    return HERMITE_OK;
}

int hermite_step_record(hermite_ctx* ctx, int n_full_steps, void* traces_dev) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (ctx->nrec == 0) return fail(ctx, HERMITE_ESTATE, "hermite_step_record without receivers");
    if (!traces_dev && n_full_steps > 0) return fail(ctx, HERMITE_EINVAL, "traces_dev is NULL");
    for (int s = 0; s < n_full_steps; ++s) {
        const int rc = hermite_step(ctx, 1);
        if (rc) return rc;
        HCHECK(ctx, hermite::launch_record(ctx->grid[0], ctx->d_rec, ctx->nrec, (double*)traces_dev + (size_t)s * ctx->nrec,
                                           ctx->stream),
               "record launch");
    }
    if (n_full_steps == 0) return hermite_step(ctx, 0);
    return HERMITE_OK;
}

int hermite_gather(hermite_ctx* ctx, double* u, double* ut, double* t_out) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (!ctx->has_state) return fail(ctx, HERMITE_ESTATE, "hermite_gather before hermite_set_initial");
    int rc = select_device(ctx);
    if (rc) return rc;
    const size_t rows = (size_t)ctx->M3, w = ctx->ncell * sizeof(double), sp = ctx->pitch * sizeof(double);
    const double* g = ctx->grid[0];
    const double* gv = g + rows * ctx->pitch;
    HCHECK(ctx, hipStreamSynchronize(ctx->stream), "sync before gather (an earlier kernel failed)");
    if (u) HCHECK(ctx, hipMemcpy2D(u, w, g, sp, w, rows, hipMemcpyDeviceToHost), "copy u");
    if (ut && ctx->nf == 2) {
        // the dual grid is dead between full steps: use it as staging
        double* tmp = ctx->grid[1];
        HCHECK(ctx, hermite::launch_scale(tmp, ctx->pitch, gv, ctx->pitch, ctx->c / ctx->h, ctx->ncell, ctx->M3,
                                          ctx->stream),
               "scale ut");
        HCHECK(ctx, hipStreamSynchronize(ctx->stream), "gather scale");
        HCHECK(ctx, hipMemcpy2D(ut, w, tmp, sp, w, rows, hipMemcpyDeviceToHost), "copy ut");
    }
    if (t_out) *t_out = (double)ctx->steps * ctx->dt;
    return HERMITE_OK;
}

int hermite_gather_device(hermite_ctx* ctx, void* u_dev, void* ut_dev) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (!ctx->has_state) return fail(ctx, HERMITE_ESTATE, "hermite_gather_device before hermite_set_initial");
    int rc = select_device(ctx);
    if (rc) return rc;
    const size_t rows = (size_t)ctx->M3, w = ctx->ncell * sizeof(double), sp = ctx->pitch * sizeof(double);
    const double* g = ctx->grid[0];
    const double* gv = g + rows * ctx->pitch;
    if (u_dev) HCHECK(ctx, hipMemcpy2DAsync(u_dev, w, g, sp, w, rows, hipMemcpyDeviceToDevice, ctx->stream), "copy u");
    if (ut_dev && ctx->nf == 2)
        HCHECK(ctx, hermite::launch_scale((double*)ut_dev, ctx->ncell, gv, ctx->pitch, ctx->c / ctx->h, ctx->ncell,
                                          ctx->M3, ctx->stream),
               "scale ut");
    return HERMITE_OK;
}

int hermite_set_source(hermite_ctx* ctx, const hermite_source* src) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (!src || src->amplitude == 0.0) {
        ctx->has_source = false;
        return HERMITE_OK;
    }
    const std::string why = hermite::check_source(*src);
    if (!why.empty()) return fail(ctx, HERMITE_EINVAL, "%s", why.c_str());
    if (ctx->opt.evolution != HERMITE_EVOLVE_TAYLOR || ctx->nf != 2)
        return fail(ctx, HERMITE_EUNSUPPORTED, "the point source needs the wave equation with Taylor evolution");
    int rc = select_device(ctx);
    if (rc) return rc;
    hermite::SourceDesc d = hermite::make_source_desc(*src, ctx->n, ctx->m, ctx->q, ctx->cfl, ctx->c);
    d.grid[0] = ctx->grid[0];
    d.grid[1] = ctx->grid[1];
    d.pitch = ctx->pitch;
    d.steps = 0;  // unused: the host passes the step count at each launch
    d.series = nullptr;  // a new source starts without an amplitude series
    const uint32_t blocks[2] = {hermite::source_blocks(d, 0), hermite::source_blocks(d, 1)};
    const uint32_t prefix[4] = {0, blocks[0], 0, blocks[1]};
    if (!ctx->d_source) HCHECK(ctx, hipMalloc(&ctx->d_source, sizeof(d)), "hipMalloc(source)");
    if (!ctx->d_source_prefix) HCHECK(ctx, hipMalloc(&ctx->d_source_prefix, sizeof(prefix)), "hipMalloc(source)");
    if (!ctx->d_source_scal) HCHECK(ctx, hipMalloc(&ctx->d_source_scal, 20 * sizeof(double)), "hipMalloc(source)");
    // earlier half steps may still read the old entry
    HCHECK(ctx, hipStreamSynchronize(ctx->stream), "sync before set_source");
    HCHECK(ctx, hipMemcpy(ctx->d_source, &d, sizeof(d), hipMemcpyHostToDevice), "upload source");
    HCHECK(ctx, hipMemcpy(ctx->d_source_prefix, prefix, sizeof(prefix), hipMemcpyHostToDevice), "upload source");
    ctx->source_blocks[0] = blocks[0];
    ctx->source_blocks[1] = blocks[1];
    ctx->source_desc = d;
    ctx->series_len = 0;
    ctx->has_source = true;
    return HERMITE_OK;
}

int hermite_set_source_series(hermite_ctx* ctx, const void* amps_dev, long long n_half) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (!ctx->has_source) return fail(ctx, HERMITE_ESTATE, "hermite_set_source_series without a source");
    if (amps_dev && n_half < 0) return fail(ctx, HERMITE_EINVAL, "n_half=%lld < 0", n_half);
    int rc = select_device(ctx);
    if (rc) return rc;
    hermite::SourceDesc d = ctx->source_desc;
    d.series = amps_dev ? (const double*)amps_dev : nullptr;
    HCHECK(ctx, hipStreamSynchronize(ctx->stream), "sync before set_source_series");
    HCHECK(ctx, hipMemcpy(ctx->d_source, &d, sizeof(d), hipMemcpyHostToDevice), "upload source");
    ctx->source_desc = d;
    ctx->series_len = amps_dev ? n_half : 0;
    return HERMITE_OK;
}

int hermite_set_receivers(hermite_ctx* ctx, int n_rec, const int* ijk) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (n_rec < 0 || n_rec > (1 << 24)) return fail(ctx, HERMITE_EINVAL, "n_rec=%d", n_rec);
    if (n_rec > 0 && !ijk) return fail(ctx, HERMITE_EINVAL, "ijk is NULL");
    std::vector<uint32_t> nodes((size_t)n_rec);
    for (int r = 0; r < n_rec; ++r) {
        const int i = ijk[3 * r], j = ijk[3 * r + 1], k = ijk[3 * r + 2];
        if (i < 0 || j < 0 || k < 0 || i >= ctx->n || j >= ctx->n || k >= ctx->n)
            return fail(ctx, HERMITE_EINVAL, "receiver %d at (%d, %d, %d) outside the grid", r, i, j, k);
        nodes[r] = (uint32_t)(((size_t)k * ctx->n + j) * ctx->n + i);
    }
    int rc = select_device(ctx);
    if (rc) return rc;
    HCHECK(ctx, hipStreamSynchronize(ctx->stream), "sync before set_receivers");
    if (ctx->d_rec) {
        (void)hipFree(ctx->d_rec);
        ctx->d_rec = nullptr;
        ctx->nrec = 0;
    }
    if (n_rec > 0) {
        HCHECK(ctx, hipMalloc(&ctx->d_rec, nodes.size() * sizeof(uint32_t)), "hipMalloc(receivers)");
        HCHECK(ctx, hipMemcpy(ctx->d_rec, nodes.data(), nodes.size() * sizeof(uint32_t), hipMemcpyHostToDevice),
               "upload receivers");
    }
    ctx->nrec = (uint32_t)n_rec;
    return HERMITE_OK;
}

namespace {

// One transposed half step: lam_src from lam_dst (off as the forward half step).
hipError_t adjoint_half(hermite_ctx* ctx, const double* lam_dst, double* lam_src, int off) {
    if (ctx->m == 3) {
        const int grid = ctx->cus >= 8 ? (ctx->cus / 8) * 8 : 8;
        return hermite::launch_adjoint_mfma(lam_dst, lam_src, (const double*)ctx->Kadj, ctx->n, ctx->pitch,
                                            off, grid, ctx->queue, ctx->stream);
    }
    return hermite::launch_adjoint(ctx->m, lam_dst, lam_src, (const double*)ctx->Kadj, ctx->n, ctx->pitch, off,
                                   ctx->stream);
}

int adjoint_supported(hermite_ctx* ctx) {
    if (ctx->nf != 2 || ctx->precision != HERMITE_PREC_FP64)
        return fail(ctx, HERMITE_EUNSUPPORTED, "the adjoint needs the wave equation in FP64");
    return HERMITE_OK;
}

}  // namespace

int hermite_adjoint_init(hermite_ctx* ctx, const void* lam_u_dev, const void* lam_ut_dev) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    int rc = adjoint_supported(ctx);
    if (rc) return rc;
    if (!ctx->has_state && !ctx->adjoint) return fail(ctx, HERMITE_ESTATE, "hermite_adjoint_init before a forward run");
    if ((lam_u_dev == nullptr) != (lam_ut_dev == nullptr))
        return fail(ctx, HERMITE_EINVAL, "lam_u_dev and lam_ut_dev must both be given or both NULL");
    if ((rc = select_device(ctx)) != HERMITE_OK) return rc;
    if (!ctx->Kadj) {
        const std::vector<double> cpoly = hermite::evolution_poly(ctx->m, ctx->opt.evolution, ctx->q, ctx->substeps);
        std::vector<double> K = hermite::fused_class_operators(ctx->m, ctx->lam, cpoly);
        if (ctx->m == 3) {
            std::vector<double> KT(hermite::adjoint_mfma_operator_doubles());
            hermite::adjoint_mfma_build_operator(K.data(), KT.data());
            K.swap(KT);
        }
        HCHECK(ctx, hipMalloc(&ctx->Kadj, K.size() * sizeof(double)), "hipMalloc(adjoint operator)");
        HCHECK(ctx, hipMemcpy(ctx->Kadj, K.data(), K.size() * sizeof(double), hipMemcpyHostToDevice),
               "upload adjoint operator");
    }
    if (ctx->m == 3 && !ctx->queue) {
        // the m = 3 transposed half step takes its work from the context's queue
        const std::vector<uint32_t> zero(hermite::kMfma4QueueWords, 0u);
        HCHECK(ctx, hipMalloc(&ctx->queue, zero.size() * sizeof(uint32_t)), "hipMalloc(queue)");
        HCHECK(ctx, hipMemcpy(ctx->queue, zero.data(), zero.size() * sizeof(uint32_t), hipMemcpyHostToDevice),
               "clear queue");
    }
    const size_t rows = (size_t)ctx->M3, w = ctx->ncell * sizeof(double), dp = ctx->pitch * sizeof(double);
    double* g = ctx->grid[0];
    double* gv = g + rows * ctx->pitch;
    if (lam_u_dev) {
        // d/d(vt) = (c/h) d/d(u_t), since u_t = (c/h) vt
        HCHECK(ctx, hipMemcpy2DAsync(g, dp, lam_u_dev, w, w, rows, hipMemcpyDeviceToDevice, ctx->stream), "copy lam_u");
        HCHECK(ctx, hermite::launch_scale(gv, ctx->pitch, (const double*)lam_ut_dev, ctx->ncell, ctx->c / ctx->h,
                                          ctx->ncell, ctx->M3, ctx->stream),
               "scale lam_ut");
    } else {
        HCHECK(ctx, hipMemsetAsync(g, 0, ctx->grid_doubles * sizeof(double), ctx->stream), "zero adjoint");
    }
    ctx->adj_steps = ctx->adjoint ? ctx->adj_steps : ctx->steps;
    ctx->adjoint = true;
    ctx->has_state = false;
    return HERMITE_OK;
}

int hermite_adjoint_step(hermite_ctx* ctx, int n_full_steps, const void* res_dev, void* grad_amps_dev) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (!ctx->adjoint) return fail(ctx, HERMITE_ESTATE, "hermite_adjoint_step before hermite_adjoint_init");
    if (n_full_steps < 0 || n_full_steps > ctx->adj_steps)
        return fail(ctx, HERMITE_EINVAL, "n_full_steps=%d outside [0, %lld]", n_full_steps, ctx->adj_steps);
    if (ctx->nrec > 0 && !res_dev && n_full_steps > 0) return fail(ctx, HERMITE_EINVAL, "res_dev is NULL");
    if (grad_amps_dev && !ctx->has_source)
        return fail(ctx, HERMITE_ESTATE, "grad_amps_dev given without a source");
    int rc = select_device(ctx);
    if (rc) return rc;
    const uint32_t need = std::max<uint32_t>(1, std::max(ctx->source_blocks[0], ctx->source_blocks[1]));
    if (grad_amps_dev && ctx->partial_cap < need) {
        HCHECK(ctx, hipStreamSynchronize(ctx->stream), "sync before reallocating partials");
        if (ctx->d_partial) (void)hipFree(ctx->d_partial);
        ctx->d_partial = nullptr;
        ctx->partial_cap = 0;
        HCHECK(ctx, hipMalloc(&ctx->d_partial, need * sizeof(double)), "hipMalloc(partials)");
        ctx->partial_cap = need;
    }
    const long long t0 = ctx->adj_steps - n_full_steps;
    double* lam_p = ctx->grid[0];
    double* lam_d = ctx->grid[1];
    for (int s = n_full_steps - 1; s >= 0; --s) {
        const long long k = t0 + s;  // the full step being reversed
        if (ctx->nrec > 0)
            HCHECK(ctx, hermite::launch_inject(lam_p, ctx->d_rec, ctx->nrec, (const double*)res_dev + (size_t)s * ctx->nrec,
                                               ctx->stream),
                   "inject launch");
        if (grad_amps_dev)
            HCHECK(ctx, hermite::launch_source_dot(ctx->d_source, ctx->d_source_prefix + 2, ctx->source_blocks[1], ctx->m,
                                                   1, k, ctx->d_source_scal, ctx->d_partial,
                                                   (double*)grad_amps_dev + 2 * s + 1, ctx->stream),
                   "source gradient launch");
        HCHECK(ctx, adjoint_half(ctx, lam_p, lam_d, 1), "adjoint half-step launch");
        if (grad_amps_dev)
            HCHECK(ctx, hermite::launch_source_dot(ctx->d_source, ctx->d_source_prefix, ctx->source_blocks[0], ctx->m, 0,
                                                   k, ctx->d_source_scal, ctx->d_partial,
                                                   (double*)grad_amps_dev + 2 * s, ctx->stream),
                   "source gradient launch");
        HCHECK(ctx, adjoint_half(ctx, lam_d, lam_p, 0), "adjoint half-step launch");
    }
    ctx->adj_steps = t0;
    return HERMITE_OK;
}

int hermite_adjoint_gather(hermite_ctx* ctx, void* gu_dev, void* gut_dev) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (!ctx->adjoint) return fail(ctx, HERMITE_ESTATE, "hermite_adjoint_gather before hermite_adjoint_init");
    int rc = select_device(ctx);
    if (rc) return rc;
    const size_t rows = (size_t)ctx->M3, w = ctx->ncell * sizeof(double), sp = ctx->pitch * sizeof(double);
    const double* g = ctx->grid[0];
    const double* gv = g + rows * ctx->pitch;
    if (gu_dev) HCHECK(ctx, hipMemcpy2DAsync(gu_dev, w, g, sp, w, rows, hipMemcpyDeviceToDevice, ctx->stream), "copy gu");
    // d/d(u_t) = (h/c) d/d(vt)
    if (gut_dev)
        HCHECK(ctx, hermite::launch_scale((double*)gut_dev, ctx->ncell, gv, ctx->pitch, ctx->h / ctx->c, ctx->ncell,
                                          ctx->M3, ctx->stream),
               "scale gut");
    return HERMITE_OK;
}

int hermite_state_finite(hermite_ctx* ctx, int* all_finite) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (!all_finite) return fail(ctx, HERMITE_EINVAL, "all_finite is NULL");
    if (!ctx->has_state && !ctx->adjoint) return fail(ctx, HERMITE_ESTATE, "hermite_state_finite before a state");
    int rc = select_device(ctx);
    if (rc) return rc;
    int* flag = nullptr;
    HCHECK(ctx, hipMalloc(&flag, sizeof(int)), "hipMalloc(flag)");
    int host = 0;
    hipError_t e = hipMemcpyAsync(flag, &host, sizeof(int), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hermite::launch_nonfinite(ctx->grid[0], ctx->pitch, ctx->ncell, ctx->nf * ctx->M3, flag, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(flag);
    if (e != hipSuccess) return hip_fail(ctx, e, "finite check");
    *all_finite = host ? 0 : 1;
    return HERMITE_OK;
}

int hermite_sync(hermite_ctx* ctx) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    int rc = select_device(ctx);
    if (rc) return rc;
    HCHECK(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    return HERMITE_OK;
}

int hermite_get_time(const hermite_ctx* ctx, double* t, long long* steps, double* dt) {
    if (!ctx) return fail(nullptr, HERMITE_EINVAL, "ctx is NULL");
    if (t) *t = (double)ctx->steps * ctx->dt;
    if (steps) *steps = ctx->steps;
    if (dt) *dt = ctx->dt;
    return HERMITE_OK;
}

void hermite_destroy(hermite_ctx* ctx) {
    if (!ctx) return;
    if (hipSetDevice(ctx->device) == hipSuccess && ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
}

const char* hermite_last_error(const hermite_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_err.c_str();
}

}  // extern "C"
