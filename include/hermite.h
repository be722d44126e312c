/*
 * hermite.h - C ABI of the MI355X (gfx950) Hermite wave solver.
 *
 * The library advances the 3D scalar wave equation u_tt = c^2 (u_x1x1 +
 * u_x2x2 + u_x3x3) on the periodic unit cube [0,1)^3 with the Hermite method
 * studied by Vargas, Chan, Hagstrom and Warburton, "GPU Acceleration of
 * Hermite Methods for the Simulation of Wave Propagation" (arXiv:1609.09841).
 *
 * Problem statement (Sec. 2): a periodic grid of n cells per side, h = 1/n;
 * each node carries the scaled derivatives h^{|d|}/d! D^d of u and of u_t for
 * every multi-index d in [0,m]^3 (Eq. 2; the paper calls m "N"). One full time
 * step dt = cfl * h / c is two half steps: primal -> dual grid, then dual ->
 * primal grid (Sec. 2). Each half step builds, on every cell, the tensor
 * Hermite interpolant of degree 2m+1 per variable from the 8 vertices (Eq. 3;
 * Sec. 3.1, Alg. 1-2) and evolves it through dt/2 (Sec. 3.2, Alg. 3-4, Taylor
 * series; or classical 4-stage Runge-Kutta, the multi-stage evolution of the
 * abstract). The coefficients of the evolved polynomial with every index <= m
 * are the new data of the node at the cell centre.
 *
 * Array layout (Sec. 3.1, the tensor u[m3][m2][m1][n3][n2][n1]): a field
 * holds (m+1)^3 * n^3 doubles ordered [d3][d2][d1][k][j][i], i (x1) fastest.
 * Node (i, j, k) is the point (i, j, k) * h.
 *
 * Errors: every int-returning call returns HERMITE_OK (0) or a negative
 * code; no call aborts or throws. On failure nothing is changed. The text of
 * the last error is returned by hermite_last_error. Device faults of
 * asynchronous work surface at the next hermite_sync / hermite_gather*.
 *
 * Threading: a context may be used by one host thread at a time.
 */
#ifndef HERMITE_H
#define HERMITE_H

#ifdef __cplusplus
extern "C" {
#endif

#define HERMITE_OK 0
#define HERMITE_EINVAL (-1)       /* bad argument: see each call */
#define HERMITE_ENOMEM (-2)       /* device allocation failed or size overflow */
#define HERMITE_EDEVICE (-3)      /* HIP runtime error (no device, launch failure, fault) */
#define HERMITE_ESTATE (-4)       /* call out of order (step/gather before set_initial) */
#define HERMITE_EUNSUPPORTED (-5) /* valid but unsupported combination of options */

/* Arithmetic of the interpolation/evolution contractions. The nodal state,
 * the corner-mean part of every new value and the half-step update are FP64
 * in every mode. FP32: the rest of the contraction on FP32 matrix cores with
 * FP32 accumulation. BF16X3: operator and inputs each split into two BF16
 * parts, three products accumulated in FP32. FP32 and BF16X3 need m = 3 and
 * fused = 1 (HERMITE_EUNSUPPORTED otherwise). At m = 3 the monomial-basis
 * interpolation cancels heavily in the high-order derivatives, so the
 * rounding of the low-precision modes shows up there first: state the error
 * against an FP64 run for every use. */
#define HERMITE_PREC_FP64 0
#define HERMITE_PREC_FP32 1
#define HERMITE_PREC_BF16X3 2

/* Kernel of the fused FP64 half step at m = 3 (ignored otherwise). All
 * compute the same contraction in FP64 with the same operator and give
 * bit-identical results; on gfx950 the 4x4-tile matrix-core kernel is the
 * fastest. Batches (hermite_batch_*) and slabs (hermite_slab_*) always run
 * the 4x4-tile kernel (a slab's lone boundary plane the 16x16 one). */
#define HERMITE_KERNEL_AUTO 0  /* the 4x4-tile matrix-core kernel */
#define HERMITE_KERNEL_MFMA 1  /* FP64 matrix cores (v_mfma_f64_16x16x4) */
#define HERMITE_KERNEL_VALU 2  /* FP64 vector FMAs, operator entries as scalar operands */
#define HERMITE_KERNEL_MFMA4 3 /* FP64 matrix cores in 4x4 tiles (v_mfma_f64_4x4x4, 4 blocks),
                                  two z-adjacent 16-cell batches per wave */

/* Equation (Sec. 2). WAVE: u_tt = c^2 Lap u as the first-order system
 * (u, u_t), two fields per node. ADVECTION: u_t = c (u_x1 + u_x2 + u_x3),
 * the paper's Eq. 1 (c = 1), one field per node: set_initial and gather then
 * ignore ut (it may be NULL). Advection needs FP64 and Taylor evolution with
 * q = 0 or q >= 3(2m+1) (the series is then exact, Sec. 3.2),
 * HERMITE_EUNSUPPORTED otherwise; both kernel organisations (fused and two
 * kernels); it has no point source. */
#define HERMITE_EQ_WAVE 0
#define HERMITE_EQ_ADVECTION 1

#define HERMITE_EVOLVE_TAYLOR 0 /* Sec. 3.2, Alg. 4: q-stage Taylor series (Horner) */
#define HERMITE_EVOLVE_RK4 1    /* classical 4-stage Runge-Kutta on the cell ODE */

typedef struct hermite_ctx hermite_ctx; /* opaque; owns all device memory */

typedef struct hermite_options {
    int precision;   /* HERMITE_PREC_*; default FP64 */
    int evolution;   /* HERMITE_EVOLVE_*; default Taylor */
    int rk_substeps; /* RK4 substeps per half step, >= 1; 0 -> 1 */
    int q;           /* Taylor stages, 1..64; 0 -> the exact count: 6m+1 for
                        the wave system (the paper's d(2N+1) = 6m+3 gives the
                        same result up to rounding, Sec. 3.2), 3(2m+1) for
                        advection */
    int fused;       /* 1: one kernel per half step (Sec. 3.3, monolithic);
                        0: interpolation and evolution kernels with the
                        reconstructed coefficients in device memory
                        (Sec. 3.1-3.2, two kernels) */
    int poison;      /* debug: 1 fills each destination grid with NaN before
                        the half step that writes it */
    int kernel;      /* fused FP64 kernel for m = 3: HERMITE_KERNEL_* */
    int equation;    /* HERMITE_EQ_*; default WAVE */
    void *stream;    /* hipStream_t to run on; NULL -> a stream owned by the
                        context. Caller keeps a given stream alive until
                        hermite_destroy. */
} hermite_options;

/* Fills *opt with the defaults (FP64, Taylor q = 6m+1, fused, own stream). */
void hermite_default_options(hermite_options *opt);

/*
 * Creates a solver for n_cells^3 periodic cells of order m (Sec. 2).
 *   n_cells: cells per side, 2 <= n_cells <= 1290
 *   m:       derivatives per dimension, 1..3
 *   cfl:     c*dt/h, 0 < cfl <= 1 and finite. The paper's stability statement
 *            (Sec. 2: waves must not cross from the cell boundary to its centre
 *            in a half step) is necessary; in 3D the Taylor method is stable
 *            up to about 0.8 and RK4 (1 substep) up to 0.5.
 *   c:       wave speed (advection: the speed along each axis), > 0 and
 *            finite
 *   opt:     NULL for defaults
 *   out:     receives the context; untouched on failure
 * Arguments are validated before any HIP call: invalid arguments return
 * HERMITE_EINVAL (HERMITE_EUNSUPPORTED for a valid but unsupported option
 * combination) even without a device. Allocates two FP64 grids of
 * 2*(m+1)^3 columns of n^3 doubles each ((m+1)^3 for advection), plus
 * 2*(2m+2)^3 columns when
 * fused == 0; each device column is padded by at most 112 doubles.
 * No kernel runs.
 */
int hermite_create(int n_cells, int m, double cfl, double c,
                   const hermite_options *opt, hermite_ctx **out);

/*
 * Sets the primal-grid state at t = 0 from host arrays u and ut (scaled
 * derivatives of u and of u_t, layout above, (m+1)^3*n^3 doubles each; the
 * caller keeps ownership). Copies synchronously. Resets t and the step count.
 */
int hermite_set_initial(hermite_ctx *ctx, const double *u, const double *ut);

/* As hermite_set_initial, from device arrays; stream-ordered on the
 * context's stream (the caller must not free them before that work ends). */
int hermite_set_initial_device(hermite_ctx *ctx, const void *u_dev, const void *ut_dev);

/*
 * Enqueues n_full_steps full steps (2 * n_full_steps half steps) on the
 * context's stream and returns without waiting. n_full_steps >= 0.
 * HERMITE_ESTATE before any set_initial.
 */
int hermite_step(hermite_ctx *ctx, int n_full_steps);

/*
 * Waits for the stream, then copies the primal-grid state to host arrays u and
 * ut (same layout as set_initial) and stores t = steps * dt in *t_out (t_out
 * may be NULL; u or ut may be NULL to skip that field).
 */
int hermite_gather(hermite_ctx *ctx, double *u, double *ut, double *t_out);

/* Stream-ordered copy of the state into device arrays (no host wait). */
int hermite_gather_device(hermite_ctx *ctx, void *u_dev, void *ut_dev);

/*
 * Point source: the solver then advances u_tt = c^2 Lap u + f with
 *   f(x, t) = amplitude * g(x) * w(t),
 *   g(x) = prod_i exp(-d_i^2 / (2 sigma^2)) / (sigma sqrt(2 pi)),
 *   w(t) = (1 - 2 beta s^2) exp(-beta s^2), s = t - t0, beta = (pi freq)^2,
 * d_i the periodic nearest-image offset of x_i from the source point x (each
 * factor taken as 0 beyond 6 sigma), a Gaussian in space times a Ricker
 * wavelet in time (an extension of Sec. 2: the local Taylor series of the
 * cell solution, Sec. 3.2, also carries the forcing; each half step adds the
 * particular solution of the cell system with zero data to the nodes of the
 * cells within 6 sigma of the source, after the homogeneous half step).
 *   src: x in any real coordinates (reduced modulo 1), sigma > 0,
 *        freq >= 0, t0 and amplitude finite; all finite. NULL (or
 *        amplitude 0) removes the source.
 * Needs Taylor evolution (HERMITE_EUNSUPPORTED with RK4); works with every
 * precision and kernel (the source term itself is FP64). Takes effect with
 * the next hermite_step; the copy is the context's, the caller keeps src.
 * Time is the context's t = steps * dt (hermite_set_initial resets it).
 */
typedef struct hermite_source {
    double x[3];      /* source point */
    double sigma;     /* standard deviation of the Gaussian */
    double freq;      /* peak frequency f0 of the wavelet */
    double t0;        /* time of the wavelet's peak */
    double amplitude; /* factor a of f */
} hermite_source;

int hermite_set_source(hermite_ctx *ctx, const hermite_source *src);

/* ------------------------------------------------------------------------
 * Receivers and gradients (adjoint sweep). An extension: the paper has no
 * adjoint. For the wave equation in FP64 (HERMITE_EUNSUPPORTED otherwise).
 * ------------------------------------------------------------------------ */

/* Receivers at primal nodes ijk[r] = (i, j, k), 0 <= i, j, k < n (host
 * array of 3 n_rec ints, copied); they record u (the value, d = 0).
 * n_rec = 0 removes them. */
int hermite_set_receivers(hermite_ctx *ctx, int n_rec, const int *ijk);

/* Scales the point source of half step h (two per full step, counted from
 * t = 0) by amps_dev[h], h < n_half (device array of doubles, read by the
 * kernels at each half step: the caller keeps it alive and unchanged while
 * steps are enqueued). Needs a source (HERMITE_ESTATE). NULL removes the
 * scaling. hermite_step fails with HERMITE_EINVAL for half steps beyond
 * n_half. */
int hermite_set_source_series(hermite_ctx *ctx, const void *amps_dev, long long n_half);

/* As hermite_step, and after each full step s writes the receivers' u to
 * traces_dev[s * n_rec + r] (device doubles). Needs receivers. */
int hermite_step_record(hermite_ctx *ctx, int n_full_steps, void *traces_dev);

/* Starts an adjoint sweep at the context's current time t = steps * dt:
 * the adjoint state (the gradient of the objective with respect to the state
 * u, u_t at t) is set from device arrays lam_u_dev, lam_ut_dev (layout of
 * hermite_set_initial), or zero when both are NULL. The forward state is
 * replaced (hermite_set_initial is needed before stepping again). */
int hermite_adjoint_init(hermite_ctx *ctx, const void *lam_u_dev, const void *lam_ut_dev);

/* n_full_steps steps of the adjoint sweep, back in time. res_dev (device,
 * n_full_steps * n_rec doubles, may be NULL without receivers): res[s][r] is
 * the derivative of the objective with respect to the trace value that
 * hermite_step_record wrote after full step t0 + s, t0 = (sweep time in
 * steps) - n_full_steps; it is added into the adjoint state at that step.
 * grad_amps_dev (device, 2 n_full_steps doubles, or NULL): receives the
 * derivative with respect to the source scaling of half steps 2 t0 .. 2 t0 +
 * 2 n_full_steps - 1 (needs a source). Each step applies the transposes of
 * the two half steps (the transpose of a fused half step: its class
 * operators transposed and the vertex butterfly reversed, gathered per node
 * over the 8 cells around it). */
int hermite_adjoint_step(hermite_ctx *ctx, int n_full_steps, const void *res_dev, void *grad_amps_dev);

/* Copies the adjoint state, i.e. the gradient with respect to u and u_t at
 * the sweep's current time, to device arrays (either may be NULL). */
int hermite_adjoint_gather(hermite_ctx *ctx, void *gu_dev, void *gut_dev);

/* Failure detection: *all_finite = 1 if every DOF of the state (or of the
 * adjoint state during an adjoint sweep) is finite, else 0 (NaN or Inf, e.g.
 * after running beyond the stable cfl range). Waits for the stream. */
int hermite_state_finite(hermite_ctx *ctx, int *all_finite);

/* Waits for all work enqueued on the context's stream. */
int hermite_sync(hermite_ctx *ctx);

/* Time reached by the enqueued steps, full steps taken, and dt. Any pointer may be NULL. */
int hermite_get_time(const hermite_ctx *ctx, double *t, long long *steps, double *dt);

/* Waits for outstanding work and frees everything the context owns. NULL is a no-op. */
void hermite_destroy(hermite_ctx *ctx);

/* Last error text of ctx, or of the calling thread when ctx is NULL
 * (for failures of hermite_create). Never NULL; "" when there was none. */
const char *hermite_last_error(const hermite_ctx *ctx);

/* ------------------------------------------------------------------------
 * Batches of independent shots. A batch owns many grids of uneven sizes and
 * orders that share cfl and c (each with its own h = 1/n and dt = cfl h / c)
 * and step together: every half step runs one launch per order present,
 * each covering all shots of that order, then one launch for all point
 * sources (the same half step as hermite_step, Sec. 2-3, per shot).
 * ------------------------------------------------------------------------ */
typedef struct hermite_batch hermite_batch; /* opaque; owns all device memory */

typedef struct hermite_shot {
    int n_cells;           /* cells per side, 2 .. 1290 */
    int m;                 /* derivatives per dimension, 1 .. 3 */
    int has_source;        /* 1: `source` forces this shot (as hermite_set_source) */
    hermite_source source;
} hermite_shot;

typedef struct hermite_batch_options {
    int precision;   /* HERMITE_PREC_* of the m = 3 shots; m = 1, 2 shots
                        always run the FP64 kernels */
    int evolution;   /* HERMITE_EVOLVE_*; sources need Taylor */
    int rk_substeps; /* as hermite_options */
    int q;           /* as hermite_options */
    int graph;       /* 1 (default): hermite_batch_step replays one captured
                        HIP graph per full step (order groups on parallel
                        branches); 0: direct launches on the stream */
    int autotune;    /* 1 (default): hermite_batch_create times every
                        candidate launch shape of each order group on the
                        batch's own grids and keeps the fastest; 0: defaults */
    void *stream;    /* hipStream_t; NULL -> a stream owned by the batch */
} hermite_batch_options;

/* Defaults: FP64, Taylor q = 6m+1, graph on, autotune on, own stream. */
void hermite_batch_default_options(hermite_batch_options *opt);

/*
 * Creates a batch of n_shots (1 .. 4096) shots, all at t = 0 with zero data.
 * shots: n_shots descriptions (copied; validated as hermite_create and
 * hermite_set_source validate theirs: HERMITE_EINVAL, HERMITE_EUNSUPPORTED
 * for a source with RK4 evolution). Allocates two grids per shot (layout of
 * hermite_create), zero-fills them and, with autotune, runs each candidate
 * shape on the dual grids (which hold no state between full steps).
 */
int hermite_batch_create(int n_shots, const hermite_shot *shots, double cfl, double c,
                         const hermite_batch_options *opt, hermite_batch **out);

/* Sets shot `shot` (0-based) from host arrays (layout and scaling of
 * hermite_set_initial; NULL u and ut: zero data) and restarts its clock at
 * t = 0. Waits for the batch's stream first; copies synchronously. */
int hermite_batch_set_initial(hermite_batch *b, int shot, const double *u, const double *ut);

/* Enqueues n_full_steps full steps of every shot (async, n_full_steps >= 0). */
int hermite_batch_step(hermite_batch *b, int n_full_steps);

/* Waits, then copies shot `shot`'s state to host arrays (either may be NULL)
 * and its time t = steps * dt into *t_out (may be NULL). */
int hermite_batch_gather(hermite_batch *b, int shot, double *u, double *ut, double *t_out);

/* Waits for all work enqueued on the batch's stream. */
int hermite_batch_sync(hermite_batch *b);

/* Launch shape chosen for the shots of order m (HERMITE_EINVAL if the batch
 * has none): *choice indexes the candidates (m = 1, 2: blocks of 64, 128,
 * 256 cells; m = 3: item runs of 1 or 4 batches, XCD-sliced or
 * interleaved, in that order) and *ms its measured half-step time (0 when
 * not tuned). Either pointer may be NULL. */
int hermite_batch_tuning(const hermite_batch *b, int m, int *choice, double *ms);

/* Waits for outstanding work and frees everything. NULL is a no-op. */
void hermite_batch_destroy(hermite_batch *b);

/* Last error of b, or of the calling thread's last failed
 * hermite_batch_create when b is NULL. Never NULL. */
const char *hermite_batch_last_error(const hermite_batch *b);

/* ------------------------------------------------------------------------
 * One z-slab of a periodic grid sharded over devices (the grid of Sec. 2
 * cut into slabs of whole cell planes; one slab per device). A slab owns
 * the node planes z0 .. z0+nz-1 of both grids and updates them with the
 * fused m = 3 FP64 half step (Sec. 3.3) on the matrix cores. The primal ->
 * dual half step reads one primal plane it does not own (z0+nz, the first
 * plane of the slab above); the dual -> primal half step one dual plane
 * (z0-1, the last plane of the slab below). The caller moves those planes
 * between half steps (peer copies, RCCL send/recv, or, for a slab holding
 * the whole grid, a copy within the slab), reading and writing the device
 * planes that hermite_slab_plane names. No collectives are made here.
 *
 * A plane is 2 (m+1)^3 rows of n^2 doubles (row r = column r of the grid
 * layout: field, then derivative multi-index, as hermite_set_initial),
 * consecutive rows `pitch_bytes` apart, each row [j][i] with i fastest.
 * Errors: as hermite_create; options other than FP64, fused, wave equation,
 * m = 3 give HERMITE_EUNSUPPORTED.
 * ------------------------------------------------------------------------ */
typedef struct hermite_slab hermite_slab; /* opaque; owns its device memory */

#define HERMITE_SLAB_PRIMAL_FIRST 0 /* own primal plane z0: the slab below reads it */
#define HERMITE_SLAB_PRIMAL_HALO 1  /* primal plane z0+nz: fill before a primal -> dual half step */
#define HERMITE_SLAB_DUAL_LAST 2    /* own dual plane z0+nz-1: the slab above reads it */
#define HERMITE_SLAB_DUAL_HALO 3    /* dual plane z0-1: fill before a dual -> primal half step */

/* n_cells: cells per side in x and y (2 .. 1290); nz: cell planes of this
 * slab, 1 <= nz, n_cells^2 (nz+1) < 2^31; cfl, c, opt as hermite_create. */
int hermite_slab_create(int n_cells, int nz, int m, double cfl, double c, const hermite_options *opt,
                        hermite_slab **out);
/* Host arrays of the slab's own planes: u, ut each (m+1)^3 nz n^2 doubles,
 * [d3][d2][d1][k][j][i] with k = 0 .. nz-1 the planes z0 .. z0+nz-1;
 * synchronous; resets the time to 0 and the next half step to primal -> dual. */
int hermite_slab_set_initial(hermite_slab *s, const double *u, const double *ut);
/* Device address of one of the four exchange planes (HERMITE_SLAB_*) and
 * the row stride in bytes. The addresses stay valid until destroy. */
int hermite_slab_plane(hermite_slab *s, int which, void **dev, size_t *pitch_bytes);
/* Enqueue one half step on the slab's stream: primal -> dual when the slab
 * has taken an even number of half steps, dual -> primal otherwise. The
 * halo plane it reads must be filled (stream-ordered) before the call.
 * Returns in *next_halo (if not NULL) the HERMITE_SLAB_*_HALO plane the
 * following half step reads. Same as hermite_slab_half_step_part with
 * HERMITE_SLAB_ALL. */
int hermite_slab_half_step(hermite_slab *s, int *next_halo);
/* One half step in two parts, so that the halo's exchange can overlap the
 * cells that do not read it: HERMITE_SLAB_INTERIOR enqueues every cell plane
 * but the one that reads the halo (the top one in a primal -> dual half
 * step, the bottom one after), and needs no halo; *next_halo then names the
 * halo this half step's HERMITE_SLAB_BOUNDARY call reads, which enqueues that
 * plane and completes the half step. The interior part neither reads nor
 * writes the halo plane or the plane the neighbour copies.
 * HERMITE_SLAB_ALL = both at once. HERMITE_ESTATE for a part out of order. */
#define HERMITE_SLAB_INTERIOR 1
#define HERMITE_SLAB_BOUNDARY 2
#define HERMITE_SLAB_ALL 3
int hermite_slab_half_step_part(hermite_slab *s, int part, int *next_halo);
/* After an even number of half steps: the slab's own planes (layout as
 * set_initial; either pointer may be NULL) and t = full steps * dt;
 * synchronous. HERMITE_ESTATE after an odd number. */
int hermite_slab_gather(hermite_slab *s, double *u, double *ut, double *t_out);
/* Copy plane `src_which` of slab `src` into plane `dst_which` of `dst`
 * (e.g. PRIMAL_FIRST of the slab above into PRIMAL_HALO of this one), as
 * one 2-D copy enqueued on `stream` (a hipStream_t; NULL = dst's stream);
 * the slabs may sit on different devices (a peer copy). The plane of src
 * must be complete when the copy runs, and dst must not read the plane
 * until it has: same stream, or events between the streams. */
int hermite_slab_copy_plane(hermite_slab *dst, int dst_which, hermite_slab *src, int src_which, void *stream);
int hermite_slab_sync(hermite_slab *s);
void hermite_slab_destroy(hermite_slab *s);
const char *hermite_slab_last_error(const hermite_slab *s);

#ifdef __cplusplus
}
#endif

#endif /* HERMITE_H */
