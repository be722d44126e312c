/*
 * Plain FP64 CPU oracle for the Hermite method applied to the 3D scalar wave
 * equation u_tt = c^2 (u_x1x1 + u_x2x2 + u_x3x3) on a periodic unit cube.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path links, loads or calls
 * this file: only the test-suite, the smoke check and the benchmark's CPU
 * baseline use it. It shares no code, header, table or constant generator
 * with the HIP library.
 *
 * It is written to be read against Vargas, Chan, Hagstrom and Warburton,
 * "GPU Acceleration of Hermite Methods for the Simulation of Wave Propagation"
 * (arXiv:1609.09841):
 *   - Sec. 2, Eq. 2: each node carries the scaled derivatives
 *     h^{|i|}/i! D^i u for every multi-index i in [0,N]^3 (here N is called m).
 *   - Sec. 2, Eq. 3: on each cell, the tensor-product polynomial of degree
 *     2m+1 per variable in the cell variable xi = (x - x_centre)/h matches
 *     the data of the 8 vertices; its coefficients are the centre data.
 *   - Sec. 3.1, Alg. 1 and Alg. 2: that polynomial is built by applying the
 *     1D Hermite matrix H along x1, then x2, then x3.
 *   - Sec. 3.2, Alg. 3: derivative of the coefficient tensor by an index shift.
 *   - Sec. 3.2, Alg. 4: the q-stage Horner loop of the Taylor evolution.
 *   - Sec. 2 (after Eq. 5): the series is evaluated at the half step and the
 *     process repeats on the other (dual/primal) grid.
 *
 * Readings of the paper used here (the paper states only the advection case):
 *   - The wave equation is taken as the first-order system (u, u_t). Inside
 *     the method u_t is carried as vt = (h/c) u_t, so that in the cell
 *     variable xi and the half-step time sigma = (t - t_n)/tau the system is
 *     u_sigma = lam * vt, vt_sigma = lam * Lap_xi u with lam = c*tau/h.
 *   - The time step in Alg. 4 is the half step tau = dt/2.
 *   - The derivative matrix has indices 0..2m+1.
 *   - Dual node (i+1/2, j+1/2, k+1/2)h is stored at index (i, j, k); the dual
 *     cell with lower corner (i, j, k) writes primal node (i+1, j+1, k+1).
 *   - "Multi-stage" evolution is classical 4-stage Runge-Kutta on the cell
 *     ODE dW/dsigma = L W, with S substeps per half step.
 *   - Point source (an extension: the paper evolves homogeneous problems):
 *     the forcing f = amp g(x) w(t) enters the vt equation as (tau h/c) f;
 *     its space and time Taylor coefficients about the cell centre and the
 *     half step's start join the series recursion. The spatial factor is a
 *     product of 1D Gaussians at the periodic nearest image, each cut to 0
 *     beyond 6 sigma; the wavelet is a Ricker wavelet.
 *
 * Array layout of a grid field: [d3][d2][d1][k][j][i], i (x1) fastest, the
 * tensor u[m3][m2][m1][n3][n2][n1] of Sec. 3.1. A two-field state is
 * [f][d3][d2][d1][k][j][i] with f = 0 for u and f = 1 for u_t.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* The oracle computes in FP64. The same source built with
 * -DORACLE_REAL='long double' gives a twin whose only purpose is to measure
 * how far FP64 rounding alone moves the FP64 build (the rounding floor that
 * any FP64 implementation of the method shares). */
#ifndef ORACLE_REAL
#define ORACLE_REAL double
#endif
typedef ORACLE_REAL real;

#define OR_MAXM 4
#define OR_MAXP (2 * OR_MAXM + 2)

/* binomial coefficient, small arguments */
static long double or_binom(int a, int b)
{
    if (b < 0 || b > a) return 0.0L;
    long double r = 1.0L;
    for (int i = 1; i <= b; ++i) r = r * (long double)(a - b + i) / (long double)i;
    return r;
}

/*
 * The 1D Hermite matrix H (Sec. 3.1; its construction is deferred by the
 * paper to its reference on Hermite method variations). With P = 2m+2,
 * H is the inverse of the confluent Vandermonde matrix V whose row
 * (side, k) holds the k-th Taylor coefficient, at xi = -1/2 (side 0) or
 * xi = +1/2 (side 1), of the monomial xi^j:  V[(side,k)][j] = C(j,k) xi^(j-k).
 * So b = H * data maps the scaled derivatives [L0..Lm, R0..Rm] of the two
 * end nodes to the monomial coefficients b_0..b_{2m+1} about the centre.
 * Gauss-Jordan elimination with partial pivoting in long double, rounded to
 * real at the end. H is row-major, H[j*P + r], r = side*(m+1) + k.
 * Returns 0, or -1 for m outside [1, 4].
 */
int oracle_hermite_matrix(int m, real *H)
{
    if (m < 1 || m > OR_MAXM) return -1;
    const int M = m + 1, P = 2 * m + 2;
    long double A[OR_MAXP][2 * OR_MAXP];
    for (int side = 0; side < 2; ++side) {
        const long double x = side ? 0.5L : -0.5L;
        for (int k = 0; k < M; ++k) {
            const int r = side * M + k;
            for (int j = 0; j < P; ++j) {
                long double v = 0.0L;
                if (j >= k) v = or_binom(j, k) * powl(x, (long double)(j - k));
                A[r][j] = v;
            }
            for (int j = 0; j < P; ++j) A[r][P + j] = (r == j) ? 1.0L : 0.0L;
        }
    }
    for (int col = 0; col < P; ++col) {
        int piv = col;
        for (int r = col + 1; r < P; ++r)
            if (fabsl(A[r][col]) > fabsl(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0L) return -2;
        if (piv != col)
            for (int j = 0; j < 2 * P; ++j) {
                long double t = A[col][j];
                A[col][j] = A[piv][j];
                A[piv][j] = t;
            }
        const long double d = A[col][col];
        for (int j = 0; j < 2 * P; ++j) A[col][j] /= d;
        for (int r = 0; r < P; ++r) {
            if (r == col || A[r][col] == 0.0L) continue;
            const long double f = A[r][col];
            for (int j = 0; j < 2 * P; ++j) A[r][j] -= f * A[col][j];
        }
    }
    /* A's right half is V^{-1}: rows are coefficient indices j, columns data r */
    for (int j = 0; j < P; ++j)
        for (int r = 0; r < P; ++r) H[j * P + r] = (real)A[j][P + r];
    return 0;
}

/*
 * Alg. 1 generalised to any axis: apply the P x P matrix H along one axis of
 * a P^3 tensor T[a3][a2][a1] (a1 fastest). axis 0 is x1, 1 is x2, 2 is x3.
 */
static void or_apply_axis(int P, const real *H, int axis, const real *in, real *out)
{
    for (int a3 = 0; a3 < P; ++a3)
        for (int a2 = 0; a2 < P; ++a2)
            for (int a1 = 0; a1 < P; ++a1) {
                int t = (axis == 0) ? a1 : (axis == 1) ? a2 : a3;
                real c = 0.0;
                for (int k = 0; k < P; ++k) {
                    int b1 = a1, b2 = a2, b3 = a3;
                    if (axis == 0) b1 = k;
                    else if (axis == 1) b2 = k;
                    else b3 = k;
                    c += H[t * P + k] * in[(b3 * P + b2) * P + b1];
                }
                out[(a3 * P + a2) * P + a1] = c;
            }
}

/*
 * Alg. 2: polynomial reconstruction of one cell. uloc is the local rank-3
 * tensor of the 8 vertices, uloc[a3][a2][a1] with a = side*(m+1) + derivative
 * order per axis; R receives the monomial coefficients R[j3][j2][j1] of the
 * interpolant in xi (Eq. 3).
 */
void oracle_interpolate_cell(int m, const real *H, const real *uloc, real *R)
{
    const int P = 2 * m + 2;
    real t1[OR_MAXP * OR_MAXP * OR_MAXP], t2[OR_MAXP * OR_MAXP * OR_MAXP];
    or_apply_axis(P, H, 0, uloc, t1);
    or_apply_axis(P, H, 1, t1, t2);
    or_apply_axis(P, H, 2, t2, R);
}

/*
 * Alg. 3 in the cell variable xi (h = 1 there): differentiate the coefficient
 * tensor along one axis, (D W)[j] = (j+1) W[j+1], zero at the top index.
 */
static void or_diff_axis(int P, int axis, const real *W, real *out)
{
    for (int j3 = 0; j3 < P; ++j3)
        for (int j2 = 0; j2 < P; ++j2)
            for (int j1 = 0; j1 < P; ++j1) {
                int t = (axis == 0) ? j1 : (axis == 1) ? j2 : j3;
                real v = 0.0;
                if (t < P - 1) {
                    int b1 = j1, b2 = j2, b3 = j3;
                    if (axis == 0) b1 = t + 1;
                    else if (axis == 1) b2 = t + 1;
                    else b3 = t + 1;
                    v = (real)(t + 1) * W[(b3 * P + b2) * P + b1];
                }
                out[(j3 * P + j2) * P + j1] = v;
            }
}

/* Laplacian in xi: sum over axes of Alg. 3 applied twice. */
void oracle_laplacian(int m, const real *W, real *out)
{
    const int P = 2 * m + 2, n3 = P * P * P;
    real d1[OR_MAXP * OR_MAXP * OR_MAXP], d2[OR_MAXP * OR_MAXP * OR_MAXP];
    for (int t = 0; t < n3; ++t) out[t] = 0.0;
    for (int axis = 0; axis < 3; ++axis) {
        or_diff_axis(P, axis, W, d1);
        or_diff_axis(P, axis, d1, d2);
        for (int t = 0; t < n3; ++t) out[t] += d2[t];
    }
}

/* The cell operator of the first-order system: L(a, b) = lam * (b, Lap a). */
static void or_apply_L(int m, real lam, const real *a, const real *b, real *la, real *lb)
{
    const int P = 2 * m + 2, n3 = P * P * P;
    oracle_laplacian(m, a, lb);
    for (int t = 0; t < n3; ++t) {
        la[t] = lam * b[t];
        lb[t] = lam * lb[t];
    }
}

/*
 * Alg. 4 for the wave system: Horner loop over k = q..1 of
 *   W <- R + (1/k) L W,
 * i.e. (Wu, Wv) <- (Ru + (lam/k) Wv, Rv + (lam/k) Lap Wu), both from the old W.
 * Ru, Rv are overwritten with the evolved coefficients at sigma = 1.
 */
void oracle_evolve_taylor(int m, int q, real lam, real *Ru, real *Rv)
{
    const int P = 2 * m + 2, n3 = P * P * P;
    real wu[OR_MAXP * OR_MAXP * OR_MAXP], wv[OR_MAXP * OR_MAXP * OR_MAXP];
    real lu[OR_MAXP * OR_MAXP * OR_MAXP], lv[OR_MAXP * OR_MAXP * OR_MAXP];
    memcpy(wu, Ru, sizeof(real) * n3);
    memcpy(wv, Rv, sizeof(real) * n3);
    for (int k = q; k >= 1; --k) {
        or_apply_L(m, lam, wu, wv, lu, lv);
        for (int t = 0; t < n3; ++t) {
            wu[t] = Ru[t] + lu[t] / (real)k;
            wv[t] = Rv[t] + lv[t] / (real)k;
        }
    }
    memcpy(Ru, wu, sizeof(real) * n3);
    memcpy(Rv, wv, sizeof(real) * n3);
}

/*
 * Classical 4-stage Runge-Kutta on dW/dsigma = L W over sigma in [0, 1] with
 * S equal substeps (the abstract's multi-stage local evolution).
 */
void oracle_evolve_rk4(int m, int S, real lam, real *Ru, real *Rv)
{
    const int P = 2 * m + 2, n3 = P * P * P;
    const real dl = 1.0 / (real)S;
    real k1u[OR_MAXP * OR_MAXP * OR_MAXP], k1v[OR_MAXP * OR_MAXP * OR_MAXP];
    real k2u[OR_MAXP * OR_MAXP * OR_MAXP], k2v[OR_MAXP * OR_MAXP * OR_MAXP];
    real k3u[OR_MAXP * OR_MAXP * OR_MAXP], k3v[OR_MAXP * OR_MAXP * OR_MAXP];
    real k4u[OR_MAXP * OR_MAXP * OR_MAXP], k4v[OR_MAXP * OR_MAXP * OR_MAXP];
    real yu[OR_MAXP * OR_MAXP * OR_MAXP], yv[OR_MAXP * OR_MAXP * OR_MAXP];
    for (int s = 0; s < S; ++s) {
        or_apply_L(m, lam, Ru, Rv, k1u, k1v);
        for (int t = 0; t < n3; ++t) { yu[t] = Ru[t] + 0.5 * dl * k1u[t]; yv[t] = Rv[t] + 0.5 * dl * k1v[t]; }
        or_apply_L(m, lam, yu, yv, k2u, k2v);
        for (int t = 0; t < n3; ++t) { yu[t] = Ru[t] + 0.5 * dl * k2u[t]; yv[t] = Rv[t] + 0.5 * dl * k2v[t]; }
        or_apply_L(m, lam, yu, yv, k3u, k3v);
        for (int t = 0; t < n3; ++t) { yu[t] = Ru[t] + dl * k3u[t]; yv[t] = Rv[t] + dl * k3v[t]; }
        or_apply_L(m, lam, yu, yv, k4u, k4v);
        for (int t = 0; t < n3; ++t) {
            Ru[t] += dl / 6.0 * (k1u[t] + 2.0 * k2u[t] + 2.0 * k3u[t] + k4u[t]);
            Rv[t] += dl / 6.0 * (k1v[t] + 2.0 * k2v[t] + 2.0 * k3v[t] + k4v[t]);
        }
    }
}

/*
 * Gather the local tensor of the cell whose lower corner is node (i, j, k) of
 * a periodic grid field g[d3][d2][d1][k][j][i] (Sec. 3.1: the (m+1)^3 values
 * of each of the 8 vertices). uloc[a3][a2][a1], a = side*(m+1) + d.
 */
void oracle_gather_cell(int n, int m, const real *g, int i, int j, int k, real *uloc)
{
    const int M = m + 1, P = 2 * M;
    const long nn = (long)n * n * n;
    for (int s3 = 0; s3 < 2; ++s3)
        for (int s2 = 0; s2 < 2; ++s2)
            for (int s1 = 0; s1 < 2; ++s1) {
                const long node = ((long)((k + s3) % n) * n + (j + s2) % n) * n + (i + s1) % n;
                for (int d3 = 0; d3 < M; ++d3)
                    for (int d2 = 0; d2 < M; ++d2)
                        for (int d1 = 0; d1 < M; ++d1) {
                            const long src = (long)((d3 * M + d2) * M + d1) * nn + node;
                            const int a1 = s1 * M + d1, a2 = s2 * M + d2, a3 = s3 * M + d3;
                            uloc[(a3 * P + a2) * P + a1] = g[src];
                        }
            }
}

/* evo: 0 = Taylor (param = q), 1 = RK4 (param = substeps S) */
static void or_evolve(int m, int evo, int param, real lam, real *Ru, real *Rv)
{
    if (evo == 0) oracle_evolve_taylor(m, param, lam, Ru, Rv);
    else oracle_evolve_rk4(m, param, lam, Ru, Rv);
}

/*
 * One half step on a periodic grid (Sec. 2): for every cell of the source grid
 * interpolate (Alg. 2), evolve through the half step (Alg. 4 or RK4) and keep
 * the coefficients with every index <= m as the data of the node at the cell
 * centre on the other grid. src and dst hold two fields, [f][M^3][n^3], in the
 * internal variables (u, vt). to_dual = 1: primal -> dual, the cell with lower
 * corner (i,j,k) writes dual (i,j,k); to_dual = 0: dual -> primal, writes
 * primal (i+1, j+1, k+1) mod n.
 */
void oracle_half_step(int n, int m, const real *H, real lam, int evo, int param,
                      const real *src, real *dst, int to_dual)
{
    const int M = m + 1, P = 2 * M, M3 = M * M * M;
    const long nn = (long)n * n * n;
    const int off = to_dual ? 0 : 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j) {
            real uloc[OR_MAXP * OR_MAXP * OR_MAXP], vloc[OR_MAXP * OR_MAXP * OR_MAXP];
            real Ru[OR_MAXP * OR_MAXP * OR_MAXP], Rv[OR_MAXP * OR_MAXP * OR_MAXP];
            for (int i = 0; i < n; ++i) {
                oracle_gather_cell(n, m, src, i, j, k, uloc);
                oracle_gather_cell(n, m, src + (long)M3 * nn, i, j, k, vloc);
                oracle_interpolate_cell(m, H, uloc, Ru);
                oracle_interpolate_cell(m, H, vloc, Rv);
                or_evolve(m, evo, param, lam, Ru, Rv);
                const long node = ((long)((k + off) % n) * n + (j + off) % n) * n + (i + off) % n;
                for (int d3 = 0; d3 < M; ++d3)
                    for (int d2 = 0; d2 < M; ++d2)
                        for (int d1 = 0; d1 < M; ++d1) {
                            const int dd = (d3 * M + d2) * M + d1;
                            const int jj = (d3 * P + d2) * P + d1;
                            dst[(long)dd * nn + node] = Ru[jj];
                            dst[(long)(M3 + dd) * nn + node] = Rv[jj];
                        }
            }
        }
}

/*
 * Full run: u and ut (scaled derivatives of u and u_t on the primal grid,
 * each [M^3][n^3]) are advanced by nsteps full steps in place. dt = cfl*h/c,
 * tau = dt/2, lam = c*tau/h. Returns 0, or a negative value on bad input.
 */
int oracle_run(int n, int m, real cfl, real c, int evo, int param, int nsteps,
               real *u, real *ut)
{
    if (n < 1 || m < 1 || m > OR_MAXM || !(cfl > 0.0) || !(c > 0.0) || nsteps < 0 || param < 1)
        return -1;
    const int M = m + 1, P = 2 * M, M3 = M * M * M;
    const long nn = (long)n * n * n, sz = (long)M3 * nn;
    const real h = 1.0 / (real)n;
    const real dt = cfl * h / c, tau = 0.5 * dt, lam = c * tau / h;
    real H[OR_MAXP * OR_MAXP];
    if (oracle_hermite_matrix(m, H) != 0) return -2;
    (void)P;
    real *a = (real *)malloc(sizeof(real) * 2 * sz);
    real *b = (real *)malloc(sizeof(real) * 2 * sz);
    if (!a || !b) { free(a); free(b); return -3; }
    for (long t = 0; t < sz; ++t) { a[t] = u[t]; a[sz + t] = (h / c) * ut[t]; }
    for (int s = 0; s < nsteps; ++s) {
        oracle_half_step(n, m, H, lam, evo, param, a, b, 1);
        oracle_half_step(n, m, H, lam, evo, param, b, a, 0);
    }
    for (long t = 0; t < sz; ++t) { u[t] = a[t]; ut[t] = (c / h) * a[sz + t]; }
    free(a);
    free(b);
    return 0;
}

/*
 * Local (non-periodic) dependency cone of one primal node after nsteps full
 * steps, for sampled checks of large grids: the node after nsteps full steps
 * depends only on the w^3 primal nodes around it, w = 2*nsteps+1. box and
 * vbox hold those nodes of u and u_t, laid out [d3][d2][d1][z][y][x] with the
 * target node at the centre (x = y = z = nsteps). n sets h = 1/n. Runs the
 * same cell algorithm on the shrinking box and returns the node's 2*M^3
 * values, u then u_t.
 */
int oracle_point_box(int n, int m, real cfl, real c, int evo, int param, int nsteps,
                     const real *ubox, const real *utbox, real *out)
{
    if (n < 1 || m < 1 || m > OR_MAXM || nsteps < 1 || param < 1) return -1;
    const int M = m + 1, P = 2 * M, M3 = M * M * M;
    const real h = 1.0 / (real)n;
    const real dt = cfl * h / c, tau = 0.5 * dt, lam = c * tau / h;
    real H[OR_MAXP * OR_MAXP];
    if (oracle_hermite_matrix(m, H) != 0) return -2;
    int w = 2 * nsteps + 1;
    const long w3 = (long)w * w * w;
    real *box = (real *)malloc(sizeof(real) * 2 * M3 * w3);
    if (!box) return -3;
    for (long t = 0; t < (long)M3 * w3; ++t) {
        box[t] = ubox[t];
        box[(long)M3 * w3 + t] = (h / c) * utbox[t];
    }
    for (int hs = 0; hs < 2 * nsteps; ++hs) {
        const int wn = w - 1;
        real *nb = (real *)malloc(sizeof(real) * 2 * M3 * (long)wn * wn * wn);
        if (!nb) { free(box); return -3; }
        for (int z = 0; z < wn; ++z)
            for (int y = 0; y < wn; ++y)
                for (int x = 0; x < wn; ++x) {
                    real uloc[OR_MAXP * OR_MAXP * OR_MAXP], vloc[OR_MAXP * OR_MAXP * OR_MAXP];
                    for (int f = 0; f < 2; ++f) {
                        real *loc = f ? vloc : uloc;
                        for (int s3 = 0; s3 < 2; ++s3)
                            for (int s2 = 0; s2 < 2; ++s2)
                                for (int s1 = 0; s1 < 2; ++s1)
                                    for (int d3 = 0; d3 < M; ++d3)
                                        for (int d2 = 0; d2 < M; ++d2)
                                            for (int d1 = 0; d1 < M; ++d1) {
                                                int dd = (d3 * M + d2) * M + d1;
                                                long sidx = (((long)(f * M3 + dd) * w + z + s3) * w + y + s2) * w + x + s1;
                                                loc[((s3 * M + d3) * P + s2 * M + d2) * P + s1 * M + d1] = box[sidx];
                                            }
                    }
                    real Ru[OR_MAXP * OR_MAXP * OR_MAXP], Rv[OR_MAXP * OR_MAXP * OR_MAXP];
                    oracle_interpolate_cell(m, H, uloc, Ru);
                    oracle_interpolate_cell(m, H, vloc, Rv);
                    or_evolve(m, evo, param, lam, Ru, Rv);
                    for (int d3 = 0; d3 < M; ++d3)
                        for (int d2 = 0; d2 < M; ++d2)
                            for (int d1 = 0; d1 < M; ++d1) {
                                int dd = (d3 * M + d2) * M + d1, jj = (d3 * P + d2) * P + d1;
                                nb[(((long)dd * wn + z) * wn + y) * wn + x] = Ru[jj];
                                nb[(((long)(M3 + dd) * wn + z) * wn + y) * wn + x] = Rv[jj];
                            }
                }
        free(box);
        box = nb;
        w = wn;
    }
    /* w == 1: the remaining node is the target primal node */
    for (int dd = 0; dd < M3; ++dd) {
        out[dd] = box[dd];
        out[M3 + dd] = (c / h) * box[M3 + dd];
    }
    free(box);
    return 0;
}

/* oracle_point_box on a full periodic grid: extracts the box around primal
 * node (i0, j0, k0) (periodic wrap) and runs it. */
int oracle_point(int n, int m, real cfl, real c, int evo, int param, int nsteps,
                 const real *u, const real *ut, int i0, int j0, int k0, real *out)
{
    if (n < 1 || m < 1 || m > OR_MAXM || nsteps < 1 || param < 1) return -1;
    const int M = m + 1, M3 = M * M * M;
    const long nn = (long)n * n * n;
    const int w = 2 * nsteps + 1;
    const long w3 = (long)w * w * w;
    real *ub = (real *)malloc(sizeof(real) * M3 * w3);
    real *vb = (real *)malloc(sizeof(real) * M3 * w3);
    if (!ub || !vb) { free(ub); free(vb); return -3; }
    for (int dd = 0; dd < M3; ++dd)
        for (int z = 0; z < w; ++z)
            for (int y = 0; y < w; ++y)
                for (int x = 0; x < w; ++x) {
                    int gi = ((i0 - nsteps + x) % n + n) % n;
                    int gj = ((j0 - nsteps + y) % n + n) % n;
                    int gk = ((k0 - nsteps + z) % n + n) % n;
                    long g = (long)dd * nn + ((long)gk * n + gj) * n + gi;
                    long b = (((long)dd * w + z) * w + y) * w + x;
                    ub[b] = u[g];
                    vb[b] = ut[g];
                }
    int rc = oracle_point_box(n, m, cfl, c, evo, param, nsteps, ub, vb, out);
    free(ub);
    free(vb);
    return rc;
}

/* ------------------------------------------------------------------------
 * Forced wave equation u_tt = c^2 Lap u + f, f(x, t) = amp g(x) w(t), with g a
 * unit-mass Gaussian of standard deviation sigma around a source point and w
 * a Ricker wavelet (1 - 2 beta s^2) exp(-beta s^2), s = t - t0,
 * beta = (pi f0)^2. (Extension of Sec. 2: the Taylor series of the cell
 * solution now also carries the forcing.) For tests, sigma <= 0 stands for a
 * spatially uniform g = 1.
 * ------------------------------------------------------------------------ */

/* Taylor coefficients e_k, k < K, of exp(p0 + p1 t + p2 t^2) about t = 0,
 * from (k+1) e_{k+1} = p1 e_k + 2 p2 e_{k-1} (the derivative of the
 * exponent times the series). */
static void or_exp_quadratic_series(real p0, real p1, real p2, int K, real *e)
{
    e[0] = exp(p0);
    for (int k = 0; k + 1 < K; ++k) {
        real v = p1 * e[k];
        if (k >= 1) v += 2.0 * p2 * e[k - 1];
        e[k + 1] = v / (real)(k + 1);
    }
}

/* Scaled Taylor coefficients h^a/a! g1^(a) of the 1D Gaussian factor
 * g1(x) = exp(-(x - s)^2 / (2 sigma^2)) / (sigma sqrt(2 pi)) at the point
 * whose nearest-image offset from s is d: the Taylor series of
 * g1(x_c + h xi) in xi. Zero beyond 6 sigma. */
int oracle_gauss_taylor(real d, real sigma, real h, int K, real *g)
{
    if (K < 1 || K > 64) return -1;
    if (sigma <= 0.0) {
        for (int a = 0; a < K; ++a) g[a] = (a == 0) ? 1.0 : 0.0;
        return 0;
    }
    if (fabs(d) > 6.0 * sigma) {
        for (int a = 0; a < K; ++a) g[a] = 0.0;
        return 0;
    }
    const real s2 = 2.0 * sigma * sigma;
    or_exp_quadratic_series(-d * d / s2, -2.0 * d * h / s2, -h * h / s2, K, g);
    const real norm = 1.0 / (sigma * sqrt(2.0 * 3.14159265358979323846264338327950288L));
    for (int a = 0; a < K; ++a) g[a] *= norm;
    return 0;
}

/* Time Taylor coefficients w_k = tau^k/k! w^(k)(ta) of the Ricker wavelet,
 * k < K: the series of (1 + 2 phi(sig)) exp(phi(sig)) with
 * phi(sig) = -beta (ta - t0 + tau sig)^2. */
int oracle_ricker_taylor(real ta, real tau, real f0, real t0, int K, real *w)
{
    if (K < 1 || K > 64) return -1;
    const real pi = 3.14159265358979323846264338327950288L;
    const real beta = pi * pi * f0 * f0, s = ta - t0;
    const real p0 = -beta * s * s, p1 = -2.0 * beta * s * tau, p2 = -beta * tau * tau;
    real e[66];
    or_exp_quadratic_series(p0, p1, p2, K, e);
    for (int k = 0; k < K; ++k) {
        real v = (1.0 + 2.0 * p0) * e[k];
        if (k >= 1) v += 2.0 * p1 * e[k - 1];
        if (k >= 2) v += 2.0 * p2 * e[k - 2];
        w[k] = v;
    }
    return 0;
}

/*
 * Forced Taylor evolution of one cell over the half step, by the forward
 * recursion of the series: W_0 = (Ru, Rv) and for s = 1..q
 *   W_s = (L W_{s-1} + (0, wk[s-1] G)) / s,
 * with L(a, b) = lam (b, Lap a); the result sum_{s<=q} W_s overwrites Ru, Rv.
 * G[j3][j2][j1] is the forcing polynomial of the cell in xi, already scaled
 * to the vt equation; wk holds q time coefficients.
 */
void oracle_evolve_taylor_forced(int m, int q, real lam, real *Ru, real *Rv, const real *G, const real *wk)
{
    const int P = 2 * m + 2, n3 = P * P * P;
    real wu[OR_MAXP * OR_MAXP * OR_MAXP], wv[OR_MAXP * OR_MAXP * OR_MAXP];
    real lu[OR_MAXP * OR_MAXP * OR_MAXP], lv[OR_MAXP * OR_MAXP * OR_MAXP];
    memcpy(wu, Ru, sizeof(real) * n3);
    memcpy(wv, Rv, sizeof(real) * n3);
    for (int s = 1; s <= q; ++s) {
        or_apply_L(m, lam, wu, wv, lu, lv);
        for (int t = 0; t < n3; ++t) {
            wu[t] = lu[t] / (real)s;
            wv[t] = (lv[t] + wk[s - 1] * G[t]) / (real)s;
            Ru[t] += wu[t];
            Rv[t] += wv[t];
        }
    }
}

/* One forced half step (as oracle_half_step, Taylor with q stages), the half
 * step starting at time ta. Cell centres: (i + 1/2) h on the primal grid's
 * cells (to_dual = 1), (i + 1) h on the dual grid's (to_dual = 0). */
static void or_half_step_forced(int n, int m, const real *H, real lam, int q, const real *src, real *dst,
                                int to_dual, real h, real tau, real c, real ta, const real *sx, real sigma,
                                real f0, real t0, real amp)
{
    const int M = m + 1, P = 2 * M, M3 = M * M * M;
    const long nn = (long)n * n * n;
    const int off = to_dual ? 0 : 1;
    real wk[64];
    oracle_ricker_taylor(ta, tau, f0, t0, q, wk);
    const real fscale = amp * tau * h / c;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j) {
            real uloc[OR_MAXP * OR_MAXP * OR_MAXP], vloc[OR_MAXP * OR_MAXP * OR_MAXP];
            real Ru[OR_MAXP * OR_MAXP * OR_MAXP], Rv[OR_MAXP * OR_MAXP * OR_MAXP];
            real G[OR_MAXP * OR_MAXP * OR_MAXP];
            for (int i = 0; i < n; ++i) {
                oracle_gather_cell(n, m, src, i, j, k, uloc);
                oracle_gather_cell(n, m, src + (long)M3 * nn, i, j, k, vloc);
                oracle_interpolate_cell(m, H, uloc, Ru);
                oracle_interpolate_cell(m, H, vloc, Rv);
                const int idx[3] = {i, j, k};
                real g1[3][OR_MAXP];
                for (int x = 0; x < 3; ++x) {
                    real d = ((real)idx[x] + 0.5 + (to_dual ? 0.0 : 0.5)) * h - sx[x];
                    d -= floor(d + 0.5);
                    oracle_gauss_taylor(d, sigma, h, P, g1[x]);
                }
                for (int a3 = 0; a3 < P; ++a3)
                    for (int a2 = 0; a2 < P; ++a2)
                        for (int a1 = 0; a1 < P; ++a1)
                            G[(a3 * P + a2) * P + a1] = fscale * g1[0][a1] * g1[1][a2] * g1[2][a3];
                oracle_evolve_taylor_forced(m, q, lam, Ru, Rv, G, wk);
                const long node = ((long)((k + off) % n) * n + (j + off) % n) * n + (i + off) % n;
                for (int d3 = 0; d3 < M; ++d3)
                    for (int d2 = 0; d2 < M; ++d2)
                        for (int d1 = 0; d1 < M; ++d1) {
                            const int dd = (d3 * M + d2) * M + d1;
                            const int jj = (d3 * P + d2) * P + d1;
                            dst[(long)dd * nn + node] = Ru[jj];
                            dst[(long)(M3 + dd) * nn + node] = Rv[jj];
                        }
            }
        }
}

/* Forced run: as oracle_run with Taylor evolution (q stages) and the point
 * source (sx, sigma, f0, t0, amp); the first half step starts at t = 0. */
int oracle_run_forced(int n, int m, real cfl, real c, int q, int nsteps, real *u, real *ut, const real *sx,
                      real sigma, real f0, real t0, real amp)
{
    if (n < 1 || m < 1 || m > OR_MAXM || !(cfl > 0.0) || !(c > 0.0) || nsteps < 0 || q < 1 || q > 64)
        return -1;
    const int M = m + 1, M3 = M * M * M;
    const long nn = (long)n * n * n, sz = (long)M3 * nn;
    const real h = 1.0 / (real)n;
    const real dt = cfl * h / c, tau = 0.5 * dt, lam = c * tau / h;
    real H[OR_MAXP * OR_MAXP];
    if (oracle_hermite_matrix(m, H) != 0) return -2;
    real *a = (real *)malloc(sizeof(real) * 2 * sz);
    real *b = (real *)malloc(sizeof(real) * 2 * sz);
    if (!a || !b) { free(a); free(b); return -3; }
    for (long t = 0; t < sz; ++t) { a[t] = u[t]; a[sz + t] = (h / c) * ut[t]; }
    for (int s = 0; s < nsteps; ++s) {
        const real tn = (real)s * dt;
        or_half_step_forced(n, m, H, lam, q, a, b, 1, h, tau, c, tn, sx, sigma, f0, t0, amp);
        or_half_step_forced(n, m, H, lam, q, b, a, 0, h, tau, c, tn + tau, sx, sigma, f0, t0, amp);
    }
    for (long t = 0; t < sz; ++t) { u[t] = a[t]; ut[t] = (c / h) * a[sz + t]; }
    free(a);
    free(b);
    return 0;
}

/* ------------------------------------------------------------------------
 * Advection (Sec. 2, Eq. 1), the equation the paper measures: one field with
 * the scaled derivatives of order <= m per axis at every node, on the same
 * primal/dual grids. Here with a speed c: u_t = c (u_x1 + u_x2 + u_x3), c = 1
 * being the paper's equation. In the cell variable xi and the half-step time
 * sigma = (t - t_n)/tau the equation reads u_sigma = lam (sum_x d/dxi_x) u
 * with lam = c tau / h, so the Cauchy-Kovalevskaya recursion of Eq. 5 (its
 * Delta t read as the half step, as for the wave system) is
 *   b_{j, s+1} = lam / (s + 1) sum_x (j_x + 1) b_{j + e_x, s},
 * and the q-stage Horner loop of Alg. 4 sums the series at sigma = 1. The
 * stage count q = 3(2m+1) of Sec. 3.2 is exact for this equation.
 * ------------------------------------------------------------------------ */

/* Sum over the three axes of Alg. 3: (G W)[j] = sum_x (j_x + 1) W[j + e_x]. */
static void or_grad_sum(int P, const real *W, real *out)
{
    const int n3 = P * P * P;
    real d[OR_MAXP * OR_MAXP * OR_MAXP];
    for (int t = 0; t < n3; ++t) out[t] = 0.0;
    for (int axis = 0; axis < 3; ++axis) {
        or_diff_axis(P, axis, W, d);
        for (int t = 0; t < n3; ++t) out[t] += d[t];
    }
}

/* Alg. 4 for advection: W <- R + (lam / k) G W for k = q .. 1. */
void oracle_evolve_advection(int m, int q, real lam, real *R)
{
    const int P = 2 * m + 2, n3 = P * P * P;
    real w[OR_MAXP * OR_MAXP * OR_MAXP], g[OR_MAXP * OR_MAXP * OR_MAXP];
    memcpy(w, R, sizeof(real) * n3);
    for (int k = q; k >= 1; --k) {
        or_grad_sum(P, w, g);
        for (int t = 0; t < n3; ++t) w[t] = R[t] + (lam / (real)k) * g[t];
    }
    memcpy(R, w, sizeof(real) * n3);
}

/* One advection half step over the whole grid (one field of (m+1)^3 columns). */
void oracle_half_step_advection(int n, int m, const real *H, real lam, int q, const real *src, real *dst,
                                int to_dual)
{
    const int M = m + 1, P = 2 * M;
    const int off = to_dual ? 0 : 1;
    const long nn = (long)n * n * n;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j) {
            real uloc[OR_MAXP * OR_MAXP * OR_MAXP], R[OR_MAXP * OR_MAXP * OR_MAXP];
            for (int i = 0; i < n; ++i) {
                oracle_gather_cell(n, m, src, i, j, k, uloc);
                oracle_interpolate_cell(m, H, uloc, R);
                oracle_evolve_advection(m, q, lam, R);
                const long node = ((long)((k + off) % n) * n + (j + off) % n) * n + (i + off) % n;
                for (int d3 = 0; d3 < M; ++d3)
                    for (int d2 = 0; d2 < M; ++d2)
                        for (int d1 = 0; d1 < M; ++d1)
                            dst[(long)((d3 * M + d2) * M + d1) * nn + node] = R[(d3 * P + d2) * P + d1];
            }
        }
}

/* nsteps full advection steps of the primal-grid field u ((m+1)^3 n^3
 * values, layout of oracle_run), dt = cfl h / c. */
int oracle_run_advection(int n, int m, real cfl, real c, int q, int nsteps, real *u)
{
    if (n < 1 || m < 1 || m > OR_MAXM || !(cfl > 0.0) || !(c > 0.0) || nsteps < 0 || q < 1 || q > 64)
        return -1;
    const int M = m + 1, M3 = M * M * M;
    const long sz = (long)M3 * n * n * n;
    const real h = 1.0 / (real)n;
    const real dt = cfl * h / c, tau = 0.5 * dt, lam = c * tau / h;
    real H[OR_MAXP * OR_MAXP];
    if (oracle_hermite_matrix(m, H) != 0) return -2;
    real *b = (real *)malloc(sizeof(real) * sz);
    if (!b) return -3;
    for (int s = 0; s < nsteps; ++s) {
        oracle_half_step_advection(n, m, H, lam, q, u, b, 1);
        oracle_half_step_advection(n, m, H, lam, q, b, u, 0);
    }
    free(b);
    return 0;
}

/* ------------------------------------------------------------------------
 * Adjoint (transpose) of the wave half step, for gradients of a misfit of
 * receiver traces (an extension: the paper has no adjoint). A half step is
 * linear: new = T E I G old (gather of the 8 vertices, interpolation,
 * evolution polynomial, truncation to j <= m), so its transpose is
 * G^T I^T E^T T^T: zero-pad the new node's data to the P^3 coefficients,
 * apply E^T = sum_s c_s (L^T)^s with L^T(a, b) = lam (Lap^T b, a), apply H^T
 * along each axis, and add the result into the 8 vertices. Each factor is
 * the plain transposed loop of the forward step.
 * ------------------------------------------------------------------------ */

/* Lap^T: out[j + 2 e_x] += (j_x + 1)(j_x + 2) V[j], the transpose of the
 * coefficient Laplacian of oracle_laplacian. */
static void or_laplacian_T(int P, const real *V, real *out)
{
    const int n3 = P * P * P;
    for (int t = 0; t < n3; ++t) out[t] = 0.0;
    for (int j3 = 0; j3 < P; ++j3)
        for (int j2 = 0; j2 < P; ++j2)
            for (int j1 = 0; j1 < P; ++j1) {
                const real v = V[(j3 * P + j2) * P + j1];
                if (j1 + 2 < P) out[(j3 * P + j2) * P + j1 + 2] += (real)((j1 + 1) * (j1 + 2)) * v;
                if (j2 + 2 < P) out[(j3 * P + j2 + 2) * P + j1] += (real)((j2 + 1) * (j2 + 2)) * v;
                if (j3 + 2 < P) out[((j3 + 2) * P + j2) * P + j1] += (real)((j3 + 1) * (j3 + 2)) * v;
            }
}

/* E^T of the q-stage Taylor evolution, by the Horner loop with L^T. */
void oracle_evolve_taylor_T(int m, int q, real lam, real *Gu, real *Gv)
{
    const int P = 2 * m + 2, n3 = P * P * P;
    real wu[OR_MAXP * OR_MAXP * OR_MAXP], wv[OR_MAXP * OR_MAXP * OR_MAXP], lt[OR_MAXP * OR_MAXP * OR_MAXP];
    memcpy(wu, Gu, sizeof(real) * n3);
    memcpy(wv, Gv, sizeof(real) * n3);
    for (int k = q; k >= 1; --k) {
        or_laplacian_T(P, wv, lt);  /* L^T (wu, wv) = lam (Lap^T wv, wu) */
        for (int t = 0; t < n3; ++t) {
            const real nu = Gu[t] + (lam / (real)k) * lt[t];
            const real nv = Gv[t] + (lam / (real)k) * wu[t];
            wu[t] = nu;
            wv[t] = nv;
        }
    }
    memcpy(Gu, wu, sizeof(real) * n3);
    memcpy(Gv, wv, sizeof(real) * n3);
}

/* Transpose of oracle_interpolate_cell: H^T along x3, x2, x1. */
void oracle_interpolate_cell_T(int m, const real *H, const real *R, real *uloc)
{
    const int P = 2 * m + 2;
    real Ht[OR_MAXP * OR_MAXP], t1[OR_MAXP * OR_MAXP * OR_MAXP], t2[OR_MAXP * OR_MAXP * OR_MAXP];
    for (int a = 0; a < P; ++a)
        for (int b = 0; b < P; ++b) Ht[a * P + b] = H[b * P + a];
    or_apply_axis(P, Ht, 2, R, t1);
    or_apply_axis(P, Ht, 1, t1, t2);
    or_apply_axis(P, Ht, 0, t2, uloc);
}

/* Transpose of one Taylor half step (oracle_half_step with evo = Taylor):
 * lam_dst holds the adjoint of the destination grid (two fields), lam_src
 * receives the adjoint of the source grid. Serial over cells (the
 * scatter-add into shared vertices stays race-free and in a fixed order). */
void oracle_adjoint_half_step(int n, int m, const real *H, real lam, int q, const real *lam_dst, real *lam_src,
                              int to_dual)
{
    const int M = m + 1, P = 2 * M, M3 = M * M * M, n3 = P * P * P;
    const long nn = (long)n * n * n;
    const int off = to_dual ? 0 : 1;
    for (long t = 0; t < 2 * (long)M3 * nn; ++t) lam_src[t] = 0.0;
    real Gu[OR_MAXP * OR_MAXP * OR_MAXP], Gv[OR_MAXP * OR_MAXP * OR_MAXP];
    real lu[OR_MAXP * OR_MAXP * OR_MAXP], lv[OR_MAXP * OR_MAXP * OR_MAXP];
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const long node = ((long)((k + off) % n) * n + (j + off) % n) * n + (i + off) % n;
                for (int t = 0; t < n3; ++t) Gu[t] = Gv[t] = 0.0;
                for (int d3 = 0; d3 < M; ++d3)
                    for (int d2 = 0; d2 < M; ++d2)
                        for (int d1 = 0; d1 < M; ++d1) {
                            const int dd = (d3 * M + d2) * M + d1, jj = (d3 * P + d2) * P + d1;
                            Gu[jj] = lam_dst[(long)dd * nn + node];
                            Gv[jj] = lam_dst[(long)(M3 + dd) * nn + node];
                        }
                oracle_evolve_taylor_T(m, q, lam, Gu, Gv);
                oracle_interpolate_cell_T(m, H, Gu, lu);
                oracle_interpolate_cell_T(m, H, Gv, lv);
                /* transpose of oracle_gather_cell: add into the 8 vertices */
                for (int a3 = 0; a3 < P; ++a3)
                    for (int a2 = 0; a2 < P; ++a2)
                        for (int a1 = 0; a1 < P; ++a1) {
                            const int s1 = a1 / M, d1 = a1 % M, s2 = a2 / M, d2 = a2 % M, s3 = a3 / M, d3 = a3 % M;
                            const long vn = ((long)((k + s3) % n) * n + (j + s2) % n) * n + (i + s1) % n;
                            const int dd = (d3 * M + d2) * M + d1, a = (a3 * P + a2) * P + a1;
                            lam_src[(long)dd * nn + vn] += lu[a];
                            lam_src[(long)(M3 + dd) * nn + vn] += lv[a];
                        }
            }
}

/* The source term of one half step alone: the forced half step applied to
 * zero data (internal scaled variables, two fields, to the other grid). */
int oracle_source_term(int n, int m, real cfl, real c, int q, int to_dual, real ta, const real *sx, real sigma,
                       real f0, real t0, real amp, real *out)
{
    if (n < 1 || m < 1 || m > OR_MAXM || !(cfl > 0.0) || !(c > 0.0) || q < 1 || q > 64) return -1;
    const int M = m + 1, M3 = M * M * M;
    const long sz = 2 * (long)M3 * n * n * n;
    const real h = 1.0 / (real)n, dt = cfl * h / c, tau = 0.5 * dt, lam = c * tau / h;
    real H[OR_MAXP * OR_MAXP];
    if (oracle_hermite_matrix(m, H) != 0) return -2;
    real *zero = (real *)calloc((size_t)sz, sizeof(real));
    if (!zero) return -3;
    or_half_step_forced(n, m, H, lam, q, zero, out, to_dual, h, tau, c, ta, sx, sigma, f0, t0, amp);
    free(zero);
    return 0;
}
