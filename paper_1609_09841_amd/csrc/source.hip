// Point-source forcing of the Hermite half step: u_tt = c^2 Lap u + f with
// f(x, t) = a g(x) w(t), g a unit-mass Gaussian of standard deviation sigma
// around x_s and w a Ricker wavelet.
//
// The half step is linear, so its forced result is the unforced one plus the
// particular solution P of the forced cell system with zero initial data. In
// the cell variables (xi, sigma) the system reads
//   u_sigma = lam vt,   vt_sigma = lam Lap_xi u + (tau h / c) f,
// and with f = a sum_b g_b xi^b sum_k w_k sigma^k (g_b: scaled Taylor
// coefficients of g at the cell centre, degree <= 2m+1 per axis; w_k: time
// Taylor coefficients of w over the half step, k < q) the Taylor series of P
// to order q gives
//   P_u = sum_i A_i Lap^i G,   P_vt = sum_i B_i Lap^i G,   G = a sum_b g_b xi^b,
// with the scalars
//   A_i = (tau h / c) sum_{k + 2 + 2i <= q} w_k k! / (k + 2 + 2i)! lam^(2i+1),
//   B_i = (tau h / c) sum_{k + 1 + 2i <= q} w_k k! / (k + 1 + 2i)! lam^(2i).
// On monomial coefficients (Lap^i G)_j = sum_{|e| = i} i!/(e1! e2! e3!)
// prod_x (j_x + 2 e_x)!/j_x! G_{j + 2e}. The kernel adds P_j, j <= m, to the
// new node of every cell within 6 sigma of the source (periodic nearest image
// per axis; beyond 6 sigma along any axis g is taken as 0).
//
// Per half step two launches serve every source of one order m: a small
// kernel forms each source's w_k, A_i and B_i from the half step's start
// time, read from the source's device-side step clock (so a captured graph
// replays with fixed arguments) or given by the host; then the main kernel,
// whose blocks are dealt to the sources by a prefix table, runs one thread
// per (box cell, j3).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch_common.h"
#include "kernels.h"

namespace hermite {
namespace {

constexpr int kMaxQ = 64;  // Taylor stages
constexpr int kThreads = 256;

// Time Taylor coefficients w_k = tau^k/k! w^(k)(ta), k < K, of the Ricker
// wavelet w = (1 - 2 beta s^2) exp(-beta s^2), s = t - t0, beta = (pi f0)^2.
// With z = sqrt(2 beta) s, w = -He_2(z) exp(-z^2/2), and since
// d/dz [He_n(z) exp(-z^2/2)] = -He_{n+1}(z) exp(-z^2/2),
// w^(k) = -(-sqrt(2 beta))^k He_{k+2}(z) exp(-z^2/2) (He: probabilists'
// Hermite polynomials, He_{n+1} = z He_n - n He_{n-1}).
__device__ void ricker_series(double ta, double tau, double f0, double t0, int K, double* w) {
    const double r = 1.4142135623730951 * 3.141592653589793 * f0;  // sqrt(2 beta)
    const double z = r * (ta - t0);
    const double g = exp(-0.5 * z * z);
    double hprev = 1.0, h = z, scale = 1.0;  // He_0, He_1; (-r tau)^k / k!
    for (int n = 1; n <= K; ++n) {
        const double nxt = z * h - (double)n * hprev;
        hprev = h;
        h = nxt;  // He_{n+1} = He_{k+2}, k = n - 1
        const int k = n - 1;
        if (k > 0) scale *= -r * tau / (double)k;
        w[k] = -scale * h * g;
    }
}

// Scalars of one half step, out[e][0][i] = A_i i!, out[e][1][i] = B_i i!
// (i <= 3m): one thread per (source e, i).
// use_series = 0: the unit-series source term (amplitude gradients).
__global__ void source_scalars_kernel(const SourceDesc* __restrict__ srcs, uint32_t ns, uint32_t from,
                                      int64_t host_steps, uint32_t use_series, double* __restrict__ out) {
    const uint32_t e = blockIdx.x, i = threadIdx.x;
    if (e >= ns) return;
    const SourceDesc& S = srcs[e];
    if (i > 3 * S.m) return;
    const int q = (int)S.q;
    const int64_t steps = host_steps >= 0 ? host_steps : S.steps;
    double w[kMaxQ];
    ricker_series((double)steps * S.dt + (from ? S.tau : 0.0), S.tau, S.f0, S.t0, q, w);
    double a = 0.0, b = 0.0;
    for (int k = 0; k + 1 + 2 * (int)i <= q; ++k) {
        double rb = 1.0;  // k! / (k + 1 + 2i)!
        for (int l = k + 1; l <= k + 1 + 2 * (int)i; ++l) rb /= (double)l;
        b += w[k] * rb;
        if (k + 2 + 2 * (int)i <= q) a += w[k] * rb / (double)(k + 2 + 2 * i);
    }
    double l2i = 1.0, ifact = 1.0;  // lam^(2i), i!
    for (uint32_t l = 1; l <= i; ++l) {
        l2i *= S.lam * S.lam;
        ifact *= (double)l;
    }
    const double f = (use_series && S.series) ? S.series[2 * steps + from] : 1.0;
    out[(size_t)e * 20 + i] = f * S.pre * a * l2i * S.lam * ifact;
    out[(size_t)e * 20 + 10 + i] = f * S.pre * b * l2i * ifact;
}

// Scaled Taylor coefficients g1[a], a < 2M, of the 1D Gaussian factor about
// the cell centre `pos` (h^a/a! d^a/dx^a N(x; s, sigma) = N (-h/sigma)^a
// He_a(z)/a!, z = d/sigma, d the nearest-image offset; 0 beyond 6 sigma).
template <int M>
__device__ __forceinline__ void gauss_coeffs(double pos, double s, double sigma, double h, double* g1) {
    double d = pos - s;
    d -= floor(d + 0.5);  // nearest periodic image, in [-1/2, 1/2)
    if (fabs(d) > 6.0 * sigma) {
#pragma unroll
        for (int a = 0; a < 2 * M; ++a) g1[a] = 0.0;
        return;
    }
    const double z = d / sigma;
    const double base = exp(-0.5 * z * z) / (sigma * 2.5066282746310002);  // sqrt(2 pi)
    const double r = -h / sigma;
    double he_prev = 0.0, he = 1.0, hm = 1.0, fac = 1.0;
#pragma unroll
    for (int a = 0; a < 2 * M; ++a) {
        g1[a] = base * hm * he / fac;
        const double nxt = z * he - (double)a * he_prev;
        he_prev = he;
        he = nxt;
        hm *= r;
        fac *= (double)(a + 1);
    }
}

// D[j][e] = (j + 2e)!/j! g1[j + 2e], e = 0 .. (2M-1-j)/2, for one axis.
template <int M>
__device__ __forceinline__ void axis_terms(const double* g1, int j, double* D) {
    double ff = 1.0;
#pragma unroll
    for (int e = 0; e < M; ++e) {
        if (j + 2 * e <= 2 * M - 1) {
            if (e > 0) ff *= (double)((j + 2 * e - 1) * (j + 2 * e));
            D[e] = ff * g1[j + 2 * e];
        } else {
            D[e] = 0.0;
        }
    }
}

// axis_terms for a runtime j (0 <= j < M), by compile-time selection so
// that no array is indexed dynamically (which would put it in scratch).
template <int M>
__device__ __forceinline__ void axis_terms_rt(const double* g1, int j, double* D) {
#pragma unroll
    for (int e = 0; e < M; ++e) D[e] = 0.0;
#pragma unroll
    for (int jc = 0; jc < M; ++jc) {
        double t[M];
        axis_terms<M>(g1, jc, t);
#pragma unroll
        for (int e = 0; e < M; ++e) D[e] = (jc == j) ? t[e] : D[e];
    }
}

// One thread per (box cell, j3): the M^2 outputs (j1, j2) of that j3, both
// fields, P_j = sum_e i!/(e1! e2! e3!) [A_i | B_i] prod_x D_x(j_x, e_x),
// i = |e|. AB: this source's scalars (A_i i!, B_i i!).
// DOT = false: add the source term to the destination grid. DOT = true:
// instead write this block's share of <grid[1 - from], source term> to
// partial[blockIdx.x] (a fixed-order tree sum over the block).
template <int M, bool DOT>
__global__ __launch_bounds__(kThreads) void source_kernel(const SourceDesc* __restrict__ srcs,
                                                          const uint32_t* __restrict__ prefix, uint32_t ns,
                                                          uint32_t from, const double* __restrict__ scal,
                                                          double* __restrict__ partial) {
    const uint32_t gi = batch::find_entry(prefix, ns, blockIdx.x);
    const SourceDesc& S = srcs[gi];
    const uint32_t* box = S.box[from];
    const uint32_t n = S.n, nbx = box[3], nby = box[4], nbz = box[5];
    const uint64_t t = (uint64_t)(blockIdx.x - prefix[gi]) * kThreads + threadIdx.x;
    double dot = 0.0;
    if (t < (uint64_t)nbx * nby * nbz * M) {
        const uint32_t cellk = (uint32_t)(t / M);  // box cells <= n^3 < 2^32
        const int j3 = (int)(t % M);
        const uint32_t ib = cellk % nbx, rest = cellk / nbx, jb = rest % nby, kb = rest / nby;
        const uint32_t i = (box[0] + ib) % n, j = (box[1] + jb) % n, k = (box[2] + kb) % n;
        // cell centre: lower corner + h/2 on the source grid (the dual grid sits
        // h/2 further along every axis)
        const double off_pos = from ? 0.5 : 0.0;
        double g1[3][2 * M];
        gauss_coeffs<M>(((double)i + 0.5 + off_pos) * S.h, S.x[0], S.sigma, S.h, g1[0]);
        gauss_coeffs<M>(((double)j + 0.5 + off_pos) * S.h, S.x[1], S.sigma, S.h, g1[1]);
        gauss_coeffs<M>(((double)k + 0.5 + off_pos) * S.h, S.x[2], S.sigma, S.h, g1[2]);
        double D3[M];
        axis_terms_rt<M>(g1[2], j3, D3);
        const double* __restrict__ AB = scal + (size_t)gi * 20;
        double A[3 * M - 2], Bv[3 * M - 2];
#pragma unroll
        for (int r = 0; r < 3 * M - 2; ++r) {
            A[r] = AB[r];
            Bv[r] = AB[10 + r];
        }
        const double inv_fact[4] = {1.0, 1.0, 0.5, 1.0 / 6.0};
        // the dual cell with lower corner (i, j, k) writes primal node (i+1, j+1, k+1)
        const uint32_t o = from ? 1u : 0u;
        const size_t node = ((size_t)((k + o) % n) * n + (j + o) % n) * n + (i + o) % n;
        double* __restrict__ dst = S.grid[1 - from];
        constexpr int M3 = M * M * M;
#pragma unroll
        for (int j2 = 0; j2 < M; ++j2) {
            double D2[M];
            axis_terms<M>(g1[1], j2, D2);
#pragma unroll
            for (int j1 = 0; j1 < M; ++j1) {
                double D1[M];
                axis_terms<M>(g1[0], j1, D1);
                double pu = 0.0, pv = 0.0;
                // e_x <= (2M-1-j_x)/2: terms beyond degree 2M-1 are zero (for
                // the runtime j3 the zero D3 entries do that)
#pragma unroll
                for (int e3 = M - 1; e3 >= 0; --e3)
#pragma unroll
                    for (int e2 = (2 * M - 1 - j2) / 2; e2 >= 0; --e2)
#pragma unroll
                        for (int e1 = (2 * M - 1 - j1) / 2; e1 >= 0; --e1) {
                            const double w = D1[e1] * D2[e2] * D3[e3] * (inv_fact[e1] * inv_fact[e2] * inv_fact[e3]);
                            pu = fma(A[e1 + e2 + e3], w, pu);
                            pv = fma(Bv[e1 + e2 + e3], w, pv);
                        }
                const int jj = (j3 * M + j2) * M + j1;
                if constexpr (DOT) {
                    dot = fma(dst[(size_t)jj * S.pitch + node], S.amp * pu, dot);
                    dot = fma(dst[(size_t)(M3 + jj) * S.pitch + node], S.amp * pv, dot);
                } else {
                    dst[(size_t)jj * S.pitch + node] += S.amp * pu;
                    dst[(size_t)(M3 + jj) * S.pitch + node] += S.amp * pv;
                }
            }
        }
    }
    if constexpr (DOT) {
        __shared__ double red[kThreads];
        red[threadIdx.x] = dot;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
    }
}

// grad = sum of the blocks' partial dot products, in block order.
__global__ void sum_partials_kernel(const double* __restrict__ partial, uint32_t blocks, double* __restrict__ grad) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0;
    for (uint32_t b = 0; b < blocks; ++b) s += partial[b];
    *grad = s;
}

__global__ void advance_clock_kernel(SourceDesc* __restrict__ srcs, uint32_t ns) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns) srcs[i].steps += 1;
}

}  // namespace

uint32_t source_blocks(const SourceDesc& s, int from) {
    const uint32_t* b = s.box[from];
    const uint64_t total = (uint64_t)b[3] * b[4] * b[5] * (s.m + 1);
    return (uint32_t)((total + kThreads - 1) / kThreads);
}

hipError_t launch_source(const SourceDesc* srcs, const uint32_t* prefix, uint32_t ns, uint32_t blocks, int m, int from,
                         long long host_steps, double* scal, hipStream_t st) {
    if (blocks == 0 || ns == 0) return hipSuccess;
    hipLaunchKernelGGL(source_scalars_kernel, dim3(ns), dim3(16), 0, st, srcs, ns, (uint32_t)from,
                       (int64_t)host_steps, 1u, scal);
    const double* sc = scal;
    double* none = nullptr;
    switch (m) {
        case 1: hipLaunchKernelGGL((source_kernel<2, false>), dim3(blocks), dim3(kThreads), 0, st, srcs, prefix, ns, (uint32_t)from, sc, none); break;
        case 2: hipLaunchKernelGGL((source_kernel<3, false>), dim3(blocks), dim3(kThreads), 0, st, srcs, prefix, ns, (uint32_t)from, sc, none); break;
        case 3: hipLaunchKernelGGL((source_kernel<4, false>), dim3(blocks), dim3(kThreads), 0, st, srcs, prefix, ns, (uint32_t)from, sc, none); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_source_dot(const SourceDesc* src, const uint32_t* prefix, uint32_t blocks, int m, int from,
                             long long host_steps, double* scal, double* partial, double* grad, hipStream_t st) {
    if (blocks == 0) {
        hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, st, (const double*)partial, 0u, grad);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(source_scalars_kernel, dim3(1), dim3(16), 0, st, src, 1u, (uint32_t)from,
                       (int64_t)host_steps, 0u, scal);
    const double* sc = scal;
    switch (m) {
        case 1: hipLaunchKernelGGL((source_kernel<2, true>), dim3(blocks), dim3(kThreads), 0, st, src, prefix, 1u, (uint32_t)from, sc, partial); break;
        case 2: hipLaunchKernelGGL((source_kernel<3, true>), dim3(blocks), dim3(kThreads), 0, st, src, prefix, 1u, (uint32_t)from, sc, partial); break;
        case 3: hipLaunchKernelGGL((source_kernel<4, true>), dim3(blocks), dim3(kThreads), 0, st, src, prefix, 1u, (uint32_t)from, sc, partial); break;
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, st, (const double*)partial, blocks, grad);
    return hipGetLastError();
}

hipError_t launch_advance_clock(SourceDesc* srcs, uint32_t ns, hipStream_t st) {
    if (ns == 0) return hipSuccess;
    hipLaunchKernelGGL(advance_clock_kernel, dim3((ns + 255) / 256), dim3(256), 0, st, srcs, ns);
    return hipGetLastError();
}

}  // namespace hermite
