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
// One launch serves every source of a batch: blocks are dealt to sources by
// a prefix table, and each block first forms its source's w_k, A_i and B_i
// in LDS from the half step's start time, read from the source's device-side
// step clock (so a captured graph replays with fixed arguments) or given by
// the host.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch_common.h"
#include "kernels.h"

namespace hermite {
namespace {

constexpr int kMaxP = 8;   // 2m + 2 for m <= 3
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

__global__ __launch_bounds__(kThreads) void source_kernel(const SourceDesc* __restrict__ srcs,
                                                          const uint32_t* __restrict__ prefix, uint32_t ns,
                                                          uint32_t from, int64_t host_steps) {
    __shared__ double sw[kMaxQ];
    __shared__ double sAB[2][10];
    const uint32_t gi = batch::find_entry(prefix, ns, blockIdx.x);
    const SourceDesc& S = srcs[gi];
    const int m = (int)S.m, M = m + 1, P = 2 * m + 2, M3 = M * M * M, q = (int)S.q;
    const int64_t steps = host_steps >= 0 ? host_steps : S.steps;
    if (threadIdx.x == 0) ricker_series((double)steps * S.dt + (from ? S.tau : 0.0), S.tau, S.f0, S.t0, q, sw);
    __syncthreads();
    if (threadIdx.x <= (unsigned)(3 * m)) {
        const int i = (int)threadIdx.x;
        double a = 0.0, b = 0.0;
        for (int k = 0; k + 1 + 2 * i <= q; ++k) {
            double rb = 1.0;  // k! / (k + 1 + 2i)!
            for (int l = k + 1; l <= k + 1 + 2 * i; ++l) rb /= (double)l;
            b += sw[k] * rb;
            if (k + 2 + 2 * i <= q) a += sw[k] * rb / (double)(k + 2 + 2 * i);
        }
        double l2i = 1.0, ifact = 1.0;  // lam^(2i), i!
        for (int l = 1; l <= i; ++l) {
            l2i *= S.lam * S.lam;
            ifact *= (double)l;
        }
        sAB[0][i] = S.pre * a * l2i * S.lam * ifact;  // A_i i!
        sAB[1][i] = S.pre * b * l2i * ifact;          // B_i i!
    }
    __syncthreads();

    const uint32_t* box = S.box[from];
    const uint32_t n = S.n, nbx = box[3], nby = box[4], nbz = box[5];
    const uint64_t t = (uint64_t)(blockIdx.x - prefix[gi]) * kThreads + threadIdx.x;
    const uint64_t nbox = (uint64_t)nbx * nby * nbz;
    if (t >= nbox * (uint64_t)M3) return;
    const uint64_t cellk = t / (uint64_t)M3;
    const int jj = (int)(t % (uint64_t)M3);
    const int j1 = jj % M, j2 = (jj / M) % M, j3 = jj / (M * M);
    const uint32_t ib = (uint32_t)(cellk % nbx), jb = (uint32_t)((cellk / nbx) % nby),
                   kb = (uint32_t)(cellk / ((uint64_t)nbx * nby));
    const uint32_t i = (box[0] + ib) % n, j = (box[1] + jb) % n, k = (box[2] + kb) % n;
    // cell centre: lower corner + h/2 on the source grid (the dual grid sits
    // h/2 further along every axis)
    const double off_pos = from ? 0.5 : 0.0;
    const double pos[3] = {((double)i + 0.5 + off_pos) * S.h, ((double)j + 0.5 + off_pos) * S.h,
                           ((double)k + 0.5 + off_pos) * S.h};
    const int jv[3] = {j1, j2, j3};
    // per axis: D_x(e) = (j_x + 2e)!/j_x! * g1_x[j_x + 2e], e = 0 .. (2m+1-j_x)/2
    double D[3][5];
    int ne[3];
    for (int x = 0; x < 3; ++x) {
        double d = pos[x] - S.x[x];
        d -= floor(d + 0.5);  // nearest periodic image, in [-1/2, 1/2)
        const double z = d / S.sigma;
        double g1[kMaxP];
        if (fabs(d) > 6.0 * S.sigma) {
            for (int a = 0; a < P; ++a) g1[a] = 0.0;
        } else {
            // g1_a = h^a/a! d^a/dx^a N(x; s, sigma) = N (-h/sigma)^a He_a(z)/a!
            const double base = exp(-0.5 * z * z) / (S.sigma * 2.5066282746310002);  // sqrt(2 pi)
            const double r = -S.h / S.sigma;
            double he_prev = 0.0, he = 1.0, hm = 1.0, fac = 1.0;
            for (int a = 0; a < P; ++a) {
                g1[a] = base * hm * he / fac;
                const double nxt = z * he - (double)a * he_prev;
                he_prev = he;
                he = nxt;
                hm *= r;
                fac *= (double)(a + 1);
            }
        }
        ne[x] = (2 * m + 1 - jv[x]) / 2 + 1;
        double ff = 1.0;  // (j + 2e)! / j!
        for (int e = 0; e < ne[x]; ++e) {
            if (e > 0) ff *= (double)((jv[x] + 2 * e - 1) * (jv[x] + 2 * e));
            D[x][e] = ff * g1[jv[x] + 2 * e];
        }
    }
    // sum_e i!/(e1! e2! e3!) [A_i | B_i] prod_x D_x(e_x), i = |e|
    const double inv_fact[5] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0};
    double pu = 0.0, pv = 0.0;
    for (int e3 = ne[2] - 1; e3 >= 0; --e3)
        for (int e2 = ne[1] - 1; e2 >= 0; --e2)
            for (int e1 = ne[0] - 1; e1 >= 0; --e1) {
                const int ii = e1 + e2 + e3;
                const double w = D[0][e1] * D[1][e2] * D[2][e3] * inv_fact[e1] * inv_fact[e2] * inv_fact[e3];
                pu = fma(sAB[0][ii], w, pu);
                pv = fma(sAB[1][ii], w, pv);
            }
    // the dual cell with lower corner (i, j, k) writes primal node (i+1, j+1, k+1)
    const uint32_t o = from ? 1u : 0u;
    const uint32_t oi = (i + o) % n, oj = (j + o) % n, ok = (k + o) % n;
    const size_t node = ((size_t)ok * n + oj) * n + oi;
    double* __restrict__ dst = S.grid[1 - from];
    dst[(size_t)jj * S.pitch + node] += S.amp * pu;
    dst[(size_t)(M3 + jj) * S.pitch + node] += S.amp * pv;
}

__global__ void advance_clock_kernel(SourceDesc* __restrict__ srcs, uint32_t ns) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns) srcs[i].steps += 1;
}

}  // namespace

uint32_t source_blocks(const SourceDesc& s, int from) {
    const uint32_t* b = s.box[from];
    const uint64_t M = s.m + 1;
    const uint64_t total = (uint64_t)b[3] * b[4] * b[5] * M * M * M;
    return (uint32_t)((total + kThreads - 1) / kThreads);
}

hipError_t launch_source(const SourceDesc* srcs, const uint32_t* prefix, uint32_t ns, uint32_t blocks, int from,
                         long long host_steps, hipStream_t st) {
    if (blocks == 0 || ns == 0) return hipSuccess;
    hipLaunchKernelGGL(source_kernel, dim3(blocks), dim3(kThreads), 0, st, srcs, prefix, ns, (uint32_t)from,
                       (int64_t)host_steps);
    return hipGetLastError();
}

hipError_t launch_advance_clock(SourceDesc* srcs, uint32_t ns, hipStream_t st) {
    if (ns == 0) return hipSuccess;
    hipLaunchKernelGGL(advance_clock_kernel, dim3((ns + 255) / 256), dim3(256), 0, st, srcs, ns);
    return hipGetLastError();
}

}  // namespace hermite
