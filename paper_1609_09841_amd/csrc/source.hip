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
// with the host-side scalars
//   A_i = (tau h / c) sum_{k + 2 + 2i <= q} w_k k! / (k + 2 + 2i)! lam^(2i+1),
//   B_i = (tau h / c) sum_{k + 1 + 2i <= q} w_k k! / (k + 1 + 2i)! lam^(2i).
// On monomial coefficients (Lap^i G)_j = sum_{|e| = i} i!/(e1! e2! e3!)
// prod_x (j_x + 2 e_x)!/j_x! G_{j + 2e}. The kernel adds P_j, j <= m, to the
// new node of every cell within 6 sigma of the source (periodic nearest image
// per axis; beyond 6 sigma along any axis g is taken as 0).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace hermite {
namespace {

constexpr int kMaxP = 8;  // 2m + 2 for m <= 3

__global__ __launch_bounds__(256) void source_kernel(double* __restrict__ dst, uint32_t n, size_t pitch, int m,
                                                     uint32_t bx0, uint32_t by0, uint32_t bz0, uint32_t nbx,
                                                     uint32_t nby, uint32_t nbz, double cx, double cy, double cz,
                                                     double h, double sigma, double amp, double off_pos,
                                                     uint32_t off_idx, SourceScalars sc) {
    const int M = m + 1, P = 2 * m + 2, M3 = M * M * M;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nbox = (uint64_t)nbx * nby * nbz;
    if (t >= nbox * (uint64_t)M3) return;
    const uint64_t cellk = t / (uint64_t)M3;
    const int jj = (int)(t % (uint64_t)M3);
    const int j1 = jj % M, j2 = (jj / M) % M, j3 = jj / (M * M);
    const uint32_t ib = (uint32_t)(cellk % nbx), jb = (uint32_t)((cellk / nbx) % nby),
                   kb = (uint32_t)(cellk / ((uint64_t)nbx * nby));
    const uint32_t i = (bx0 + ib) % n, j = (by0 + jb) % n, k = (bz0 + kb) % n;
    // cell centre (lower corner + h/2 on the source grid; off_pos = 0 for the
    // primal grid, 1/2 for the dual grid, in units of h)
    const double pos[3] = {((double)i + 0.5 + off_pos) * h, ((double)j + 0.5 + off_pos) * h,
                           ((double)k + 0.5 + off_pos) * h};
    const double src[3] = {cx, cy, cz};
    const int jv[3] = {j1, j2, j3};
    // per axis: D_x(e) = (j_x + 2e)!/j_x! * g1_x[j_x + 2e], e = 0 .. (2m+1-j_x)/2
    double D[3][5];
    int ne[3];
    for (int x = 0; x < 3; ++x) {
        double d = pos[x] - src[x];
        d -= floor(d + 0.5);  // nearest periodic image, in [-1/2, 1/2)
        const double z = d / sigma;
        double g1[kMaxP];
        if (fabs(d) > 6.0 * sigma) {
            for (int a = 0; a < P; ++a) g1[a] = 0.0;
        } else {
            // g1_a = h^a/a! d^a/dx^a N(x; s, sigma) = N (-h/sigma)^a He_a(z)/a!
            // (He: probabilists' Hermite polynomials, He_{a+1} = z He_a - a He_{a-1})
            const double base = exp(-0.5 * z * z) / (sigma * 2.5066282746310002);  // sqrt(2 pi)
            const double r = -h / sigma;
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
                pu = fma(sc.Ai[ii], w, pu);  // Ai, Bi already carry the factor i!
                pv = fma(sc.Bi[ii], w, pv);
            }
    const uint32_t oi = (i + off_idx) % n, oj = (j + off_idx) % n, ok = (k + off_idx) % n;
    const size_t node = ((size_t)ok * n + oj) * n + oi;
    dst[(size_t)jj * pitch + node] += amp * pu;
    dst[(size_t)(M3 + jj) * pitch + node] += amp * pv;
}

}  // namespace

hipError_t launch_source(double* dst, int n, size_t pitch, int m, const SourceBox& box, const double* centre,
                         double h, double sigma, double amp, int to_dual, const SourceScalars& sc,
                         hipStream_t st) {
    if (m < 1 || m > 3 || box.nx > (uint32_t)n || box.ny > (uint32_t)n || box.nz > (uint32_t)n)
        return hipErrorInvalidValue;
    const uint64_t M3 = (uint64_t)((m + 1) * (m + 1) * (m + 1));
    const uint64_t total = (uint64_t)box.nx * box.ny * box.nz * M3;
    if (total == 0) return hipSuccess;
    const double off_pos = to_dual ? 0.0 : 0.5;
    const uint32_t off_idx = to_dual ? 0u : 1u;
    hipLaunchKernelGGL(source_kernel, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, dst, (uint32_t)n, pitch, m, box.x0,
                       box.y0, box.z0, box.nx, box.ny, box.nz, centre[0], centre[1], centre[2], h, sigma, amp,
                       off_pos, off_idx, sc);
    return hipGetLastError();
}

}  // namespace hermite
