// Host-side constant tables of the Hermite half step, built in long double
// and rounded once to FP64.
#include "constants.h"

#include <cmath>
#include <vector>

namespace hermite {

namespace {

long double binom(int a, int b) {
    if (b < 0 || b > a) return 0.0L;
    long double r = 1.0L;
    for (int i = 1; i <= b; ++i) r = r * (long double)(a - b + i) / (long double)i;
    return r;
}

long double fact(int a) {
    long double r = 1.0L;
    for (int i = 2; i <= a; ++i) r *= (long double)i;
    return r;
}

std::vector<long double> poly_mul(const std::vector<long double>& a, const std::vector<long double>& b) {
    std::vector<long double> r(a.size() + b.size() - 1, 0.0L);
    for (size_t i = 0; i < a.size(); ++i)
        for (size_t j = 0; j < b.size(); ++j) r[i + j] += a[i] * b[j];
    return r;
}

}  // namespace

int nout(int M, int p) { return (M + 1 - p) / 2; }

int rows_max(int m) {
    const int no = nout(m + 1, 0);
    return 2 * no * no * no;
}

// Two-point Hermite basis on t = xi + 1/2 in [0, 1]: the polynomial whose
// k-th scaled derivative at t = 0 is 1, whose other scaled derivatives of
// order <= m at t = 0 vanish, and which has a zero of order m+1 at t = 1 is
//     phi_k(t) = t^k (1 - t)^(m+1) sum_{v=0}^{m-k} C(m+v, v) t^v,
// because the truncated sum is the series of (1 - t)^-(m+1) to order m-k.
// The right-end basis is (-1)^k phi_k(1 - t).
std::vector<double> hermite_matrix(int m) {
    const int M = m + 1, P = 2 * m + 2;
    std::vector<double> H((size_t)P * P, 0.0);
    for (int k = 0; k < M; ++k) {
        std::vector<long double> tk(k + 1, 0.0L);
        tk[k] = 1.0L;
        std::vector<long double> one_minus_t = {1.0L, -1.0L};
        std::vector<long double> pw = {1.0L};
        for (int r = 0; r < M; ++r) pw = poly_mul(pw, one_minus_t);
        std::vector<long double> s(m - k + 1, 0.0L);
        for (int v = 0; v <= m - k; ++v) s[v] = binom(m + v, v);
        std::vector<long double> phi = poly_mul(poly_mul(tk, pw), s);  // in t, degree 2m+1
        // substitute t = xi + 1/2
        for (int j = 0; j < P; ++j) {
            long double bj = 0.0L;
            for (int i = j; i < (int)phi.size(); ++i)
                bj += phi[i] * binom(i, j) * std::pow(0.5L, (long double)(i - j));
            H[(size_t)j * P + k] = (double)bj;
            const double sgn = ((j + k) % 2 == 0) ? 1.0 : -1.0;
            H[(size_t)j * P + M + k] = sgn * (double)bj;
        }
    }
    return H;
}

std::vector<double> hermite_parity_blocks(int m) {
    const int M = m + 1, P = 2 * m + 2;
    const std::vector<double> H = hermite_matrix(m);
    std::vector<double> B((size_t)2 * M * M, 0.0);
    for (int p = 0; p < 2; ++p)
        for (int i = 0; i < M; ++i)
            for (int k = 0; k < M; ++k) B[((size_t)p * M + i) * M + k] = H[(size_t)(p + 2 * i) * P + M + k];
    return B;
}

std::vector<double> evolution_poly(int m, int evolution, int q, int rk_substeps) {
    const int smax = 6 * m + 1;
    std::vector<long double> c(smax + 1, 0.0L);
    if (evolution == 0) {
        for (int s = 0; s <= smax && s <= q; ++s) c[s] = 1.0L / fact(s);
    } else {
        const long double S = (long double)rk_substeps;
        std::vector<long double> g(5);
        for (int t = 0; t <= 4; ++t) g[t] = 1.0L / (fact(t) * std::pow(S, (long double)t));
        std::vector<long double> acc = {1.0L};
        for (int i = 0; i < rk_substeps; ++i) {
            acc = poly_mul(acc, g);
            if ((int)acc.size() > smax + 1) acc.resize(smax + 1);
        }
        for (int s = 0; s <= smax && s < (int)acc.size(); ++s) c[s] = acc[s];
    }
    std::vector<double> out(smax + 1);
    for (int s = 0; s <= smax; ++s) out[s] = (double)c[s];
    return out;
}

// The evolution polynomial sum_s c_s L^s with L(a, b) = lam (b, Lap a) splits,
// since L^2 = lam^2 Lap on each field, into
//   u <- sum_r c_2r lam^2r Lap^r u + c_2r+1 lam^2r+1 Lap^r v
//   v <- sum_r c_2r lam^2r Lap^r v + c_2r-1 lam^2r-1 Lap^r u   (r >= 1 in the last term).
// On monomial coefficients, (Lap^r W)[j] = sum_{|e| = r} r!/(e1! e2! e3!)
//   prod_x (j_x + 2 e_x)!/j_x! * W[j + 2e]  (each second derivative shifts one
// index by 2). Outputs j <= m per axis; inputs k = j + 2e keep the parity of j,
// so the map is block diagonal over the 8 parity classes.
std::vector<double> fused_class_operators(int m, double lam, const std::vector<double>& cpoly) {
    const int M = m + 1, M3 = M * M * M, NC = 2 * M3, RM = rows_max(m);
    const std::vector<double> B = hermite_parity_blocks(m);
    std::vector<double> K((size_t)8 * RM * NC, 0.0);
    std::vector<long double> lp(6 * m + 2);
    lp[0] = 1.0L;
    for (size_t s = 1; s < lp.size(); ++s) lp[s] = lp[s - 1] * (long double)lam;
    auto cp = [&](int s) -> long double { return (s >= 0 && s < (int)cpoly.size()) ? (long double)cpoly[s] : 0.0L; };
    for (int pc = 0; pc < 8; ++pc) {
        const int p[3] = {pc & 1, (pc >> 1) & 1, (pc >> 2) & 1};
        const int no[3] = {nout(M, p[0]), nout(M, p[1]), nout(M, p[2])};
        const int nof = no[0] * no[1] * no[2];
        for (int fo = 0; fo < 2; ++fo)
            for (int o3 = 0; o3 < no[2]; ++o3)
                for (int o2 = 0; o2 < no[1]; ++o2)
                    for (int o1 = 0; o1 < no[0]; ++o1) {
                        const int row = fo * nof + (o3 * no[1] + o2) * no[0] + o1;
                        const int o[3] = {o1, o2, o3};
                        std::vector<long double> acc((size_t)NC, 0.0L);
                        for (int e3 = 0; o3 + e3 < M; ++e3)
                            for (int e2 = 0; o2 + e2 < M; ++e2)
                                for (int e1 = 0; o1 + e1 < M; ++e1) {
                                    const int e[3] = {e1, e2, e3};
                                    const int r = e1 + e2 + e3;
                                    long double D = fact(r) / (fact(e1) * fact(e2) * fact(e3));
                                    for (int x = 0; x < 3; ++x) {
                                        const int jx = p[x] + 2 * o[x];
                                        D *= fact(jx + 2 * e[x]) / fact(jx);
                                    }
                                    // weights from field fi to output field fo
                                    long double w[2];
                                    if (fo == 0) {
                                        w[0] = cp(2 * r) * lp[2 * r];
                                        w[1] = cp(2 * r + 1) * lp[2 * r + 1];
                                    } else {
                                        w[1] = cp(2 * r) * lp[2 * r];
                                        w[0] = (r >= 1) ? cp(2 * r - 1) * lp[2 * r - 1] : 0.0L;
                                    }
                                    // input coefficient index along x: i_x = o_x + e_x
                                    for (int d3 = 0; d3 < M; ++d3)
                                        for (int d2 = 0; d2 < M; ++d2)
                                            for (int d1 = 0; d1 < M; ++d1) {
                                                const long double hb =
                                                    (long double)B[((size_t)p[0] * M + o1 + e1) * M + d1] *
                                                    (long double)B[((size_t)p[1] * M + o2 + e2) * M + d2] *
                                                    (long double)B[((size_t)p[2] * M + o3 + e3) * M + d3];
                                                const int dd = (d3 * M + d2) * M + d1;
                                                for (int fi = 0; fi < 2; ++fi) acc[(size_t)fi * M3 + dd] += w[fi] * D * hb;
                                            }
                                }
                        for (int col = 0; col < NC; ++col)
                            K[((size_t)pc * RM + row) * NC + col] = (double)acc[(size_t)col];
                    }
    }
    return K;
}

std::vector<double> advection_translation(int m, double lam) {
    const int M = m + 1, P = 2 * m + 2;
    std::vector<double> E((size_t)M * P, 0.0);
    for (int j = 0; j < M; ++j)
        for (int k = j; k < P; ++k)
            E[(size_t)j * P + k] = (double)(binom(k, j) * std::pow((long double)lam, (long double)(k - j)));
    return E;
}

std::vector<double> advection_axis_operator(int m, double lam) {
    const int M = m + 1, P = 2 * m + 2;
    const std::vector<double> H = hermite_matrix(m);
    std::vector<double> K((size_t)M * P, 0.0);
    for (int j = 0; j < M; ++j)
        for (int a = 0; a < P; ++a) {
            long double acc = 0.0L;
            for (int k = j; k < P; ++k)
                acc += binom(k, j) * std::pow((long double)lam, (long double)(k - j)) * (long double)H[(size_t)k * P + a];
            K[(size_t)j * P + a] = (double)acc;
        }
    return K;
}

}  // namespace hermite
