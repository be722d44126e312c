// Host-side constant tables of the Hermite half step (FP64).
//
// Notation: m = derivatives per dimension, M = m+1, P = 2m+2 (1D polynomial
// length, degree 2m+1). Cell variable xi = (x - x_centre)/h in [-1/2, 1/2].
#pragma once

#include <vector>

namespace hermite {

// 1D Hermite matrix H (Sec. 3.1), P x P row-major, H[j*P + a]: monomial
// coefficient b_j of the interpolant from the data a = side*M + k (scaled
// derivative k at xi = -1/2 for side 0, +1/2 for side 1). Built from the
// closed-form two-point Hermite basis; every entry is a short dyadic
// rational, exact in FP64.
std::vector<double> hermite_matrix(int m);

// Parity blocks of H. H[j][(0,k)] = (-1)^(j+k) H[j][(1,k)], so for output
// parity p the coefficients b_{p+2i} depend only on the combinations
// c_p[k] = R_k + (-1)^(p+k) L_k:  b_{p+2i} = sum_k Hp[p][i][k] c_p[k].
// Returned as [2][M][M].
std::vector<double> hermite_parity_blocks(int m);

// Coefficients c_s (s = 0..6m+1) of the evolution polynomial E(L) = sum c_s L^s
// applied to the cell state over one half step, with L the cell operator of the
// wave system in the half-step time. Taylor with q stages: c_s = 1/s!, s <= q.
// RK4 with S substeps: (sum_{t<=4} (L/S)^t / t!)^S. Powers above 6m+1 vanish
// on the cell space and are dropped.
std::vector<double> evolution_poly(int m, int evolution, int q, int rk_substeps);

// Fused operator per parity class (see kernels): for class p = (p1,p2,p3)
// (bit x of p is the parity of the coefficient index along axis x+1), the map
// from the 2*M^3 class inputs c_p[f][d3][d2][d1] to the class outputs
// [f][o3][o2][o1] (new node data j = p + 2o with every j_x <= m):
// evolution polynomial (with lam = c*tau/h) composed with the parity blocks.
// Layout [8][rows_max][2*M^3], rows_max = 2*nout(p=0)^3, unused rows zero.
std::vector<double> fused_class_operators(int m, double lam, const std::vector<double>& cpoly);

// Advection u_t = c (u_x1 + u_x2 + u_x3): with the exact stage count the
// half step translates each cell polynomial by lam (1, 1, 1), lam = c tau/h,
// so interpolation, evolution and truncation compose per axis into
// K1 = T E H, M x P row-major, K1[j][a] = sum_k C(k, j) lam^(k-j) H[k][a].
std::vector<double> advection_axis_operator(int m, double lam);
// The translation part alone, E[j][k] = C(k, j) lam^(k-j), M x P row-major
// (rows j <= m): the evolution half of the two-kernel advection step.
std::vector<double> advection_translation(int m, double lam);

int rows_max(int m);
int nout(int M, int p);

}  // namespace hermite
