/* Host-only driver of the C oracle for AddressSanitizer / UBSan runs: small
 * cases of every entry point the tests use, on heap buffers of exactly the
 * documented sizes, so that any out-of-bounds access or undefined behaviour
 * in the oracle aborts the run. Built and run by tests/test_sanitize_cpu.py. */
#include <stdio.h>
#include <stdlib.h>

int oracle_hermite_matrix(int m, double *H);
int oracle_run(int n, int m, double cfl, double c, int evo, int param, int nsteps, double *u, double *ut);
int oracle_run_forced(int n, int m, double cfl, double c, int q, int nsteps, double *u, double *ut, const double *sx,
                      double sigma, double f0, double t0, double amp);
int oracle_run_advection(int n, int m, double cfl, double c, int q, int nsteps, double *u);
int oracle_point(int n, int m, double cfl, double c, int evo, int param, int nsteps, const double *u,
                 const double *ut, int i, int j, int k, double *out);
void oracle_adjoint_half_step(int n, int m, const double *H, double lam, int q, const double *lam_dst,
                              double *lam_src, int to_dual);
int oracle_source_term(int n, int m, double cfl, double c, int q, int to_dual, double ta, const double *sx,
                       double sigma, double f0, double t0, double amp, double *out);

static double *field(long count, unsigned seed)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)count);
    srand(seed);
    for (long t = 0; t < count; ++t) a[t] = (double)rand() / RAND_MAX - 0.5;
    return a;
}

int main(void)
{
    int bad = 0;
    const double sx[3] = {0.3, 0.8, 0.55};
    for (int m = 1; m <= 3; ++m) {
        const int n = 3, M = m + 1, P = 2 * M;
        const long sz = (long)M * M * M * n * n * n;
        double *u = field(sz, 1), *ut = field(sz, 2), *out = field(2 * M * M * M, 3), *H = field(P * P, 4);
        bad |= oracle_hermite_matrix(m, H) != 0;
        bad |= oracle_run(n, m, 0.5, 1.0, 0, 6 * m + 1, 2, u, ut) != 0;
        bad |= oracle_run(n, m, 0.5, 1.0, 1, 2, 1, u, ut) != 0;
        bad |= oracle_point(n, m, 0.5, 1.0, 0, 6 * m + 1, 1, u, ut, 2, 0, 1, out) != 0;
        bad |= oracle_run_forced(n, m, 0.5, 1.0, 6 * m + 1, 2, u, ut, sx, 0.2, 2.0, 0.1, 1.0) != 0;
        bad |= oracle_run_advection(n, m, 0.5, 1.0, 3 * (2 * m + 1), 2, u) != 0;
        double *ld = field(2 * sz, 5), *ls = field(2 * sz, 6);
        oracle_adjoint_half_step(n, m, H, 0.25, 6 * m + 1, ld, ls, 1);
        oracle_adjoint_half_step(n, m, H, 0.25, 6 * m + 1, ls, ld, 0);
        bad |= oracle_source_term(n, m, 0.5, 1.0, 6 * m + 1, 0, 0.05, sx, 0.2, 2.0, 0.1, 1.0, ld) != 0;
        free(u); free(ut); free(out); free(H); free(ld); free(ls);
    }
    printf(bad ? "oracle driver: a call failed\n" : "oracle driver: ok\n");
    return bad;
}
