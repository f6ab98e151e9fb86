/*
 * Oracle (test infrastructure only): direct O(N^2) DDA matrix-vector product
 * in double precision, plain C + OpenMP.
 *
 * Not part of the product.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this file's shared object.
 *
 * Computes y = A x for the DDA system A P = E (guide, section "Choice of
 * Iterative Algorithm", eq. AP=E), where for sites j != l
 *
 *   A_jl = exp(i k r)/r * [ k^2 (n n - I) + (i k r - 1)/r^2 (3 n n - I) ],
 *   r = |r_j - r_l|,  n = (r_j - r_l)/r,
 *
 * i.e. minus the retarded field tensor of a point dipole in Gaussian units
 * (Draine 1988, cited in the guide's introduction), and the diagonal block is
 * alpha_j^{-1} I with a scalar inverse polarizability per site.  The sum is
 * taken term by term over all pairs: no FFT, no blocking.
 *
 * Layout: r is N x 3 doubles (site coordinates in units of d), x and y are
 * N x 3 complex doubles (site-major, Cartesian component fastest), ainv is N
 * complex doubles.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>

typedef double complex cplx;

void oracle_matvec(int64_t n, const double* r, double k, const cplx* ainv,
                   const cplx* x, cplx* y)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < n; ++j) {
        cplx acc[3] = {0, 0, 0};
        const double rjx = r[3 * j], rjy = r[3 * j + 1], rjz = r[3 * j + 2];
        for (int64_t l = 0; l < n; ++l) {
            if (l == j) continue;
            const double dx = rjx - r[3 * l], dy = rjy - r[3 * l + 1], dz = rjz - r[3 * l + 2];
            const double rr = sqrt(dx * dx + dy * dy + dz * dz);
            const double nv[3] = {dx / rr, dy / rr, dz / rr};
            const cplx phase = cexp(I * k * rr) / rr;
            const cplx c1 = k * k;                             /* multiplies (n n - I) */
            const cplx c2 = (I * k * rr - 1.0) / (rr * rr);    /* multiplies (3 n n - I) */
            const cplx xl[3] = {x[3 * l], x[3 * l + 1], x[3 * l + 2]};
            for (int a = 0; a < 3; ++a) {
                cplx s = 0;
                for (int b = 0; b < 3; ++b) {
                    const double nn = nv[a] * nv[b];
                    const double id = (a == b) ? 1.0 : 0.0;
                    s += (c1 * (nn - id) + c2 * (3.0 * nn - id)) * xl[b];
                }
                acc[a] += phase * s;
            }
        }
        for (int a = 0; a < 3; ++a) y[3 * j + a] = acc[a] + ainv[j] * x[3 * j + a];
    }
}

/*
 * Rows of the same product for a subset of sites only: y_s = (A x)_{rows[s]}.
 * Lets a test check a large GPU product at sampled sites, one row at a time.
 */
void oracle_matvec_rows(int64_t n, const double* r, double k, const cplx* ainv,
                        const cplx* x, int64_t nrows, const int64_t* rows, cplx* y)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nrows; ++s) {
        const int64_t j = rows[s];
        cplx acc[3] = {0, 0, 0};
        const double rjx = r[3 * j], rjy = r[3 * j + 1], rjz = r[3 * j + 2];
        for (int64_t l = 0; l < n; ++l) {
            if (l == j) continue;
            const double dx = rjx - r[3 * l], dy = rjy - r[3 * l + 1], dz = rjz - r[3 * l + 2];
            const double rr = sqrt(dx * dx + dy * dy + dz * dz);
            const double nv[3] = {dx / rr, dy / rr, dz / rr};
            const cplx phase = cexp(I * k * rr) / rr;
            const cplx c1 = k * k;
            const cplx c2 = (I * k * rr - 1.0) / (rr * rr);
            const cplx xl[3] = {x[3 * l], x[3 * l + 1], x[3 * l + 2]};
            for (int a = 0; a < 3; ++a) {
                cplx s2 = 0;
                for (int b = 0; b < 3; ++b) {
                    const double nn = nv[a] * nv[b];
                    const double id = (a == b) ? 1.0 : 0.0;
                    s2 += (c1 * (nn - id) + c2 * (3.0 * nn - id)) * xl[b];
                }
                acc[a] += phase * s2;
            }
        }
        for (int a = 0; a < 3; ++a) y[3 * s + a] = acc[a] + ainv[j] * x[3 * j + a];
    }
}

/* Threads OpenMP will use for the loops above. */
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }
