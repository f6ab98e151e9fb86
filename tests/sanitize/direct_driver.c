/*
 * Test driver for the oracle's direct pair sum under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_oracle_sanitized.py with
 * gcc, host code only).  Reads one problem from a binary file, runs the full
 * product and the sampled-row product, writes both results.
 *
 * Input file:  int64 n, int64 nrows, double k, r[n][3], ainv[n] (complex),
 *              x[n][3] (complex), rows[nrows] (int64)
 * Output file: y[n][3] (complex), ys[nrows][3] (complex)
 */
#include <complex.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;

void oracle_matvec(int64_t n, const double* r, double k, const cplx* ainv, const cplx* x, cplx* y);
void oracle_matvec_rows(int64_t n, const double* r, double k, const cplx* ainv, const cplx* x,
                        int64_t nrows, const int64_t* rows, cplx* y);

static void* read_exact(FILE* f, size_t bytes)
{
    void* p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

int main(int argc, char** argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s in.bin out.bin\n", argv[0]);
        return 2;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t hdr[2];
    double k;
    if (fread(hdr, sizeof hdr, 1, f) != 1 || fread(&k, sizeof k, 1, f) != 1) return 2;
    const int64_t n = hdr[0], nrows = hdr[1];
    double* r = read_exact(f, (size_t)n * 3 * sizeof(double));
    cplx* ainv = read_exact(f, (size_t)n * sizeof(cplx));
    cplx* x = read_exact(f, (size_t)n * 3 * sizeof(cplx));
    int64_t* rows = read_exact(f, (size_t)nrows * sizeof(int64_t));
    fclose(f);
    cplx* y = malloc((size_t)n * 3 * sizeof(cplx));
    cplx* ys = malloc((size_t)(nrows ? nrows : 1) * 3 * sizeof(cplx));
    oracle_matvec(n, r, k, ainv, x, y);
    oracle_matvec_rows(n, r, k, ainv, x, nrows, rows, ys);
    FILE* g = fopen(argv[2], "wb");
    if (!g) return 2;
    fwrite(y, sizeof(cplx), (size_t)n * 3, g);
    fwrite(ys, sizeof(cplx), (size_t)nrows * 3, g);
    fclose(g);
    free(r);
    free(ainv);
    free(x);
    free(rows);
    free(y);
    free(ys);
    return 0;
}
