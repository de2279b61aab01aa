/*
 * CPU oracle for the adaptive-region hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, serial, obviously-correct C for what the region variants compute.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * it; the product library never does, and the two share no code.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (contraction off so that a*b+c is never fused: every sum and product is
 * rounded on its own, as the definitions below state).
 *
 * Regions (the paper's workloads are a stencil code -- the Heat benchmark of
 * Table 3 -- and a sparse relaxation -- AMGMk of Table 3; these are the
 * plain definitions of the two region kinds the adaptive runtime runs):
 *
 *  orc_jacobi7   7-point Jacobi sweep on an nx*ny*nz FP64 grid, x fastest,
 *                neighbours weighted 1/6 and the centre 0, values outside
 *                the grid read as +0.0 (zero Dirichlet ghost layer).  One
 *                sweep: v = (((((xm+xp)+ym)+yp)+zm)+zp) * C, C = fl(1/6),
 *                applied S times.
 *  orc_spmv_plain      y_i = sum_k val[k]*x[col[k]] summed left to right
 *                      from +0.0, each product rounded on its own.
 *  orc_spmv_canonical  the same sum in the fixed pairwise order: products
 *                      p_k = fl(val[k]*x[col[k]]) of row i, indexed by their
 *                      position r in the row, padded with -0.0 to the next
 *                      power of two, reduced level by level (leaf 2m with
 *                      2m+1, then pairs of pairs); an empty row gives +0.0.
 *
 * Error behaviour: functions return 0 on success, -1 on bad sizes, -2 when
 * a temporary cannot be allocated.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double jac_at(const double* u, int nx, int ny, int nz, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= nx || j >= ny || k >= nz) return 0.0;
    return u[((int64_t)k * ny + j) * nx + i];
}

int orc_jacobi7(const double* u0, double* out, int nx, int ny, int nz, int sweeps)
{
    if (nx < 0 || ny < 0 || nz < 0 || sweeps < 0) return -1;
    const int64_t n = (int64_t)nx * ny * nz;
    const double c = 1.0 / 6.0;
    if (n == 0) return 0;
    if (sweeps == 0) { memcpy(out, u0, (size_t)n * sizeof(double)); return 0; }
    double* a = (double*)malloc((size_t)n * sizeof(double));
    double* b = (double*)malloc((size_t)n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -2; }
    memcpy(a, u0, (size_t)n * sizeof(double));
    for (int s = 0; s < sweeps; ++s) {
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    double v = jac_at(a, nx, ny, nz, i - 1, j, k);
                    v = v + jac_at(a, nx, ny, nz, i + 1, j, k);
                    v = v + jac_at(a, nx, ny, nz, i, j - 1, k);
                    v = v + jac_at(a, nx, ny, nz, i, j + 1, k);
                    v = v + jac_at(a, nx, ny, nz, i, j, k - 1);
                    v = v + jac_at(a, nx, ny, nz, i, j, k + 1);
                    b[((int64_t)k * ny + j) * nx + i] = v * c;
                }
        double* t = a; a = b; b = t;
    }
    memcpy(out, a, (size_t)n * sizeof(double));
    free(a);
    free(b);
    return 0;
}

int orc_spmv_plain(int n, const int32_t* row_ptr, const int32_t* col, const double* val,
                   const double* x, double* y)
{
    if (n < 0) return -1;
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            double p = val[k] * x[col[k]];
            acc = acc + p;
        }
        y[i] = acc;
    }
    return 0;
}

int orc_spmv_canonical(int n, const int32_t* row_ptr, const int32_t* col, const double* val,
                       const double* x, double* y)
{
    if (n < 0) return -1;
    int32_t maxlen = 0;
    for (int i = 0; i < n; ++i) {
        int32_t len = row_ptr[i + 1] - row_ptr[i];
        if (len < 0) return -1;
        if (len > maxlen) maxlen = len;
    }
    int64_t cap = 1;
    while (cap < maxlen) cap *= 2;
    double* s = (double*)malloc((size_t)cap * sizeof(double));
    if (!s) return -2;
    for (int i = 0; i < n; ++i) {
        const int32_t b = row_ptr[i], len = row_ptr[i + 1] - b;
        if (len == 0) { y[i] = 0.0; continue; }
        int64_t width = 1;
        while (width < len) width *= 2;
        for (int64_t r = 0; r < width; ++r)
            s[r] = (r < len) ? val[b + r] * x[col[b + r]] : -0.0;
        /* level by level: node m of the next level = node 2m + node 2m+1 */
        for (int64_t w = width; w > 1; w /= 2)
            for (int64_t m = 0; m < w / 2; ++m)
                s[m] = s[2 * m] + s[2 * m + 1];
        y[i] = s[0];
    }
    free(s);
    return 0;
}

/* Weighted Jacobi relaxation (the AMGMk relax kernel of Table 3):
 * `sweeps` applications of x <- x + (omega * (b - A x)) / d, each row sum of
 * A x in the canonical order above, then one subtraction, one
 * multiplication, one division and one addition, each rounded (no FMA).
 * x is read, the last sweep lands in y; d holds the diagonal of A. */
int orc_relax(int n, const int32_t* row_ptr, const int32_t* col, const double* val,
              const double* x, const double* b, const double* d, double omega, int sweeps,
              double* y)
{
    if (n < 0 || sweeps < 0) return -1;
    double* cur = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double* ax = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!cur || !ax) { free(cur); free(ax); return -2; }
    memcpy(cur, x, (size_t)n * sizeof(double));
    for (int s = 0; s < sweeps; ++s) {
        int rc = orc_spmv_canonical(n, row_ptr, col, val, cur, ax);
        if (rc != 0) { free(cur); free(ax); return rc; }
        for (int i = 0; i < n; ++i) {
            double r = b[i] - ax[i];
            double t = omega * r;
            double u = t / d[i];
            cur[i] = cur[i] + u;
        }
    }
    memcpy(y, cur, (size_t)n * sizeof(double));
    free(cur);
    free(ax);
    return 0;
}
