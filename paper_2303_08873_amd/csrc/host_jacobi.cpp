// Host-CPU (OpenMP) variants of the 7-point FP64 Jacobi region: the
// "execution target" alternative of the paper's CPU-vs-GPU use case
// (Sec. 3.2, device selection).  Same arithmetic order as the GPU variants;
// built with -ffp-contract=off, so results are bit-identical to them.
//
// Tiling: the (k, j-tile, i-tile) space is shared by the OpenMP team; a tile
// is `by` rows of `bx` points (bx = 0: whole rows).  Ghost neighbours come
// from a zero row so that the inner loop is branch-free and vectorises.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/adaptomp.h"

namespace ao {

namespace {

constexpr double kC = 0x1.5555555555555p-3;  // fl(1/6)

void sweep(const double* __restrict__ src, double* __restrict__ dst, int nx, int ny, int nz,
           int bx, int by, const double* zeros) {
    const int tx = (bx <= 0 || bx > nx) ? nx : bx;
    const int ty = (by <= 0 || by > ny) ? ny : by;
    const int nti = (nx + tx - 1) / tx, ntj = (ny + ty - 1) / ty;
    const int64_t plane = (int64_t)nx * ny;
    const int64_t ntiles = (int64_t)nz * ntj * nti;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < ntiles; ++t) {
        const int ti = (int)(t % nti);
        const int tj = (int)((t / nti) % ntj);
        const int k = (int)(t / ((int64_t)nti * ntj));
        const int i0 = ti * tx, i1 = std::min(nx, i0 + tx);
        const int j0 = tj * ty, j1 = std::min(ny, j0 + ty);
        for (int j = j0; j < j1; ++j) {
            const double* c = src + k * plane + (int64_t)j * nx;
            const double* ym = j > 0 ? c - nx : zeros;
            const double* yp = j + 1 < ny ? c + nx : zeros;
            const double* zm = k > 0 ? c - plane : zeros;
            const double* zp = k + 1 < nz ? c + plane : zeros;
            double* d = dst + k * plane + (int64_t)j * nx;
            int i = i0;
            if (i == 0) {
                const double xp = nx > 1 ? c[1] : 0.0;
                double v = 0.0 + xp;
                v = v + ym[0];
                v = v + yp[0];
                v = v + zm[0];
                v = v + zp[0];
                d[0] = v * kC;
                i = 1;
            }
            const int iend = std::min(i1, nx - 1);
#pragma omp simd
            for (int ii = i; ii < iend; ++ii) {
                double v = c[ii - 1] + c[ii + 1];
                v = v + ym[ii];
                v = v + yp[ii];
                v = v + zm[ii];
                v = v + zp[ii];
                d[ii] = v * kC;
            }
            if (i1 == nx && nx - 1 >= i) {
                const int ii = nx - 1;
                double v = c[ii - 1] + 0.0;
                v = v + ym[ii];
                v = v + yp[ii];
                v = v + zm[ii];
                v = v + zp[ii];
                d[ii] = v * kC;
            }
        }
    }
}

}  // namespace

void jacobi_host_sweeps(const ao_variant& v, const double* u0, double* out, double* tmp, int nx,
                        int ny, int nz, int sweeps) {
    const int64_t n = (int64_t)nx * ny * nz;
    if (n == 0) return;
    if (sweeps == 0) {
        memcpy(out, u0, (size_t)n * sizeof(double));
        return;
    }
    std::vector<double> zeros((size_t)nx, 0.0);
    const double* src = u0;
    for (int s = 0; s < sweeps; ++s) {
        double* dst = ((sweeps - 1 - s) % 2 == 0) ? out : tmp;
        sweep(src, dst, nx, ny, nz, v.bx, v.by, zeros.data());
        src = dst;
    }
}

}  // namespace ao
