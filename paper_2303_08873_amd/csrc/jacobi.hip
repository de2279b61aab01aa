// GPU variants of the 7-point FP64 Jacobi region (gfx950, wave64).
//
// Every variant evaluates each point as
//   (((((xm + xp) + ym) + yp) + zm) + zp) * C,   C = fl(1/6),
// with +0.0 for neighbours outside the grid, in this exact order and with
// no contraction (the library is built with -ffp-contract=off), so all
// variants -- and the host variants -- return bit-identical results.
//
// Families:
//  direct  one thread per point, block bx*by over (x, y), one z-plane per
//          block row of the grid; neighbours come straight from global
//          memory (the L2 / Infinity Cache absorb the 6x re-reads).
//  zmarch  block bx*by owns an x-y tile and marches bz consecutive planes:
//          the z-neighbours stay in registers (below / cur / above) and the
//          in-plane neighbours come from an LDS copy of the plane tile plus
//          a one-point halo, so each interior point is read from global
//          memory once per sweep.
//
// Both map blockIdx.x to tiles XCD-aware: the hardware deals workgroups to
// the 8 XCDs round-robin, so consecutive logical tiles (which share z- and
// y-neighbour planes) are remapped to the same XCD and meet in its L2.
#include "internal.h"

namespace ao {
namespace {

constexpr double kC = 0x1.5555555555555p-3;  // fl(1/6)
constexpr unsigned kXcds = 8;

__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned n) {
    const unsigned xcd = b % kXcds, local = b / kXcds;
    const unsigned per = n / kXcds, rem = n % kXcds;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

template <bool NT>
__device__ __forceinline__ void store(double* p, double v) {
    if constexpr (NT) {
        __builtin_nontemporal_store(v, p);
    } else {
        *p = v;
    }
}

template <bool NT>
__global__ __launch_bounds__(1024) void jac_direct(const double* __restrict__ src,
                                                   double* __restrict__ dst, int nx, int ny,
                                                   int nz, int nbx, int nby, unsigned nblocks) {
    const unsigned b = xcd_remap(blockIdx.x, nblocks);
    const int bi = (int)(b % (unsigned)nbx);
    const unsigned t = b / (unsigned)nbx;
    const int bj = (int)(t % (unsigned)nby);
    const int k = (int)(t / (unsigned)nby);
    const int i = bi * (int)blockDim.x + (int)threadIdx.x;
    const int j = bj * (int)blockDim.y + (int)threadIdx.y;
    if (i >= nx || j >= ny || k >= nz) return;
    const size_t plane = (size_t)nx * (size_t)ny;
    const size_t idx = (size_t)k * plane + (size_t)j * (size_t)nx + (size_t)i;
    const double xm = i > 0 ? src[idx - 1] : 0.0;
    const double xp = i + 1 < nx ? src[idx + 1] : 0.0;
    const double ym = j > 0 ? src[idx - nx] : 0.0;
    const double yp = j + 1 < ny ? src[idx + nx] : 0.0;
    const double zm = k > 0 ? src[idx - plane] : 0.0;
    const double zp = k + 1 < nz ? src[idx + plane] : 0.0;
    double v = xm + xp;
    v = v + ym;
    v = v + yp;
    v = v + zm;
    v = v + zp;
    store<NT>(dst + idx, v * kC);
}

template <bool NT>
__global__ __launch_bounds__(1024) void jac_zmarch(const double* __restrict__ src,
                                                   double* __restrict__ dst, int nx, int ny,
                                                   int nz, int nbx, int nby, int bz,
                                                   unsigned nblocks) {
    extern __shared__ double tile[];  // (BY + 2) rows of (BX + 2)
    const int BX = (int)blockDim.x, BY = (int)blockDim.y, W = BX + 2;
    const unsigned b = xcd_remap(blockIdx.x, nblocks);
    const int bi = (int)(b % (unsigned)nbx);
    const unsigned t = b / (unsigned)nbx;
    const int bj = (int)(t % (unsigned)nby);
    const int kb = (int)(t / (unsigned)nby);
    const int tx = (int)threadIdx.x, ty = (int)threadIdx.y;
    const int i = bi * BX + tx, j = bj * BY + ty;
    const bool in = (i < nx) && (j < ny);
    const int k0 = kb * bz;
    const int k1 = min(nz, k0 + bz);
    const size_t plane = (size_t)nx * (size_t)ny;
    const size_t col = in ? (size_t)j * (size_t)nx + (size_t)i : 0;
    double below = (in && k0 > 0) ? src[(size_t)(k0 - 1) * plane + col] : 0.0;
    double cur = in ? src[(size_t)k0 * plane + col] : 0.0;
    double* const c = tile + (ty + 1) * W + (tx + 1);
    for (int k = k0; k < k1; ++k) {
        const double above = (in && k + 1 < nz) ? src[(size_t)(k + 1) * plane + col] : 0.0;
        const double* sp = src + (size_t)k * plane;
        __syncthreads();  // the previous plane's LDS reads are done
        c[0] = cur;
        if (tx == 0) c[-1] = (i > 0 && j < ny) ? sp[(size_t)j * nx + (i - 1)] : 0.0;
        if (tx == BX - 1) c[1] = (i + 1 < nx && j < ny) ? sp[(size_t)j * nx + (i + 1)] : 0.0;
        if (ty == 0) c[-W] = (j > 0 && i < nx) ? sp[(size_t)(j - 1) * nx + i] : 0.0;
        if (ty == BY - 1) c[W] = (j + 1 < ny && i < nx) ? sp[(size_t)(j + 1) * nx + i] : 0.0;
        __syncthreads();
        if (in) {
            double v = c[-1] + c[1];
            v = v + c[-W];
            v = v + c[W];
            v = v + below;
            v = v + above;
            store<NT>(dst + (size_t)k * plane + col, v * kC);
        }
        below = cur;
        cur = above;
    }
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

}  // namespace

hipError_t jacobi_gpu_sweep(const ao_variant& v, const double* src, double* dst, int nx, int ny,
                            int nz, hipStream_t s) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return hipSuccess;
    const int bx = v.bx, by = v.by;
    if (bx <= 0 || by <= 0 || (int64_t)bx * by > 1024 || (bx * by) % 64 != 0)
        return hipErrorInvalidConfiguration;
    const bool nt = (v.flags & AO_VF_NT_STORE) != 0;
    const int nbx = cdiv(nx, bx), nby = cdiv(ny, by);
    if (v.family == AO_FAM_JACOBI_DIRECT) {
        const int64_t nb = (int64_t)nbx * nby * nz;
        if (nb > 0x7fffffff) return hipErrorInvalidConfiguration;
        const dim3 grid((unsigned)nb), block(bx, by);
        if (nt)
            hipLaunchKernelGGL(jac_direct<true>, grid, block, 0, s, src, dst, nx, ny, nz, nbx, nby,
                               (unsigned)nb);
        else
            hipLaunchKernelGGL(jac_direct<false>, grid, block, 0, s, src, dst, nx, ny, nz, nbx,
                               nby, (unsigned)nb);
        return hipGetLastError();
    }
    if (v.family == AO_FAM_JACOBI_ZMARCH) {
        const int bz = v.bz;
        if (bz <= 0) return hipErrorInvalidConfiguration;
        const size_t lds = (size_t)(bx + 2) * (by + 2) * sizeof(double);
        if (lds > 64 * 1024) return hipErrorInvalidConfiguration;
        const int64_t nb = (int64_t)nbx * nby * cdiv(nz, bz);
        if (nb > 0x7fffffff) return hipErrorInvalidConfiguration;
        const dim3 grid((unsigned)nb), block(bx, by);
        if (nt)
            hipLaunchKernelGGL(jac_zmarch<true>, grid, block, lds, s, src, dst, nx, ny, nz, nbx,
                               nby, bz, (unsigned)nb);
        else
            hipLaunchKernelGGL(jac_zmarch<false>, grid, block, lds, s, src, dst, nx, ny, nz, nbx,
                               nby, bz, (unsigned)nb);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

}  // namespace ao
