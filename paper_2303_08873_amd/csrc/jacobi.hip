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
//  zreg    no LDS and no barriers: each wave owns a (64*VX)-wide x strip of
//          R rows and marches bz planes.  Plane k-1, k and k+1 of its R rows
//          live in registers (the plane k+1 rows are the loads issued in
//          iteration k), the x-neighbours come from the adjacent lanes by
//          cross-lane moves (the two strip edges are loaded by lanes 0 and
//          63), the y-neighbours from the wave's own rows plus two halo rows.
//          A block is 4 such waves stacked in y (tile 64*VX x 4R).  With the
//          halo-prefetch flag the halo of plane k+1 is also loaded during
//          plane k, so no iteration waits on its own loads.
//  zreg_t2 the register z-march with two sweeps fused per pass (temporal
//          blocking): half the HBM traffic per sweep; strips of 64 lanes
//          overlap by one point per side so the intermediate sweep's
//          x-neighbours stay inside the wave (62 outputs per strip).
//
// All map blockIdx.x to tiles XCD-aware: the hardware deals workgroups to
// the 8 XCDs round-robin, so consecutive logical tiles (which share z- and
// y-neighbour planes) are remapped to the same XCD and meet in its L2.
#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.h"
#include "lanes.h"
#include "zmarch.h"

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

// All S sweeps of a grid of at most kLdsPoints points in one workgroup: the
// grid and its next sweep live in LDS (two copies), one barrier per sweep.
// Each thread owns the points tid + 1024 m and keeps their neighbour masks
// (bit 0..5: x-1, x+1, y-1, y+1, z-1, z+1 inside the grid) across sweeps.
// Same sum order and ghost values as jac_direct.
constexpr int kLdsPoints = 8192;
constexpr int kLdsPer = kLdsPoints / 1024;
__global__ __launch_bounds__(1024) void jac_lds_sweeps(const double* __restrict__ src,
                                                       double* __restrict__ dst, int nx, int ny,
                                                       int nz, int sweeps) {
    __shared__ double g[2][kLdsPoints];
    const int n = nx * ny * nz, plane = nx * ny, tid = (int)threadIdx.x;
    int mask[kLdsPer];
#pragma unroll
    for (int m = 0; m < kLdsPer; ++m) {
        const int p = tid + 1024 * m;
        mask[m] = 0;
        if (p < n) {
            const int i = p % nx, t = p / nx, j = t % ny, k = t / ny;
            mask[m] = (i > 0) | (i + 1 < nx) << 1 | (j > 0) << 2 | (j + 1 < ny) << 3 |
                      (k > 0) << 4 | (k + 1 < nz) << 5;
            g[0][p] = src[p];
        }
    }
    __syncthreads();
    int cur = 0;
    for (int s = 0; s < sweeps; ++s) {
        const double* a = g[cur];
        double* b = g[cur ^ 1];
#pragma unroll
        for (int m = 0; m < kLdsPer; ++m) {
            const int p = tid + 1024 * m;
            if (p < n) {
                const int f = mask[m];
                const double xm = (f & 1) ? a[p - 1] : 0.0;
                const double xp = (f & 2) ? a[p + 1] : 0.0;
                const double ym = (f & 4) ? a[p - nx] : 0.0;
                const double yp = (f & 8) ? a[p + nx] : 0.0;
                const double zm = (f & 16) ? a[p - plane] : 0.0;
                const double zp = (f & 32) ? a[p + plane] : 0.0;
                double v = xm + xp;
                v = v + ym;
                v = v + yp;
                v = v + zm;
                v = v + zp;
                b[p] = v * kC;
            }
        }
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int m = 0; m < kLdsPer; ++m) {
        const int p = tid + 1024 * m;
        if (p < n) dst[p] = g[cur][p];
    }
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

constexpr int kZregWaves = 4;

template <int VX>
struct Vec;
template <>
struct Vec<1> {
    double v[1];
};
template <>
struct Vec<2> {
    double v[2];
};

// Load VX consecutive points of one row starting at x = i (zero outside the
// grid or when `ok` is false).
template <int VX>
__device__ __forceinline__ Vec<VX> load_row(const double* __restrict__ row, int i, int nx,
                                            bool ok) {
    Vec<VX> r;
    if constexpr (VX == 2) {
        if (ok && i + 1 < nx) {
            const double2 t = *reinterpret_cast<const double2*>(row + i);
            r.v[0] = t.x;
            r.v[1] = t.y;
        } else {
            r.v[0] = (ok && i < nx) ? row[i] : 0.0;
            r.v[1] = 0.0;
        }
    } else {
        r.v[0] = (ok && i < nx) ? row[i] : 0.0;
    }
    return r;
}

template <int R, int VX, bool NT, bool PF>
__global__ __launch_bounds__(64 * kZregWaves) void jac_zreg(const double* __restrict__ src,
                                                             double* __restrict__ dst, int nx,
                                                             int ny, int nz, int nbx, int nby,
                                                             int bz, unsigned nblocks) {
    constexpr int TW = 64 * VX;
    const unsigned b = xcd_remap(blockIdx.x, nblocks);
    const int bi = (int)(b % (unsigned)nbx);
    const unsigned t = b / (unsigned)nbx;
    const int bj = (int)(t % (unsigned)nby);
    const int kb = (int)(t / (unsigned)nby);
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int i0 = bi * TW;
    const int i = i0 + lane * VX;
    const int j0 = (bj * kZregWaves + wave) * R;
    if (j0 >= ny) return;  // whole wave outside the grid (uniform)
    const int k0 = kb * bz;
    const int k1 = min(nz, k0 + bz);
    const size_t plane = (size_t)nx * (size_t)ny;
    // edge lanes fetch the neighbour just outside the strip
    const int ie = (lane == 0) ? i0 - 1 : i0 + TW;
    const bool edge = (lane == 0 && i0 > 0) || (lane == 63 && i0 + TW < nx);
    auto row_ptr = [&](int k, int j) { return src + (size_t)k * plane + (size_t)j * nx; };
    // in-plane halo of plane k: rows j0-1 and j0+R, and the two strip edges
    struct Halo {
        Vec<VX> ym, yp;
        double ex[R];
    };
    auto load_halo = [&](int k, Halo& h) {
        const bool ok = k < nz;
        h.ym = load_row<VX>(row_ptr(min(k, nz - 1), max(j0 - 1, 0)), i, nx, ok && j0 > 0);
        h.yp = load_row<VX>(row_ptr(min(k, nz - 1), min(j0 + R, ny - 1)), i, nx, ok && j0 + R < ny);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool okj = j0 + r < ny;
            h.ex[r] = (ok && edge && okj) ? row_ptr(min(k, nz - 1), min(j0 + r, ny - 1))[ie] : 0.0;
        }
    };

    Vec<VX> below[R], cur[R], above[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool okj = j0 + r < ny;
        below[r] = load_row<VX>(k0 > 0 ? row_ptr(k0 - 1, min(j0 + r, ny - 1)) : src, i, nx,
                                okj && k0 > 0);
        cur[r] = load_row<VX>(row_ptr(k0, min(j0 + r, ny - 1)), i, nx, okj);
    }
    Halo hc;
    if constexpr (PF) load_halo(k0, hc);
    for (int k = k0; k < k1; ++k) {
        const bool has_up = k + 1 < nz;
        Halo hn;
        if constexpr (PF) {
            load_halo(k + 1, hn);  // consumed next iteration
        } else {
            load_halo(k, hc);      // consumed now
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool okj = j0 + r < ny;
            above[r] = load_row<VX>(has_up ? row_ptr(k + 1, min(j0 + r, ny - 1)) : src, i, nx,
                                    okj && has_up);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = j0 + r;
            // x neighbours: within the lane, then across lanes
            const double left = from_left(cur[r].v[VX - 1]);
            const double right = from_right(cur[r].v[0]);
            const double xl = (lane == 0) ? hc.ex[r] : left;
            const double xr = (lane == 63) ? hc.ex[r] : right;
#pragma unroll
            for (int q = 0; q < VX; ++q) {
                const double xm = (q == 0) ? xl : cur[r].v[q - 1];
                const double xp = (q == VX - 1) ? xr : cur[r].v[q + 1];
                const double ym = (r == 0) ? hc.ym.v[q] : cur[r - 1].v[q];
                const double yp = (r == R - 1) ? hc.yp.v[q] : cur[r + 1].v[q];
                double v = xm + xp;
                v = v + ym;
                v = v + yp;
                v = v + below[r].v[q];
                v = v + above[r].v[q];
                if (j < ny && i + q < nx)
                    store<NT>(dst + (size_t)k * plane + (size_t)j * nx + (i + q), v * kC);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            below[r] = cur[r];
            cur[r] = above[r];
        }
        if constexpr (PF) hc = hn;
    }
}

// Two sweeps per pass (temporal blocking factor 2).  A wave owns 64 lanes
// of x starting at i0 = 62*bi - 1 and R output rows; it keeps the input u on
// rows j0-2 .. j0+R+1 for planes k-1, k, k+1 and the first-sweep values v on
// rows j0-1 .. j0+R for planes k-2, k-1, k, all in registers.  In iteration
// k it loads u(k+1), computes v(k) on all 64 lanes (strip edges from lanes 0
// and 63's extra loads), then w(k-1) = J(v) on lanes 1..62.  v at positions
// outside the grid is forced to +0.0 -- the ghost value a separate second
// sweep would read -- so w is bit-identical to two sweeps.  With PF the
// loads of plane k+2 (and the strip edges of plane k+1) are issued during
// iteration k, so an iteration never waits on loads it issued itself.
template <int R, bool NT, bool PF>
__device__ __forceinline__ void zreg_t2_body(const double* __restrict__ src,
                                             double* __restrict__ dst, int nx, int ny, int nz,
                                             int nbx, int nby, int bz, unsigned nblocks) {
    constexpr int RU = R + 4, RV = R + 2;
    const unsigned b = xcd_remap(blockIdx.x, nblocks);
    const int bi = (int)(b % (unsigned)nbx);
    const unsigned t = b / (unsigned)nbx;
    const int bj = (int)(t % (unsigned)nby);
    const int kb = (int)(t / (unsigned)nby);
    const int lane = (int)(threadIdx.x & 63);
    const int wave = wave_index();
    const int i0 = 62 * bi - 1;
    const int i = i0 + lane;
    const int j0 = (bj * kZregWaves + wave) * R;
    if (j0 >= ny) return;  // wave-uniform
    const int k0 = kb * bz;
    const int k1 = min(nz, k0 + bz);
    const size_t plane = (size_t)nx * (size_t)ny;
    const bool xin = i >= 0 && i < nx;
    const int ie = (lane == 0) ? i0 - 1 : i0 + 64;
    const bool eok = (lane == 0 || lane == 63) && ie >= 0 && ie < nx;
    // unmasked loads at clamped (wave-uniform) rows and planes and clamped x,
    // zeroed afterwards outside the grid (nx * 8 < 2^32 on the host side)
    const unsigned bo = (unsigned)min(max(i, 0), nx - 1) * 8u;
    const unsigned boe = (unsigned)min(max(ie, 0), nx - 1) * 8u;
    auto ld = [&](int k, int j, unsigned off, bool ok) -> double {
        const bool in = k >= 0 && k < nz && j >= 0 && j < ny;  // wave-uniform
        const int kc = min(max(k, 0), nz - 1), jc = min(max(j, 0), ny - 1);
        const char* row = (const char*)(src + ((size_t)kc * plane + (size_t)jc * nx));
        const double v = *(const double*)(row + off);
        return (ok && in) ? v : 0.0;
    };
    // registers hold only the rows each plane is read at:
    //   um[q] = u(k-1) on rows j0-1+q   (centre rows of v)
    //   uc[q], up[q] = u(k), u(k+1) on rows j0-2+q
    //   vm[r] = v(k-2) on rows j0+r     (centre rows of w)
    //   vc[q], vn[q] = v(k-1), v(k) on rows j0-1+q
    double um[RV], uc[RU], up[RU];
    double vm[R], vc[RV], vn[RV];
#pragma unroll
    for (int q = 0; q < RV; ++q) um[q] = ld(k0 - 2, j0 - 1 + q, bo, xin);
#pragma unroll
    for (int q = 0; q < RU; ++q) uc[q] = ld(k0 - 1, j0 - 2 + q, bo, xin);
#pragma unroll
    for (int r = 0; r < R; ++r) vm[r] = 0.0;  // v(k0-3) is never read
#pragma unroll
    for (int q = 0; q < RV; ++q) vc[q] = 0.0;  // v(k0-2) only feeds w(k0-1), never stored
    double upn[PF ? RU : 1], exn[PF ? RV : 1];
    if constexpr (PF) {
#pragma unroll
        for (int q = 0; q < RU; ++q) upn[q] = ld(k0, j0 - 2 + q, bo, xin);
#pragma unroll
        for (int q = 0; q < RV; ++q) exn[q] = ld(k0 - 1, j0 - 1 + q, boe, eok);
    }
    for (int k = k0 - 1; k <= k1; ++k) {
        double ex[RV];
        if constexpr (PF) {
#pragma unroll
            for (int q = 0; q < RU; ++q) up[q] = upn[q];
#pragma unroll
            for (int q = 0; q < RV; ++q) ex[q] = exn[q];
            if (k < k1) {  // wave-uniform; plane k+2 / edges of k+1 for the next iteration
#pragma unroll
                for (int q = 0; q < RU; ++q) upn[q] = ld(k + 2, j0 - 2 + q, bo, xin);
#pragma unroll
                for (int q = 0; q < RV; ++q) exn[q] = ld(k + 1, j0 - 1 + q, boe, eok);
            }
        } else {
#pragma unroll
            for (int q = 0; q < RU; ++q) up[q] = ld(k + 1, j0 - 2 + q, bo, xin);
#pragma unroll
            for (int q = 0; q < RV; ++q) ex[q] = ld(k, j0 - 1 + q, boe, eok);
        }
        // v(k) on rows j0-1 .. j0+R, all lanes
        const bool kin = k >= 0 && k < nz;
#pragma unroll
        for (int q = 0; q < RV; ++q) {
            const int j = j0 - 1 + q;
            const double c = uc[q + 1];
            const double xm = from_left_or(c, ex[q]), xp = from_right_or(c, ex[q]);
            double v = xm + xp;
            v = v + uc[q];
            v = v + uc[q + 2];
            v = v + um[q];
            v = v + up[q + 1];
            vn[q] = (kin && xin && j >= 0 && j < ny) ? v * kC : 0.0;
        }
        // w(k-1) on rows j0 .. j0+R-1, lanes 1..62
        const int kw = k - 1;
        if (kw >= k0 && kw < k1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int j = j0 + r;
                const double c = vc[r + 1];
                const double xm = from_left(c), xp = from_right(c);
                double w = xm + xp;
                w = w + vc[r];
                w = w + vc[r + 2];
                w = w + vm[r];
                w = w + vn[r + 1];
                if (lane >= 1 && lane <= 62 && xin && j < ny)
                    store<NT>(dst + (size_t)kw * plane + (size_t)j * nx + i, w * kC);
            }
        }
#pragma unroll
        for (int q = 0; q < RV; ++q) um[q] = uc[q + 1];
#pragma unroll
        for (int q = 0; q < RU; ++q) uc[q] = up[q];
#pragma unroll
        for (int r = 0; r < R; ++r) vm[r] = vc[r + 1];
#pragma unroll
        for (int q = 0; q < RV; ++q) vc[q] = vn[q];
    }
}

template <int R, bool NT, bool PF>
__global__ __launch_bounds__(64 * kZregWaves) void jac_zreg_t2(const double* __restrict__ src,
                                                                double* __restrict__ dst, int nx,
                                                                int ny, int nz, int nbx, int nby,
                                                                int bz, unsigned nblocks) {
    zreg_t2_body<R, NT, PF>(src, dst, nx, ny, nz, nbx, nby, bz, nblocks);
}

// The same kernel compiled for at least 4 waves per SIMD (register budget
// 128; the compiler may spill a little).
template <int R, bool NT, bool PF>
__global__ __launch_bounds__(64 * kZregWaves) __attribute__((amdgpu_waves_per_eu(4, 8)))
void jac_zreg_t2_occ(const double* __restrict__ src, double* __restrict__ dst, int nx, int ny,
                     int nz, int nbx, int nby, int bz, unsigned nblocks) {
    zreg_t2_body<R, NT, PF>(src, dst, nx, ny, nz, nbx, nby, bz, nblocks);
}

// T sweeps per pass (temporal blocking factor T >= 2), the two-sweep scheme
// generalised: one wave runs tb_column (zmarch.h) on its 64-lane strip,
// starting at i0 = (66 - 2T)*bi - (T - 1), storing lanes T-1 .. 64-T.  PF
// selects the march's early next-plane loads, ST the staged (global->LDS)
// level 0 for waves inside the grid.
template <int T, int R, bool NT, bool PF, bool ST>
__device__ __forceinline__ void zreg_tb_body(const double* __restrict__ src,
                                             double* __restrict__ dst, int nx, int ny, int nz,
                                             int nbx, int nby, int bz, unsigned nblocks) {
    constexpr int W = 66 - 2 * T;
    const unsigned b = xcd_remap(blockIdx.x, nblocks);
    const int bi = (int)(b % (unsigned)nbx);
    const unsigned t = b / (unsigned)nbx;
    const int bj = (int)(t % (unsigned)nby);
    const int kb = (int)(t / (unsigned)nby);
    const int wave = wave_index();
    const int j0 = (bj * kZregWaves + wave) * R;
    if (j0 >= ny) return;  // wave-uniform
    const int k0 = kb * bz;
    const int i0 = W * bi - (T - 1);
    // every column (with the strip-edge loads) and row (with the T-row halo)
    // the wave touches inside the grid: the march without per-lane selects
    const bool inner = i0 >= 1 && i0 + 64 < nx && j0 >= T && j0 + R + T <= ny;  // wave-uniform
    if constexpr (ST && !PF) {
        // staged level 0: columns x0 .. x0+67 from the even x0 = i0-2 or i0-3
        const int x0 = i0 - 2 - (i0 & 1);
        const bool fits = nx >= 2 && (size_t)nx * (size_t)ny * 8u < ((size_t)1 << 32) &&
                          (!(nx & 1) || x0 + 68 <= nx);  // wave-uniform
        // boundary waves stage too where the extra selects still fit two
        // waves per SIMD (up to 4 rows per wave for four sweeps, 6 for three)
        constexpr bool kEdges = (T == 4 && R <= 4) || (T == 3 && R <= 6);
        __shared__ __attribute__((aligned(16))) char stg[zm::stage_lds_bytes<T, R>()];
        if (fits && inner && x0 >= 0 && x0 + 68 <= nx) {
            zm::tb_column<T, R, NT, false, true, true, true>(src, dst, nx, ny, nz, i0, j0, k0,
                                                             min(nz, k0 + bz), T - 1, 64 - T, stg);
            return;
        }
        if constexpr (kEdges) {
            if (fits) {
                zm::tb_column<T, R, NT, false, true, false, true>(src, dst, nx, ny, nz, i0, j0, k0,
                                                                  min(nz, k0 + bz), T - 1, 64 - T,
                                                                  stg);
                return;
            }
        }
    }
    if (inner)
        zm::tb_column<T, R, NT, PF, true, true>(src, dst, nx, ny, nz, i0, j0, k0, min(nz, k0 + bz),
                                                T - 1, 64 - T);
    else
        zm::tb_column<T, R, NT, PF>(src, dst, nx, ny, nz, i0, j0, k0, min(nz, k0 + bz), T - 1,
                                    64 - T);
}

template <int T, int R, bool NT, bool PF, bool ST>
__global__ __launch_bounds__(64 * kZregWaves) void jac_zreg_tb(const double* __restrict__ src,
                                                                double* __restrict__ dst, int nx,
                                                                int ny, int nz, int nbx, int nby,
                                                                int bz, unsigned nblocks) {
    zreg_tb_body<T, R, NT, PF, ST>(src, dst, nx, ny, nz, nbx, nby, bz, nblocks);
}

// Every register z-march kernel takes (src, dst, nx, ny, nz, nbx, nby, bz,
// blocks) and runs 4-wave workgroups over nbx * nby columns of blocks times
// ceil(nz / bz) z-chunks.
using ColumnKernel = void (*)(const double*, double*, int, int, int, int, int, int, unsigned);

template <int T, int R>
ColumnKernel pick_zreg_tb(bool nt, bool pf, bool st) {
    if (st && nt) return jac_zreg_tb<T, R, true, false, true>;
    if (st) return jac_zreg_tb<T, R, false, false, true>;
    if (nt && pf) return jac_zreg_tb<T, R, true, true, false>;
    if (nt) return jac_zreg_tb<T, R, true, false, false>;
    if (pf) return jac_zreg_tb<T, R, false, true, false>;
    return jac_zreg_tb<T, R, false, false, false>;
}

template <int R, bool PF>
ColumnKernel pick_zreg_t2(bool nt, bool occ) {
    if (occ && nt) return jac_zreg_t2_occ<R, true, PF>;
    if (occ) return jac_zreg_t2_occ<R, false, PF>;
    if (nt) return jac_zreg_t2<R, true, PF>;
    return jac_zreg_t2<R, false, PF>;
}

template <int R, int VX>
ColumnKernel pick_zreg(bool nt, bool pf) {
    if (nt && pf) return jac_zreg<R, VX, true, true>;
    if (nt) return jac_zreg<R, VX, true, false>;
    if (pf) return jac_zreg<R, VX, false, true>;
    return jac_zreg<R, VX, false, false>;
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Throughput of a CU running two, or three and more, of a register
// z-march's workgroups at once, relative to one (they hide each other's
// latencies), and the cost margin within which fill_planes takes fewer,
// longer chunks (less halo traffic).  Fitted on MI355X to a sweep of 13 and
// 14 chunk lengths of the staged three- and four-sweep marches over 50
// grids (40 of the cost model's shape law, 10 cubes and slabs): among the
// measured lengths the rule's picks run within 0.3% (three sweeps) and
// 0.4% (four) of the fastest, geometric mean.
constexpr double kFillGain2 = 1.4, kFillGain3 = 1.5, kFillTolerance = 0.03;

// CUs of the current device and workgroups of kernel k each keeps resident
// at once (its occupancy), cached per kernel and device; false when the
// runtime cannot say.
bool residency(ColumnKernel k, int* cus, int* per_cu) {
    static std::mutex mu;
    static std::vector<std::pair<std::pair<const void*, int>, std::pair<int, int>>> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const std::pair<const void*, int> key((const void*)k, dev);
    std::lock_guard<std::mutex> g(mu);
    for (const auto& e : cache)
        if (e.first == key) {
            *cus = e.second.first;
            *per_cu = e.second.second;
            return true;
        }
    int occ = 0, n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k, 64 * kZregWaves, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    cache.push_back({key, {n, occ}});
    *cus = n;
    *per_cu = occ;
    return true;
}

// What a full launch of a register z-march variant runs: its kernel, the
// sweeps it fuses and its nbx * nby columns of blocks.
struct ColumnShape {
    ColumnKernel k = nullptr;
    int T = 1, nbx = 0, nby = 0;
};

// The shape of variant v on an nx * ny * nz grid (all positive), after the
// host-side checks of its family; hipErrorInvalidConfiguration when the
// variant does not fit a kernel.
hipError_t column_shape(const ao_variant& v, int nx, int ny, int nz, ColumnShape* c) {
    const bool nt = (v.flags & AO_VF_NT_STORE) != 0;
    const bool pf = (v.flags & AO_VF_HALO_PREFETCH) != 0;
    const int R = v.by;
    if (v.bz <= 0 || nz <= 0) return hipErrorInvalidConfiguration;
    if (v.family == AO_FAM_JACOBI_ZREG) {
        // strips of bx = 64 or 128 points (128: an even nx), by rows per wave
        const int VX = v.bx / 64;
        if (v.bx != 64 && v.bx != 128) return hipErrorInvalidConfiguration;
        if (VX == 2 && (nx & 1)) return hipErrorInvalidConfiguration;
#define AO_ZREG(RR, VV) \
    if (R == RR && VX == VV) c->k = pick_zreg<RR, VV>(nt, pf);
        AO_ZREG(1, 1) AO_ZREG(2, 1) AO_ZREG(4, 1) AO_ZREG(8, 1)
        AO_ZREG(1, 2) AO_ZREG(2, 2) AO_ZREG(4, 2) AO_ZREG(8, 2)
#undef AO_ZREG
        c->T = 1;
        c->nbx = cdiv(nx, v.bx);
    } else if (v.family == AO_FAM_JACOBI_ZREG_T2) {
        const bool occ = (v.flags & AO_VF_OCCUPANCY) != 0;
        if (v.bx != 64 || nx > (1 << 28)) return hipErrorInvalidConfiguration;
#define AO_T2(RR) \
    if (R == RR) c->k = pf ? pick_zreg_t2<RR, true>(nt, occ) : pick_zreg_t2<RR, false>(nt, occ);
        AO_T2(1) AO_T2(2) AO_T2(3) AO_T2(4) AO_T2(6) AO_T2(8) AO_T2(10) AO_T2(12) AO_T2(16)
#undef AO_T2
        c->T = 2;
        c->nbx = cdiv(nx, 62);
    } else if (v.family == AO_FAM_JACOBI_ZREG_T3 || v.family == AO_FAM_JACOBI_ZREG_T4) {
        const int T = v.family == AO_FAM_JACOBI_ZREG_T3 ? 3 : 4;
        const bool st = (v.flags & AO_VF_STAGED) != 0;
        if (v.bx != 64 || nx > (1 << 28) || (st && pf)) return hipErrorInvalidConfiguration;
#define AO_TB(TT, RR) \
    if (T == TT && R == RR) c->k = pick_zreg_tb<TT, RR>(nt, pf, st);
        AO_TB(3, 1) AO_TB(3, 2) AO_TB(3, 3) AO_TB(3, 4) AO_TB(3, 5) AO_TB(3, 6) AO_TB(3, 8)
        AO_TB(4, 1) AO_TB(4, 2) AO_TB(4, 3) AO_TB(4, 4) AO_TB(4, 5)
#undef AO_TB
        c->T = T;
        c->nbx = cdiv(nx, 66 - 2 * T);
    }
    if (!c->k) return hipErrorInvalidConfiguration;
    c->nby = cdiv(ny, kZregWaves * R);
    return hipSuccess;
}

// Planes per block of a launch of shape c for variant v: v.bz, or with
// AO_VF_FILL_Z the chunk fill_planes picks for `cus` CUs holding `per_cu`
// of its workgroups each (the kernel's own residency on the current device
// when cus <= 0; v.bz if the runtime cannot say).
int column_planes(const ao_variant& v, const ColumnShape& c, int nz, int cus, int per_cu) {
    if (!(v.flags & AO_VF_FILL_Z)) return v.bz;
    if (cus <= 0 && !residency(c.k, &cus, &per_cu)) return v.bz;
    return fill_planes((int64_t)c.nbx * c.nby, nz, v.bz, 2 * (c.T - 1), cus, per_cu);
}

// One launch of a register z-march variant: src -> dst.
hipError_t launch_columns(const ao_variant& v, hipStream_t s, const double* src, double* dst,
                          int nx, int ny, int nz) {
    ColumnShape c;
    const hipError_t e = column_shape(v, nx, ny, nz, &c);
    if (e != hipSuccess) return e;
    const int bz = column_planes(v, c, nz, 0, 0);
    const int64_t nb = (int64_t)c.nbx * c.nby * ((nz + bz - 1) / bz);
    if (bz <= 0 || nb > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(c.k, dim3((unsigned)nb), dim3(64 * kZregWaves), 0, s, src, dst, nx, ny, nz,
                       c.nbx, c.nby, bz, (unsigned)nb);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy(const double* __restrict__ src,
                                              double* __restrict__ dst, int64_t n, int nt) {
    const int64_t base = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (base + 3 < n) {
        const double2 a = *reinterpret_cast<const double2*>(src + base);
        const double2 c = *reinterpret_cast<const double2*>(src + base + 2);
        if (nt) {
            __builtin_nontemporal_store(a.x, dst + base);
            __builtin_nontemporal_store(a.y, dst + base + 1);
            __builtin_nontemporal_store(c.x, dst + base + 2);
            __builtin_nontemporal_store(c.y, dst + base + 3);
        } else {
            *reinterpret_cast<double2*>(dst + base) = a;
            *reinterpret_cast<double2*>(dst + base + 2) = c;
        }
    } else {
        for (int64_t q = base; q < n; ++q) dst[q] = src[q];
    }
}

}  // namespace

int fill_planes(int64_t columns, int nz, int bz_max, int halo, int cus, int per_cu) {
    const int top = std::min(bz_max, nz);
    if (top < 1 || columns < 1 || cus < 1) return std::max(top, 1);
    const int lo = std::max(1, top - 4095);
    const int64_t k = std::max(per_cu, 1);
    auto gain = [](int64_t j) { return j >= 3 ? kFillGain3 : j == 2 ? kFillGain2 : 1.0; };
    auto cost = [&](int bz) {
        const int64_t blocks = columns * ((nz + bz - 1) / bz);
        const int64_t n = (blocks + cus - 1) / cus;  // workgroups on the busiest CU
        // rounds of k at once, then the n mod k left over
        const int64_t full = n / k, r = n % k;
        return (double)(bz + halo) *
               ((double)(full * k) / gain(k) + (r ? (double)r / gain(r) : 0.0));
    };
    double best = cost(top);
    for (int bz = top - 1; bz >= lo; --bz) best = std::min(best, cost(bz));
    // the fewest chunks within the margin, cut into equal lengths
    int chunks = INT32_MAX;
    for (int bz = top; bz >= lo; --bz)
        if (cost(bz) <= best * (1.0 + kFillTolerance)) chunks = std::min(chunks, (nz + bz - 1) / bz);
    return chunks == INT32_MAX ? top : (nz + chunks - 1) / chunks;
}

bool lds_sweeps_fit(int nx, int ny, int nz) {
    return nx > 0 && ny > 0 && nz > 0 && (int64_t)nx * ny * nz <= kLdsPoints;
}

hipError_t jacobi_gpu_lds_sweeps(const double* src, double* dst, int nx, int ny, int nz,
                                 int sweeps, hipStream_t s) {
    if (!lds_sweeps_fit(nx, ny, nz) || sweeps < 0) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(jac_lds_sweeps, dim3(1), dim3(1024), 0, s, src, dst, nx, ny, nz, sweeps);
    return hipGetLastError();
}

hipError_t jacobi_gpu_sweep(const ao_variant& v, const double* src, double* dst, int nx, int ny,
                            int nz, hipStream_t s) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return hipSuccess;
    const int bx = v.bx, by = v.by;
    if (bx <= 0 || by <= 0) return hipErrorInvalidConfiguration;
    if (v.family != AO_FAM_JACOBI_ZREG && ((int64_t)bx * by > 1024 || (bx * by) % 64 != 0))
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
    if (v.family == AO_FAM_JACOBI_ZREG) {
        // a 128-point strip takes 16-byte accesses
        if (bx == 128 && (((uintptr_t)src & 15) || ((uintptr_t)dst & 15)))
            return hipErrorInvalidConfiguration;
        return launch_columns(v, s, src, dst, nx, ny, nz);
    }
    return hipErrorInvalidValue;
}

hipError_t jacobi_gpu_double_sweep(const ao_variant& v, const double* src, double* dst, int nx,
                                  int ny, int nz, hipStream_t s) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return hipSuccess;
    if (v.family != AO_FAM_JACOBI_ZREG_T2) return hipErrorInvalidConfiguration;
    return launch_columns(v, s, src, dst, nx, ny, nz);
}

hipError_t jacobi_gpu_multi_sweep(const ao_variant& v, const double* src, double* dst, int nx,
                                 int ny, int nz, hipStream_t s) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return hipSuccess;
    if (v.family != AO_FAM_JACOBI_ZREG_T3 && v.family != AO_FAM_JACOBI_ZREG_T4)
        return hipErrorInvalidConfiguration;
    return launch_columns(v, s, src, dst, nx, ny, nz);
}

hipError_t jacobi_gpu_planes(const ao_variant& v, int nx, int ny, int nz, int cus, int per_cu,
                             int* planes) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || !planes) return hipErrorInvalidValue;
    ColumnShape c;
    const hipError_t e = column_shape(v, nx, ny, nz, &c);
    if (e != hipSuccess) return e;
    *planes = column_planes(v, c, nz, cus, per_cu);
    return hipSuccess;
}

hipError_t hbm_copy(const double* src, double* dst, int64_t n, bool nt, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return hipErrorInvalidValue;
    const int64_t blocks = (n + 1023) / 1024;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n, nt ? 1 : 0);
    return hipGetLastError();
}

}  // namespace ao
