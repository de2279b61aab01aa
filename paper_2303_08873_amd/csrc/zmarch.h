// The register z-march with T sweeps fused per pass, for one wave: shared by
// the per-grid kernels and the batched kernel (device code only).
//
// Level l holds the values after l sweeps (level 0 = input).  The wave owns
// 64 lanes of x starting at i0 and the output rows j0 .. j0+R-1; level l
// lives on NL(l) = R + 2(T - l) rows from j0 - (T - l).  In iteration k the
// wave loads level 0 at plane k+1, then computes level l at plane k - l + 1
// for l = 1..T from level l-1 on planes k-l .. k-l+2: the plane below (kept
// only for the centre rows of level l), the centre plane and the plane just
// computed.  Level 1 takes its strip edges from lanes 0 and 63's extra loads;
// level l is exact on lanes l-1 .. 64-l.  Every level below T is forced to
// +0.0 outside the grid -- the ghost value a separate sweep would read -- so
// the result is bit-identical to T separate sweeps.  Planes computed before
// a level's inputs are loaded only feed planes that are never stored.  The
// sum order is the region's ((((xm+xp)+ym)+yp)+zm)+zp, then one multiply by
// fl(1/6).
#pragma once

#include <hip/hip_runtime.h>

#include "lanes.h"

namespace ao {
namespace zm {

constexpr double kSixth = 0x1.5555555555555p-3;  // fl(1/6)

template <bool NT>
__device__ __forceinline__ void put(double* p, double v) {
    if constexpr (NT) {
        __builtin_nontemporal_store(v, p);
    } else {
        *p = v;
    }
}

template <int T, int R>
struct TbShape;
// LDS bytes one wave needs for the staged level 0 (two plane buffers of
// 16-byte pieces, 34 pieces per staged row, one 1 KiB copy per 64 pieces),
// and a block of 4 waves
template <int T, int R>
constexpr int stage_wave_bytes() { return 2 * (((R + 2 * T) * 34 + 63) / 64) * 1024; }
template <int T, int R>
constexpr int stage_lds_bytes() { return 4 * stage_wave_bytes<T, R>(); }

template <int T, int R>
struct TbShape {
    static constexpr int nl(int l) { return R + 2 * (T - l); }
    // offset of level l in the packed centre / fresh arrays: sum of nl(0..l-1)
    static constexpr int off(int l) { return l * (R + 2 * T) - l * (l - 1); }
    // offset of level l in the packed below array (rows of level l+1): sum
    // of nl(1..l)
    static constexpr int offm(int l) { return l * (R + 2 * T) - l * (l + 1); }
    static constexpr int kAll = off(T);
    static constexpr int kBelow = offm(T);
};

// One level: level L at plane p from level L-1, then the next level up to
// STOP.  The arrays are the caller's register arrays; every index is a
// compile-time constant once inlined, so they stay in registers.  INNER:
// every row and column the wave touches lies inside the grid, so only whole
// planes can lie outside (a wave-uniform test instead of per-lane selects).
// hold (non-null): level T is written there instead of stored (the caller
// stores it later).
template <int T, int R, int L, bool NT, int STOP = T, bool INNER = false>
__device__ __forceinline__ void tb_level(const double* below, const double* centre,
                                         double* fresh, const double* ex, double* dst,
                                         int k, int j0, int nx, int ny, int nz, int k0, int k1,
                                         size_t plane, int lane, int i, bool xin, bool lane_out,
                                         double* hold = nullptr) {
    using S = TbShape<T, R>;
    const int p = k - L + 1;
    if (L == T && !(p >= k0 && p < k1)) return;  // wave-uniform
    const int jl = j0 - (T - L);
    const bool pin = p >= 0 && p < nz;
#pragma unroll
    for (int q = 0; q < S::nl(L); ++q) {
        const int j = jl + q;
        const double c = centre[S::off(L - 1) + q + 1];
        // level 1 takes lane 0's and lane 63's outer neighbours from ex
        const double xm = L == 1 ? from_left_or(c, ex[q]) : from_left(c);
        const double xp = L == 1 ? from_right_or(c, ex[q]) : from_right(c);
        double v = xm + xp;
        v = v + centre[S::off(L - 1) + q];
        v = v + centre[S::off(L - 1) + q + 2];
        v = v + below[S::offm(L - 1) + q];
        v = v + fresh[S::off(L - 1) + q + 1];
        if constexpr (L < T) {
            if constexpr (INNER)
                fresh[S::off(L) + q] = v * kSixth;
            else
                fresh[S::off(L) + q] = (pin && xin && j >= 0 && j < ny) ? v * kSixth : 0.0;
        } else if (hold) {
            hold[q] = v * kSixth;
        } else {
            if (lane_out && (INNER || j < ny))
                put<NT>(dst + (size_t)p * plane + (size_t)j * nx + i, v * kSixth);
        }
    }
    if constexpr (INNER && L < T) {
        if (!pin) {  // wave-uniform: the plane lies outside the grid
#pragma unroll
            for (int q = 0; q < S::nl(L); ++q) fresh[S::off(L) + q] = 0.0;
        }
    }
    if constexpr (L < STOP)
        tb_level<T, R, L + 1, NT, STOP, INNER>(below, centre, fresh, ex, dst, k, j0, nx, ny, nz, k0,
                                               k1, plane, lane, i, xin, lane_out, hold);
}

// Level 1 at plane k with every lane's x-neighbours supplied by nbr(q, xm,
// xp) for its row q (the staged march reads them from the plane's staged
// rows in LDS: no cross-lane moves).  Neighbours outside the grid must come
// as 0 wherever the centre point lies inside; where the centre point or its
// plane lies outside, the value is zeroed here as in tb_level, so what nbr
// returns there does not matter.  T >= 2 (level 1 is not the stored one).
template <int T, int R, bool INNER, typename Nbr>
__device__ __forceinline__ void tb_level1_nbr(const double* below, const double* centre,
                                              double* fresh, Nbr nbr, int k, int j0, int ny,
                                              int nz, bool xin) {
    static_assert(T >= 2, "level 1 is an intermediate level");
    using S = TbShape<T, R>;
    const bool pin = k >= 0 && k < nz;
    const int jl = j0 - (T - 1);
#pragma unroll
    for (int q = 0; q < S::nl(1); ++q) {
        const int j = jl + q;
        double xm, xp;
        nbr(q, xm, xp);
        double v = xm + xp;
        v = v + centre[S::off(0) + q];
        v = v + centre[S::off(0) + q + 2];
        v = v + below[S::offm(0) + q];
        v = v + fresh[S::off(0) + q + 1];
        if constexpr (INNER)
            fresh[S::off(1) + q] = v * kSixth;
        else
            fresh[S::off(1) + q] = (pin && xin && j >= 0 && j < ny) ? v * kSixth : 0.0;
    }
    if constexpr (INNER) {
        if (!pin) {  // wave-uniform: the plane lies outside the grid
#pragma unroll
            for (int q = 0; q < S::nl(1); ++q) fresh[S::off(1) + q] = 0.0;
        }
    }
}

// Shift every level by one plane: below <- centre (centre rows of the next
// level), centre <- fresh.
template <int T, int R, int L, int STOP = T - 1>
__device__ __forceinline__ void tb_rotate(double* below, double* centre, const double* fresh) {
    using S = TbShape<T, R>;
#pragma unroll
    for (int q = 0; q < S::nl(L + 1); ++q) below[S::offm(L) + q] = centre[S::off(L) + q + 1];
#pragma unroll
    for (int q = 0; q < S::nl(L); ++q) centre[S::off(L) + q] = fresh[S::off(L) + q];
    if constexpr (L < STOP) tb_rotate<T, R, L + 1, STOP>(below, centre, fresh);
}

// T sweeps of src on the wave's column: lanes hold x = i0 + lane, output
// rows j0 .. j0+R-1 (j0 < ny), output planes [k0, k1); level T is stored on
// lanes lane_lo .. lane_hi that lie inside the grid (the caller keeps that
// window within T-1 .. 64-T).  Every load stays inside the grid (masked,
// or at clamped coordinates); the whole wave must call this (cross-lane
// moves).  EARLY: the next plane's level-0 rows
// and strip edges are loaded as soon as level 1 has consumed this plane's
// (into the same registers), so they are in flight while levels 2..T
// compute instead of at the top of the next iteration; level T is then
// stored one iteration late, just before those loads are issued, so the
// loads are always the youngest memory operations and waiting for them
// never waits for stores issued after them.  SROW: the row
// indices are wave-uniform (the caller's j0 comes from wave_index()), so
// loads go to clamped rows through scalar row bases; otherwise rows are
// per-lane values and out-of-grid loads are masked (fewer scalar registers,
// for kernels that inline several marches).  STAGE (without EARLY): level 0
// arrives through asynchronous global->LDS copies one plane ahead (see the
// staged loop below); the caller keeps the plane below 2^32 bytes, nx >= 2,
// and -- when nx is odd -- the staged columns (68 from an even x at most 3
// left of i0) inside the grid on the right; with INNER also on the left;
// wave w stages in bytes [w * wave_bytes, w * wave_bytes +
// stage_wave_bytes<T, R>()) of stage_lds.
template <int T, int R, bool NT, bool EARLY = false, bool SROW = true, bool INNER = false,
          bool STAGE = false>
__device__ __forceinline__ void tb_column(const double* __restrict__ src, double* __restrict__ dst,
                                          int nx, int ny, int nz, int i0, int j0, int k0, int k1,
                                          int lane_lo, int lane_hi, char* stage_lds = nullptr,
                                          int wave_bytes = stage_wave_bytes<T, R>()) {
    using S = TbShape<T, R>;
    const int lane = (int)(threadIdx.x & 63);
    const int i = i0 + lane;
    const size_t plane = (size_t)nx * (size_t)ny;
    const bool xin = i >= 0 && i < nx;
    const int ie = (lane == 0) ? i0 - 1 : i0 + 64;
    const bool eok = (lane == 0 || lane == 63) && ie >= 0 && ie < nx;
    const bool lane_out = lane >= lane_lo && lane <= lane_hi && xin;
    // Row loads: the row's base address is wave-uniform (j and k are), each
    // lane reads at its x clamped into the row, and rows and planes outside
    // the grid are clamped too; the value is zeroed afterwards where the
    // point lies outside.  No load is masked or branched around (so loads
    // stay batched ahead of their first use) and one 32-bit byte offset
    // serves every row (the caller keeps nx * 8 below 2^32).
    const unsigned bo = (unsigned)min(max(i, 0), nx - 1) * 8u;
    const unsigned boe = (unsigned)min(max(ie, 0), nx - 1) * 8u;
    auto ld = [&](int k, int j, bool edge) -> double {
        const bool ok = edge ? eok : xin;
        const bool in = k >= 0 && k < nz && j >= 0 && j < ny;
        if constexpr (INNER) {  // rows and columns inside: no clamp, no select
            const int kc = min(max(k, 0), nz - 1);
            const char* row = (const char*)(src + ((size_t)kc * plane + (size_t)j * nx));
            return *(const double*)(row + (edge ? boe : bo));
        } else if constexpr (SROW) {
            const int kc = min(max(k, 0), nz - 1), jc = min(max(j, 0), ny - 1);
            const char* row = (const char*)(src + ((size_t)kc * plane + (size_t)jc * nx));
            const double v = *(const double*)(row + (edge ? boe : bo));
            return (ok && in) ? v : 0.0;
        } else {
            return (ok && in) ? src[(size_t)k * plane + (size_t)j * nx + (edge ? ie : i)] : 0.0;
        }
    };
    // INNER loads read a clamped plane; a plane outside the grid is zeroed
    // after its loads are issued (wave-uniform)
    auto zero_out = [&](int k, double* a, int n) {
        if constexpr (INNER || STAGE) {
            if (k < 0 || k >= nz) {
                for (int q = 0; q < n; ++q) a[q] = 0.0;
            }
        }
    };
    double below[S::kBelow], centre[S::kAll], fresh[S::kAll];
    const int ka = k0 - T + 1;  // first iteration: level 1 at plane ka
#pragma unroll
    for (int q = 0; q < S::nl(1); ++q) below[q] = ld(ka - 1, j0 - (T - 1) + q, false);
#pragma unroll
    for (int q = 0; q < S::nl(0); ++q) centre[q] = ld(ka, j0 - T + q, false);
    zero_out(ka - 1, below, S::nl(1));
    zero_out(ka, centre, S::nl(0));
#pragma unroll
    for (int q = S::nl(1); q < S::kBelow; ++q) below[q] = 0.0;
#pragma unroll
    for (int q = S::nl(0); q < S::kAll; ++q) centre[q] = 0.0;
    if constexpr (EARLY && T >= 2) {
        const int kend = k1 + T - 2;
        double ex[S::nl(1)];
#pragma unroll
        for (int q = 0; q < S::nl(0); ++q) fresh[q] = ld(ka + 1, j0 - T + q, false);
#pragma unroll
        for (int q = 0; q < S::nl(1); ++q) ex[q] = ld(ka, j0 - (T - 1) + q, true);
        zero_out(ka + 1, fresh, S::nl(0));
        zero_out(ka, ex, S::nl(1));
        double hold[R];
        int hold_p = -1;  // plane of hold (wave-uniform); stored when in [k0, k1)
        auto store_hold = [&]() {
            if (hold_p >= k0 && hold_p < k1) {
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int j = j0 + q;
                    if (lane_out && (INNER || j < ny))
                        put<NT>(dst + (size_t)hold_p * plane + (size_t)j * nx + i, hold[q]);
                }
            }
        };
        for (int k = ka; k <= kend; ++k) {
            tb_level<T, R, 1, NT, 1, INNER>(below, centre, fresh, ex, dst, k, j0, nx, ny, nz, k0, k1,
                                            plane, lane, i, xin, lane_out);
            // level 0 moves on one plane; level 1's new plane stays in fresh
            tb_rotate<T, R, 0, 0>(below, centre, fresh);
            store_hold();
            if (k < kend) {  // wave-uniform: the next iteration's plane and edges
#pragma unroll
                for (int q = 0; q < S::nl(0); ++q) fresh[q] = ld(k + 2, j0 - T + q, false);
#pragma unroll
                for (int q = 0; q < S::nl(1); ++q) ex[q] = ld(k + 1, j0 - (T - 1) + q, true);
                zero_out(k + 2, fresh, S::nl(0));
                zero_out(k + 1, ex, S::nl(1));
            }
            tb_level<T, R, 2, NT, T, INNER>(below, centre, fresh, ex, dst, k, j0, nx, ny, nz, k0, k1,
                                            plane, lane, i, xin, lane_out, hold);
            hold_p = k - T + 1;
            tb_rotate<T, R, 1>(below, centre, fresh);
        }
        store_hold();
        return;
    }
    if constexpr (STAGE && !EARLY) {
        // Staged level 0: every plane's level-0 rows (68 columns from the
        // even x0 = i0-2 or i0-3, so the strip edges too) are copied
        // global->LDS by 16-byte pieces into one of two per-wave buffers, one
        // plane ahead, so the copies hold no registers and are in flight
        // while a whole plane computes.  Pieces and rows outside the grid
        // (boundary waves) are copied from clamped coordinates -- with x0
        // even a piece never straddles x = 0, nor x = nx-1 when nx is even
        // -- and the values read back are zeroed where the point lies
        // outside; planes outside the grid are zeroed whole.  With four
        // fused sweeps level 1 takes every lane's x-neighbours straight from
        // plane k's staged rows (one two-address LDS read per row, no
        // cross-lane moves; 72 fewer VALU instructions per plane), so plane
        // k's buffer is refilled with plane k+2 only after level 1; with
        // fewer sweeps level 1 uses the cross-lane moves and the strip
        // edges read up front (the LDS form costs those marches a wave per
        // SIMD) and the buffer is refilled before level 1.  The copies are
        // inline assembly with their waits written out: at the top of each
        // iteration vmcnt(0) covers the copy of plane k+1 issued in the
        // previous iteration and the stores issued before it (level T is
        // stored one iteration late, ahead of the copy, so the copy is
        // always the youngest memory operation); lgkmcnt(0) before a buffer
        // is refilled drains the reads of its previous plane; a last
        // vmcnt(0) leaves no copy writing LDS when the wave ends.
        constexpr int kRowB = 68 * 8;                // one staged row
        constexpr int kPieces = S::nl(0) * 34;       // 16-byte pieces per plane
        constexpr int kCopies = (kPieces + 63) / 64;  // copy instructions per plane
        constexpr int kBuf = kCopies * 1024;         // bytes per plane buffer
        // stage_lds: the caller's LDS block, one slot of wave_bytes (at least
        // 2 buffers x kBuf bytes) per wave.  A caller whose waves run items of
        // different (T, R) without a barrier between them passes one fixed
        // stride for all, so a wave's slot never moves into a neighbour's.
        static_assert(2 * kBuf == stage_wave_bytes<T, R>(), "staging slot size");
        const int wv = wave_index();
        char* mine = stage_lds + wv * wave_bytes;
        const unsigned lds0 =
            (unsigned)(uintptr_t)((__attribute__((address_space(3))) char*)mine);
        const int x0 = i0 - 2 - (i0 & 1);  // even
        unsigned poff[kCopies];  // lane's byte offset within a plane, per copy
#pragma unroll
        for (int p = 0; p < kCopies; ++p) {
            const int g = p * 64 + lane;
            const int r = min(g / 34, S::nl(0) - 1), c = min(g - r * 34, 33);
            const int jr = min(max(j0 - T + r, 0), ny - 1);
            const int xr = min(max(x0 + 2 * c, 0), nx - 2);
            poff[p] = (unsigned)(((size_t)jr * nx + (size_t)xr) * 8u);
        }
        auto stage = [&](int kp) {  // plane kp (clamped into the grid) -> buffer kp & 1
            const char* pb = (const char*)(src + (size_t)min(max(kp, 0), nz - 1) * plane);
            const unsigned m0 = lds0 + (unsigned)((kp & 1) * kBuf);
#pragma unroll
            for (int p = 0; p < kCopies; ++p)
                // (one wait state between the M0 write and the copy that reads it)
                asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off"
                             :
                             : "s"(m0 + (unsigned)(p * 1024)), "v"((const void*)(pb + poff[p]))
                             : "memory", "m0");
        };
        // lane's x offset in a staged row (its neighbours at -8 and +8
        // bytes: columns 1 .. 67 of the 68), and (fewer than four sweeps)
        // the strip edges x = i0-1 on lane 0 and x = i0+64 on lane 63
        static_assert(T >= 2, "the staged march fuses at least two sweeps");
        constexpr bool kNbrLds = T >= 4;
        const int sh = i0 - x0;  // 2 or 3
        const int xo = (lane + sh) * 8;
        const int eo = lane == 0 ? (sh - 1) * 8 : lane == 63 ? (64 + sh) * 8 : xo;
        const bool xm_ok = i - 1 >= 0 && i - 1 < nx, xp_ok = i + 1 >= 0 && i + 1 < nx;
        auto rd = [&](int kp, int q, int off) -> double {
            return *(const double*)(mine + (kp & 1) * kBuf + q * kRowB + off);
        };
        const int kend = k1 + T - 2;
        double hold[R];
        int hold_p = -1;
        auto store_hold = [&]() {
            if (hold_p >= k0 && hold_p < k1) {
#pragma unroll
                for (int q = 0; q < R; ++q)
                    if (lane_out && (INNER || j0 + q < ny))
                        put<NT>(dst + (size_t)hold_p * plane + (size_t)(j0 + q) * nx + i, hold[q]);
            }
        };
        stage(ka);
        stage(ka + 1);
        for (int k = ka; k <= kend; ++k) {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
            for (int q = 0; q < S::nl(0); ++q) {
                const double v = rd(k + 1, q, xo);
                if constexpr (INNER) {
                    fresh[q] = v;
                } else {
                    const int j = j0 - T + q;
                    fresh[q] = (xin && j >= 0 && j < ny) ? v : 0.0;
                }
            }
            zero_out(k + 1, fresh, S::nl(0));
            if constexpr (kNbrLds) {
                store_hold();
                // level 1's row q is level 0's row q + 1 of plane k
                auto nbr = [&](int q, double& xm, double& xp) {
                    xm = rd(k, q + 1, xo - 8);
                    xp = rd(k, q + 1, xo + 8);
                    if constexpr (!INNER) {
                        xm = xm_ok ? xm : 0.0;
                        xp = xp_ok ? xp : 0.0;
                    }
                };
                tb_level1_nbr<T, R, INNER>(below, centre, fresh, nbr, k, j0, ny, nz, xin);
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // plane k's reads are done
                if (k < kend) stage(k + 2);  // wave-uniform; refills plane k's buffer
                tb_level<T, R, 2, NT, T, INNER>(below, centre, fresh, nullptr, dst, k, j0, nx, ny,
                                                nz, k0, k1, plane, lane, i, xin, lane_out, hold);
            } else {
                double ex[S::nl(1)];
#pragma unroll
                for (int q = 0; q < S::nl(1); ++q) {
                    const double v = rd(k, q + 1, eo);
                    if constexpr (INNER) {
                        ex[q] = v;
                    } else {
                        const int j = j0 - (T - 1) + q;
                        ex[q] = (eok && j >= 0 && j < ny) ? v : 0.0;
                    }
                }
                zero_out(k, ex, S::nl(1));
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // plane k's reads are done
                store_hold();
                if (k < kend) stage(k + 2);  // wave-uniform; refills plane k's buffer
                tb_level<T, R, 1, NT, T, INNER>(below, centre, fresh, ex, dst, k, j0, nx, ny, nz,
                                                k0, k1, plane, lane, i, xin, lane_out, hold);
            }
            hold_p = k - T + 1;
            tb_rotate<T, R, 0>(below, centre, fresh);
        }
        store_hold();
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        return;
    }
    for (int k = ka; k <= k1 + T - 2; ++k) {
        double ex[S::nl(1)];
#pragma unroll
        for (int q = 0; q < S::nl(0); ++q) fresh[q] = ld(k + 1, j0 - T + q, false);
#pragma unroll
        for (int q = 0; q < S::nl(1); ++q) ex[q] = ld(k, j0 - (T - 1) + q, true);
        zero_out(k + 1, fresh, S::nl(0));
        zero_out(k, ex, S::nl(1));
        tb_level<T, R, 1, NT, T, INNER>(below, centre, fresh, ex, dst, k, j0, nx, ny, nz, k0, k1,
                                        plane, lane, i, xin, lane_out);
        tb_rotate<T, R, 0>(below, centre, fresh);
    }
}

}  // namespace zm
}  // namespace ao
