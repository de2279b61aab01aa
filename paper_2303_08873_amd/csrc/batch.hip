// Batched execution of many uneven Jacobi instances in one launch per sweep.
//
// Every (instance, tile) pair is a work item; a persistent kernel -- grid
// sized to the machine, each workgroup striding over the item list --
// performs one sweep of every instance, and the S sweeps are captured once
// in a HIP graph so a single graph launch runs the whole batch.  Instances
// are bucketed by their largest dimension and each bucket uses one tile
// shape, picked by the autotuner (batch_autotune) from a fixed candidate
// table by timing the bucket alone.  The per-point arithmetic is the
// region's ((((xm+xp)+ym)+yp)+zm)+zp) * fl(1/6), so each instance's result
// is bit-identical to a standalone run.
//
// Tile kinds:
//  direct  tx*ty*tz points, threads stride over them, six neighbour loads
//          each (small grids, where a 64-wide strip would idle lanes);
//  zreg    the register z-march: each of the 4 waves owns a 64-wide strip of
//          R rows and marches tz planes, x-neighbours by cross-lane moves;
//  fused   the register z-march with two sweeps fused per pass (zmarch.h):
//          64 lanes, 62 stored columns, R rows per wave.  An instance on a
//          fused tile runs ceil(S/2) passes, the first one a single sweep
//          on the same tile when S is odd.  Fused tiles run in a kernel of
//          their own (it needs more registers than the others).
#include <math.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "internal.h"
#include "lanes.h"
#include "zmarch.h"

namespace ao {
namespace {

constexpr double kC = 0x1.5555555555555p-3;  // fl(1/6)
constexpr int kThreads = 256;
constexpr int kBuckets = 5;

enum {
    kDirect = 0, kZreg1 = 1, kZreg2 = 2, kZreg4 = 4,      // one sweep per pass
    kFused1 = 11, kFused2 = 12, kFused4 = 14,              // two sweeps per pass
    kTri1 = 21, kTri2 = 22, kTri4 = 24                     // three sweeps per pass
};
__host__ __device__ constexpr bool is_fused(int kind) { return kind > 10 && kind < 20; }
__host__ __device__ constexpr bool is_tri(int kind) { return kind > 20; }
struct TileCfg {
    int kind, tx, ty, tz;
};
// candidate tiles (index = candidate id)
constexpr TileCfg kCands[] = {
    {kDirect, 8, 8, 4},  {kDirect, 16, 16, 1}, {kDirect, 16, 8, 2},  {kDirect, 32, 8, 1},
    {kDirect, 64, 4, 1}, {kDirect, 16, 16, 4}, {kDirect, 8, 8, 16},  {kZreg1, 64, 4, 16},
    {kZreg2, 64, 8, 32}, {kZreg2, 64, 8, 64},  {kZreg1, 64, 4, 64},  {kZreg2, 64, 8, 16},
    {kZreg4, 64, 16, 24}, {kZreg4, 64, 16, 32}, {kZreg4, 64, 16, 64}, {kZreg2, 64, 8, 24},
    {kFused1, 62, 4, 16}, {kFused2, 62, 8, 16},  {kFused2, 62, 8, 32},  {kFused4, 62, 16, 16},
    {kFused4, 62, 16, 32}, {kFused1, 62, 4, 32},
    {kTri1, 60, 4, 16},    {kTri2, 60, 8, 16},   {kTri4, 60, 16, 16},   {kTri4, 60, 16, 32},
    {kTri2, 60, 8, 32},    {kTri4, 60, 16, 24},  {kTri4, 60, 16, 12},   {kTri2, 60, 8, 24},
    {kTri2, 60, 8, 8},
};
constexpr int kNumCands = (int)(sizeof(kCands) / sizeof(kCands[0]));
// default candidate per bucket before autotuning
constexpr int kDefaultCand[kBuckets] = {0, 3, 6, 19, 19};
static_assert(kCands[19].kind == kFused4 && kCands[19].tz == 16, "default tile of the large buckets");
__constant__ TileCfg c_cands[kNumCands];

struct Item {
    int32_t inst, x0, y0, z0, cand;
};
struct Inst {
    const double* u0;
    double* out;
    double* tmp;
    int32_t nx, ny, nz, sweeps;
};

// launches an instance takes on a tile kind: one per sweep, one per pair of
// sweeps on two-sweep tiles, one per three sweeps on three-sweep tiles (the
// first pass then takes the S mod 3 remaining sweeps)
__host__ __device__ inline int passes_of(int sweeps, int kind) {
    return is_tri(kind) ? (sweeps + 2) / 3 : is_fused(kind) ? (sweeps + 1) / 2 : sweeps;
}

__device__ __forceinline__ const double* src_of(const Inst& in, int s) {
    return s == 0 ? in.u0 : (((in.sweeps - s) % 2 == 0) ? in.out : in.tmp);
}
__device__ __forceinline__ double* dst_of(const Inst& in, int s) {
    return ((in.sweeps - 1 - s) % 2 == 0) ? in.out : in.tmp;
}

__device__ void tile_direct(const Inst& in, const double* __restrict__ src, double* __restrict__ dst,
                            const Item& it, const TileCfg& c) {
    const int nx = in.nx, ny = in.ny, nz = in.nz;
    const size_t plane = (size_t)nx * ny;
    const int npts = c.tx * c.ty * c.tz;
    for (int p = (int)threadIdx.x; p < npts; p += kThreads) {
        const int i = it.x0 + p % c.tx;
        const int j = it.y0 + (p / c.tx) % c.ty;
        const int k = it.z0 + p / (c.tx * c.ty);
        if (i >= nx || j >= ny || k >= nz) continue;
        const size_t idx = (size_t)k * plane + (size_t)j * nx + i;
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
        dst[idx] = v * kC;
    }
}

template <int R>
__device__ void tile_zreg(const Inst& in, const double* __restrict__ src, double* __restrict__ dst,
                          const Item& it, const TileCfg& c) {
    const int nx = in.nx, ny = in.ny, nz = in.nz;
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const int i0 = it.x0, i = i0 + lane;
    const int j0 = it.y0 + wave * R;
    if (j0 >= ny) return;  // wave-uniform
    const int k0 = it.z0, k1 = min(nz, k0 + c.tz);
    const size_t plane = (size_t)nx * ny;
    const bool xin = i < nx;
    const int ie = (lane == 0) ? i0 - 1 : i0 + 64;
    const bool edge = (lane == 0 && i0 > 0) || (lane == 63 && i0 + 64 < nx);
    auto at = [&](int k, int j, int x, bool ok) -> double {
        return ok ? src[(size_t)k * plane + (size_t)j * nx + x] : 0.0;
    };
    double below[R], cur[R], above[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool okj = j0 + r < ny;
        below[r] = at(k0 - 1, j0 + r, i, okj && xin && k0 > 0);
        cur[r] = at(k0, j0 + r, i, okj && xin);
    }
    for (int k = k0; k < k1; ++k) {
        const double ymv = at(k, j0 - 1, i, j0 > 0 && xin);
        const double ypv = at(k, j0 + R, i, j0 + R < ny && xin);
        double ex[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool okj = j0 + r < ny;
            ex[r] = at(k, j0 + r, ie, edge && okj);
            above[r] = at(k + 1, j0 + r, i, okj && xin && k + 1 < nz);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double left = from_left(cur[r]);
            const double right = from_right(cur[r]);
            const double xm = (lane == 0) ? ex[r] : left;
            const double xp = (lane == 63) ? ex[r] : right;
            const double ym = (r == 0) ? ymv : cur[r - 1];
            const double yp = (r == R - 1) ? ypv : cur[r + 1];
            double v = xm + xp;
            v = v + ym;
            v = v + yp;
            v = v + below[r];
            v = v + above[r];
            if (xin && j0 + r < ny) dst[(size_t)k * plane + (size_t)(j0 + r) * nx + i] = v * kC;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            below[r] = cur[r];
            cur[r] = above[r];
        }
    }
}

// Items are dealt in windows of gridDim.x; inside a window the workgroup ->
// item map is XCD-aware (workgroups go to the 8 XCDs round-robin), so each
// XCD takes a contiguous run of neighbouring tiles and their halos meet in
// its L2.
__device__ __forceinline__ int xcd_slot(int b, int g) {
    const int xcd = b % 8, local = b / 8, per = g / 8, rem = g % 8;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

__global__ __launch_bounds__(kThreads) void k_batch_sweep(const Inst* __restrict__ insts,
                                                          const Item* __restrict__ items,
                                                          int nitems, int sweep) {
    const int g = (int)gridDim.x;
    const int slot = xcd_slot((int)blockIdx.x, g);
    for (int w = slot; w < nitems; w += g) {
        const Item it = items[w];
        const Inst in = insts[it.inst];
        if (sweep >= in.sweeps) continue;
        const TileCfg c = c_cands[it.cand];
        const double* src = src_of(in, sweep);
        double* dst = dst_of(in, sweep);
        if (c.kind == kDirect)
            tile_direct(in, src, dst, it, c);
        else if (c.kind == kZreg1)
            tile_zreg<1>(in, src, dst, it, c);
        else if (c.kind == kZreg2)
            tile_zreg<2>(in, src, dst, it, c);
        else
            tile_zreg<4>(in, src, dst, it, c);
    }
}

// One pass of a two-sweep tile column: one sweep (single) or two on lanes
// 1 .. 62 of the strip starting at i0; two-sweep passes of waves whose
// columns and rows (with the 2-row halo) lie inside the grid take the march
// without per-lane selects.
template <int R>
__device__ __forceinline__ void pair_column(bool single, const double* src, double* dst,
                                            const Inst& in, int i0, int j0, int z0, int k1) {
    if (single) {
        zm::tb_column<1, R, false, false, false>(src, dst, in.nx, in.ny, in.nz, i0, j0, z0, k1, 1, 62);
    } else {
        const bool inner = i0 >= 1 && i0 + 64 < in.nx && j0 >= 2 && j0 + R + 2 <= in.ny;
        if (inner)
            zm::tb_column<2, R, false, false, false, true>(src, dst, in.nx, in.ny, in.nz, i0, j0, z0,
                                                           k1, 1, 62);
        else
            zm::tb_column<2, R, false, false, false>(src, dst, in.nx, in.ny, in.nz, i0, j0, z0, k1,
                                                     1, 62);
    }
}

// Pass `pass` of every instance on a fused tile: ping-pong over ceil(S/2)
// passes so the last one lands in `out`; pass 0 is a single sweep when S is
// odd.  Strip x0 (a multiple of 62) is computed on lanes x0-1 .. x0+62.
__global__ __launch_bounds__(kThreads) void k_batch_fused(const Inst* __restrict__ insts,
                                                          const Item* __restrict__ items,
                                                          int nitems, int pass) {
    const int g = (int)gridDim.x;
    const int slot = xcd_slot((int)blockIdx.x, g);
    const int wave = (int)(threadIdx.x >> 6);
    for (int w = slot; w < nitems; w += g) {
        const Item it = items[w];
        const Inst in = insts[it.inst];
        const int P = passes_of(in.sweeps, kFused1);
        if (pass >= P) continue;  // (the two-sweep kernel only sees two-sweep tiles)
        const TileCfg c = c_cands[it.cand];
        const double* src = pass == 0 ? in.u0 : (((P - pass) % 2 == 0) ? in.out : in.tmp);
        double* dst = ((P - 1 - pass) % 2 == 0) ? in.out : in.tmp;
        const bool single = (in.sweeps & 1) && pass == 0;
        const int R = c.kind - 10;
        const int j0 = it.y0 + wave * R;
        if (j0 >= in.ny) continue;  // wave-uniform
        const int k1 = min(in.nz, it.z0 + c.tz);
        const int i0 = it.x0 - 1;
        if (R == 1)
            pair_column<1>(single, src, dst, in, i0, j0, it.z0, k1);
        else if (R == 2)
            pair_column<2>(single, src, dst, in, i0, j0, it.z0, k1);
        else
            pair_column<4>(single, src, dst, in, i0, j0, it.z0, k1);
    }
}

// One pass of a three-sweep tile column: T = 1, 2 or 3 sweeps on lanes
// 2 .. 61 of the strip starting at i0; two- and three-sweep passes of waves
// whose columns and rows (with the T-row halo) lie inside the grid take the
// march without per-lane selects.  Two- and three-sweep passes receive
// level 0 through the staged global->LDS copies (stg: the block's staging area)
// where the staged columns allow it: a plane below 2^32 bytes and, for odd
// nx, the 68 staged columns (from the even x0 = i0-2 or i0-3) inside the
// grid on the right -- and on both sides for the path without selects.
// Waves of one block run items of different (T, R) with no barrier between
// them (a wave skips an item at once when its rows lie outside the grid), so
// every staged march of the three-sweep kernel takes one fixed per-wave slot,
// that of the widest tile: wave w owns bytes [w * kStageWave, (w+1) *
// kStageWave) of the block's staging area whatever item it is on.
constexpr int kStageWave = zm::stage_wave_bytes<3, 4>();
template <int T, int R>
constexpr bool slot_fits() {
    return zm::stage_wave_bytes<T, R>() <= kStageWave && 4 * kStageWave == zm::stage_lds_bytes<3, 4>();
}
static_assert(slot_fits<2, 1>() && slot_fits<2, 2>() && slot_fits<2, 4>() && slot_fits<3, 1>() &&
                  slot_fits<3, 2>() && slot_fits<3, 4>(),
              "every staged (T, R) of the three-sweep tiles fits the fixed per-wave slot");

template <int R>
__device__ __forceinline__ void tri_column(int T, const double* src, double* dst, const Inst& in,
                                           int i0, int j0, int z0, int k1, char* stg) {
    if (T == 1) {
        zm::tb_column<1, R, false, false, false>(src, dst, in.nx, in.ny, in.nz, i0, j0, z0, k1, 2, 61);
    } else if (T == 2) {
        const bool inner = i0 >= 1 && i0 + 64 < in.nx && j0 >= 2 && j0 + R + 2 <= in.ny;
        const int x0 = i0 - 2 - (i0 & 1);
        const bool fits = in.nx >= 2 && (size_t)in.nx * (size_t)in.ny * 8u < ((size_t)1 << 32) &&
                          (!(in.nx & 1) || x0 + 68 <= in.nx);
        if (fits && inner && x0 >= 0 && x0 + 68 <= in.nx)
            zm::tb_column<2, R, false, false, false, true, true>(src, dst, in.nx, in.ny, in.nz, i0,
                                                                 j0, z0, k1, 2, 61, stg, kStageWave);
        else if (fits)
            zm::tb_column<2, R, false, false, false, false, true>(src, dst, in.nx, in.ny, in.nz, i0,
                                                                  j0, z0, k1, 2, 61, stg, kStageWave);
        else if (inner)
            zm::tb_column<2, R, false, false, false, true>(src, dst, in.nx, in.ny, in.nz, i0, j0, z0,
                                                           k1, 2, 61);
        else
            zm::tb_column<2, R, false, false, false>(src, dst, in.nx, in.ny, in.nz, i0, j0, z0, k1,
                                                     2, 61);
    } else {
        const bool inner = i0 >= 1 && i0 + 64 < in.nx && j0 >= 3 && j0 + R + 3 <= in.ny;
        const int x0 = i0 - 2 - (i0 & 1);
        const bool fits = in.nx >= 2 && (size_t)in.nx * (size_t)in.ny * 8u < ((size_t)1 << 32) &&
                          (!(in.nx & 1) || x0 + 68 <= in.nx);
        if (fits && inner && x0 >= 0 && x0 + 68 <= in.nx)
            zm::tb_column<3, R, false, false, false, true, true>(src, dst, in.nx, in.ny, in.nz, i0,
                                                                 j0, z0, k1, 2, 61, stg, kStageWave);
        else if (fits)
            zm::tb_column<3, R, false, false, false, false, true>(src, dst, in.nx, in.ny, in.nz, i0,
                                                                  j0, z0, k1, 2, 61, stg, kStageWave);
        else if (inner)
            zm::tb_column<3, R, false, false, false, true>(src, dst, in.nx, in.ny, in.nz, i0, j0, z0,
                                                           k1, 2, 61);
        else
            zm::tb_column<3, R, false, false, false>(src, dst, in.nx, in.ny, in.nz, i0, j0, z0, k1,
                                                     2, 61);
    }
}

// Pass `pass` of every instance on a three-sweep tile: ping-pong over
// ceil(S/3) passes so the last one lands in `out`; pass 0 takes the S mod 3
// remaining sweeps when S is not a multiple of 3.  Strip x0 (a multiple of
// 60) is computed on lanes x0-2 .. x0+61 and stored on x0 .. x0+59.
__global__ __launch_bounds__(kThreads) void k_batch_fused3(const Inst* __restrict__ insts,
                                                           const Item* __restrict__ items,
                                                           int nitems, int pass) {
    const int g = (int)gridDim.x;
    const int slot = xcd_slot((int)blockIdx.x, g);
    const int wave = (int)(threadIdx.x >> 6);
    // staging area of the widest tile (4 rows per wave), one fixed slot per
    // wave; a wave's staged march ends with its copies landed and its reads
    // done, so its next item reuses the slot at once
    __shared__ __attribute__((aligned(16))) char stg[4 * kStageWave];
    for (int w = slot; w < nitems; w += g) {
        const Item it = items[w];
        const Inst in = insts[it.inst];
        const int P = passes_of(in.sweeps, kTri1);
        if (pass >= P) continue;
        const TileCfg c = c_cands[it.cand];
        const double* src = pass == 0 ? in.u0 : (((P - pass) % 2 == 0) ? in.out : in.tmp);
        double* dst = ((P - 1 - pass) % 2 == 0) ? in.out : in.tmp;
        const int rem = in.sweeps % 3;
        const int T = (pass == 0 && rem) ? rem : 3;
        const int R = c.kind - 20;
        const int j0 = it.y0 + wave * R;
        if (j0 >= in.ny) continue;  // wave-uniform
        const int k1 = min(in.nz, it.z0 + c.tz);
        const int i0 = it.x0 - 2;
        if (R == 1)
            tri_column<1>(T, src, dst, in, i0, j0, it.z0, k1, stg);
        else if (R == 2)
            tri_column<2>(T, src, dst, in, i0, j0, it.z0, k1, stg);
        else
            tri_column<4>(T, src, dst, in, i0, j0, it.z0, k1, stg);
    }
}

int bucket_of(int nx, int ny, int nz) {
    const int m = std::max(nx, std::max(ny, nz));
    if (m <= 16) return 0;
    if (m <= 32) return 1;
    if (m <= 64) return 2;
    if (m <= 128) return 3;
    return 4;
}

// Work of one item: the points of a one-point-per-thread tile inside the
// grid; for the register marches, the waves that hold rows inside the grid
// times the planes each marches (its chunk inside the grid plus the 2(T-1)
// halo planes of T fused sweeps) -- a wave runs its whole 64-lane strip
// whatever the columns inside the grid.
int64_t item_cost(const Inst& in, const TileCfg& c, int x, int y, int z) {
    const int64_t wx = std::min(c.tx, in.nx - x), wy = std::min(c.ty, in.ny - y),
                  wz = std::min(c.tz, in.nz - z);
    if (c.kind == kDirect) return wx * wy * wz;
    const int R = c.kind % 10, T = is_tri(c.kind) ? 3 : is_fused(c.kind) ? 2 : 1;
    return ((wy + R - 1) / R) * (wz + 2 * (T - 1));
}

}  // namespace
}  // namespace ao

using namespace ao;

struct ao_batch {
    std::vector<Inst> insts;
    std::vector<int> bucket;
    int cand[kBuckets];
    Inst* d_insts = nullptr;
    Item* d_items = nullptr;   // single-sweep tiles (direct, zreg)
    int nitems = 0;
    int launches = 0;          // passes of the single-sweep tiles
    Item* d_items_f = nullptr;  // two-sweep tiles
    int nitems_f = 0;
    int launches_f = 0;
    Item* d_items_3 = nullptr;  // three-sweep tiles
    int nitems_3 = 0;
    int launches_3 = 0;
    int items_per_bucket[kBuckets] = {0};
    double* scratch = nullptr;
    int grid = 0, grid_f = 0, grid_3 = 0;  // workgroups of each persistent kernel
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_dirty = true;
    ~ao_batch() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (cap_stream) hipStreamDestroy(cap_stream);
        if (d_items) hipFree(d_items);
        if (d_items_f) hipFree(d_items_f);
        if (d_items_3) hipFree(d_items_3);
        if (d_insts) hipFree(d_insts);
        if (scratch) hipFree(scratch);
    }
};

namespace ao {
namespace {

std::vector<Item> make_items(const ao_batch* b, int only_bucket, int cand_override) {
    std::vector<std::pair<int64_t, Item>> v;
    for (size_t q = 0; q < b->insts.size(); ++q) {
        const int bk = b->bucket[q];
        if (only_bucket >= 0 && bk != only_bucket) continue;
        const int cand = cand_override >= 0 ? cand_override : b->cand[bk];
        const TileCfg& c = kCands[cand];
        const Inst& in = b->insts[q];
        if ((int64_t)in.nx * in.ny * in.nz == 0 || in.sweeps == 0) continue;
        for (int z = 0; z < in.nz; z += c.tz)
            for (int y = 0; y < in.ny; y += c.ty)
                for (int x = 0; x < in.nx; x += c.tx)
                    v.push_back({item_cost(in, c, x, y, z), Item{(int32_t)q, x, y, z, cand}});
    }
    // larger items first (the strided loop then ends with the small ones);
    // upload_list deals them out in alternating directions
    std::stable_sort(v.begin(), v.end(), [](const auto& a, const auto& c) { return a.first > c.first; });
    std::vector<Item> out;
    out.reserve(v.size());
    for (auto& p : v) out.push_back(p.second);
    return out;
}

// Uploads a kernel's items (largest first) for a grid of g workgroups, each
// taking every g-th item: every other round of g items is reversed, so the
// workgroup that takes a round's largest item takes the next round's
// smallest and the workgroups' totals stay close.
hipError_t upload_list(Item** d, int* count, std::vector<Item> items, int g) {
    if (*d) hipFree(*d);
    *d = nullptr;
    *count = (int)items.size();
    if (items.empty()) return hipSuccess;
    g = std::max(1, std::min(g, (int)items.size()));
    for (size_t r0 = g; r0 < items.size(); r0 += 2 * (size_t)g)
        std::reverse(items.begin() + r0, items.begin() + std::min(items.size(), r0 + g));
    hipError_t e = hipMalloc(d, items.size() * sizeof(Item));
    if (e == hipSuccess)
        e = hipMemcpy(*d, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice);
    return e;
}

// Splits the work list by kernel (single-sweep / two-sweep / three-sweep
// tiles) and counts the launches each kernel needs.
hipError_t upload_items(ao_batch* b, const std::vector<Item>& items) {
    std::vector<Item> single, fused, tri;
    b->launches = b->launches_f = b->launches_3 = 0;
    for (const Item& it : items) {
        const int kind = kCands[it.cand].kind;
        const int P = passes_of(b->insts[it.inst].sweeps, kind);
        if (is_tri(kind)) {
            tri.push_back(it);
            b->launches_3 = std::max(b->launches_3, P);
        } else if (is_fused(kind)) {
            fused.push_back(it);
            b->launches_f = std::max(b->launches_f, P);
        } else {
            single.push_back(it);
            b->launches = std::max(b->launches, P);
        }
    }
    hipError_t e = upload_list(&b->d_items, &b->nitems, std::move(single), b->grid);
    if (e == hipSuccess) e = upload_list(&b->d_items_f, &b->nitems_f, std::move(fused), b->grid_f);
    if (e == hipSuccess) e = upload_list(&b->d_items_3, &b->nitems_3, std::move(tri), b->grid_3);
    return e;
}

hipError_t launch_sweeps(ao_batch* b, hipStream_t s) {
    for (const Inst& in : b->insts) {  // zero sweeps: the result is the input
        const size_t n = (size_t)in.nx * in.ny * in.nz;
        if (in.sweeps == 0 && n > 0) {
            hipError_t e = hipMemcpyAsync(in.out, in.u0, n * 8, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
        }
    }
    const int grid = std::min(b->nitems, b->grid), grid_f = std::min(b->nitems_f, b->grid_f);
    const int grid_3 = std::min(b->nitems_3, b->grid_3);
    const int L = std::max(b->launches, std::max(b->launches_f, b->launches_3));
    for (int l = 0; l < L; ++l) {
        if (l < b->launches && b->nitems > 0)
            hipLaunchKernelGGL(k_batch_sweep, dim3(grid), dim3(kThreads), 0, s, b->d_insts,
                               b->d_items, b->nitems, l);
        if (l < b->launches_f && b->nitems_f > 0)
            hipLaunchKernelGGL(k_batch_fused, dim3(grid_f), dim3(kThreads), 0, s, b->d_insts,
                               b->d_items_f, b->nitems_f, l);
        if (l < b->launches_3 && b->nitems_3 > 0)
            hipLaunchKernelGGL(k_batch_fused3, dim3(grid_3), dim3(kThreads), 0, s, b->d_insts,
                               b->d_items_3, b->nitems_3, l);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int rebuild(ao_batch* b) {
    hipError_t e = upload_items(b, make_items(b, -1, -1));
    if (e != hipSuccess) return fail(AO_EHIP, std::string("batch items: ") + hipGetErrorString(e));
    for (int k = 0; k < kBuckets; ++k) b->items_per_bucket[k] = 0;
    for (size_t q = 0; q < b->insts.size(); ++q) {
        const TileCfg& c = kCands[b->cand[b->bucket[q]]];
        const Inst& in = b->insts[q];
        if ((int64_t)in.nx * in.ny * in.nz == 0 || in.sweeps == 0) continue;
        b->items_per_bucket[b->bucket[q]] += ((in.nx + c.tx - 1) / c.tx) *
                                             ((in.ny + c.ty - 1) / c.ty) *
                                             ((in.nz + c.tz - 1) / c.tz);
    }
    b->graph_dirty = true;
    return AO_OK;
}

}  // namespace
}  // namespace ao

extern "C" {

int batch_create(const ao_args* inst, int count, ao_batch** out) {
    if (!out || count < 1 || !inst) return fail(AO_EINVAL, "need count >= 1 instances and out");
    std::unique_ptr<ao_batch> b(new (std::nothrow) ao_batch());
    if (!b) return fail(AO_ENOMEM, "batch allocation");
    size_t total = 0;
    for (int q = 0; q < count; ++q) {
        const ao_args& a = inst[q];
        if (a.kind != AO_JACOBI7_F64 || a.resident != 1)
            return fail(AO_EINVAL, "batched instances must be device-resident Jacobi regions");
        if (a.nx < 0 || a.ny < 0 || a.nz < 0 || a.sweeps < 0)
            return fail(AO_EINVAL, "negative size or sweep count");
        if (a.nx > (1 << 28)) return fail(AO_EINVAL, "nx above 2^28");
        const size_t n = (size_t)a.nx * a.ny * a.nz;
        if (n > 0 && (!a.u0 || !a.out)) return fail(AO_EINVAL, "u0/out is NULL");
        if (n > 0) {
            const char* u = (const char*)a.u0;
            const char* o = (const char*)a.out;
            if (u < o + n * 8 && o < u + n * 8) return fail(AO_EINVAL, "u0 and out overlap");
        }
        total += n;
    }
    hipError_t e = hipMalloc(&b->scratch, std::max<size_t>(total, 1) * sizeof(double));
    if (e != hipSuccess) return fail(AO_ENOMEM, std::string("batch scratch: ") + hipGetErrorString(e));
    size_t off = 0;
    for (int q = 0; q < count; ++q) {
        const ao_args& a = inst[q];
        Inst in{a.u0, a.out, b->scratch + off, a.nx, a.ny, a.nz, a.sweeps};
        off += (size_t)a.nx * a.ny * a.nz;
        b->insts.push_back(in);
        b->bucket.push_back(bucket_of(a.nx, a.ny, a.nz));
    }
    for (int k = 0; k < kBuckets; ++k) b->cand[k] = kDefaultCand[k];
    e = hipMalloc(&b->d_insts, b->insts.size() * sizeof(Inst));
    if (e == hipSuccess)
        e = hipMemcpy(b->d_insts, b->insts.data(), b->insts.size() * sizeof(Inst),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_cands), kCands, sizeof(kCands));
    if (e != hipSuccess) return fail(AO_EHIP, std::string("batch upload: ") + hipGetErrorString(e));
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // each persistent kernel runs as many workgroups as the device keeps
    // resident at once, so no workgroup waits for another to finish before
    // it starts striding over the items (8 per CU when the runtime cannot say)
    auto resident = [&](const void* k) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kThreads, 0) != hipSuccess ||
            per_cu < 1) {
            (void)hipGetLastError();
            per_cu = 8;
        }
        return std::max(1, cus) * per_cu;
    };
    b->grid = resident((const void*)k_batch_sweep);
    b->grid_f = resident((const void*)k_batch_fused);
    b->grid_3 = resident((const void*)k_batch_fused3);
    int rc = rebuild(b.get());
    if (rc) return rc;
    *out = b.release();
    return AO_OK;
}

int batch_autotune(ao_batch* b, void* stream, int warmup, int reps, int* chosen) {
    if (!b || warmup < 0 || reps < 1) return fail(AO_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return fail(AO_EHIP, "event creation");
    // median time of one execution of the items currently uploaded
    auto median_ms = [&](double* med) {
        std::vector<double> ts;
        for (int r = 0; r < warmup + reps && e == hipSuccess; ++r) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) e = launch_sweeps(b, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (r >= warmup) ts.push_back(ms);
        }
        if (e != hipSuccess) return;
        std::sort(ts.begin(), ts.end());
        *med = ts.size() % 2 ? ts[ts.size() / 2]
                             : 0.5 * (ts[ts.size() / 2 - 1] + ts[ts.size() / 2]);
    };
    int result[kBuckets];
    // first each bucket alone, every candidate tile
    for (int k = 0; k < kBuckets && e == hipSuccess; ++k) {
        result[k] = -1;
        bool any = false;
        for (int bk : b->bucket) any = any || bk == k;
        if (!any) continue;
        double best = INFINITY;
        for (int c = 0; c < kNumCands && e == hipSuccess; ++c) {
            e = upload_items(b, make_items(b, k, c));
            double med = INFINITY;
            if (e == hipSuccess) median_ms(&med);
            if (e == hipSuccess && med < best) {
                best = med;
                result[k] = c;
            }
        }
        if (e == hipSuccess) b->cand[k] = result[k];
    }
    // then each bucket again, largest first, timing the whole batch with
    // every other bucket on its current tile: the buckets share the
    // persistent kernels, so the tile a bucket runs best alone on (fewer,
    // larger tiles) can balance worse beside the others
    for (int k = kBuckets - 1; k >= 0 && e == hipSuccess; --k) {
        if (result[k] < 0) continue;
        double best = INFINITY;
        int pick = result[k];
        for (int c = 0; c < kNumCands && e == hipSuccess; ++c) {
            b->cand[k] = c;
            e = upload_items(b, make_items(b, -1, -1));
            double med = INFINITY;
            if (e == hipSuccess) median_ms(&med);
            if (e == hipSuccess && med < best) {
                best = med;
                pick = c;
            }
        }
        b->cand[k] = pick;
        result[k] = pick;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        rebuild(b);
        return fail(AO_EHIP, std::string("autotune: ") + hipGetErrorString(e));
    }
    int rc = rebuild(b);
    if (rc) return rc;
    if (chosen)
        for (int k = 0; k < kBuckets; ++k) chosen[k] = result[k];
    return AO_OK;
}

int batch_run(ao_batch* b, void* stream, int use_graph) {
    if (!b) return fail(AO_EINVAL, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (!use_graph) {
        e = launch_sweeps(b, s);
        if (e != hipSuccess) return fail(AO_EHIP, std::string("batch run: ") + hipGetErrorString(e));
        return AO_OK;
    }
    if (b->graph_dirty || !b->exec) {
        if (b->exec) hipGraphExecDestroy(b->exec);
        if (b->graph) hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        if (!b->cap_stream) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = launch_sweeps(b, b->cap_stream);
            e = hipStreamEndCapture(b->cap_stream, &b->graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(AO_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        }
        b->graph_dirty = false;
    }
    e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return fail(AO_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
    return AO_OK;
}

int batch_info(const ao_batch* b, int* instances, int* items, int* tiles_xyz) {
    if (!b) return fail(AO_EINVAL, "batch is NULL");
    for (int k = 0; k < kBuckets; ++k) {
        int cnt = 0;
        for (int bk : b->bucket) cnt += bk == k;
        if (instances) instances[k] = cnt;
        if (items) items[k] = b->items_per_bucket[k];
        if (tiles_xyz) {
            const TileCfg& c = kCands[b->cand[k]];
            tiles_xyz[3 * k] = c.tx;
            tiles_xyz[3 * k + 1] = c.ty;
            tiles_xyz[3 * k + 2] = c.tz;
        }
    }
    return AO_OK;
}

int batch_min_traffic(const ao_batch* b, double* bytes) {
    if (!b || !bytes) return fail(AO_EINVAL, "batch or bytes is NULL");
    double t = 0.0;
    for (size_t q = 0; q < b->insts.size(); ++q) {
        const Inst& in = b->insts[q];
        const double n = (double)in.nx * in.ny * in.nz;
        const int kind = kCands[b->cand[b->bucket[q]]].kind;
        // a zero-sweep instance is one copy: 16 B per point as well
        t += 16.0 * n * (in.sweeps == 0 ? 1 : passes_of(in.sweeps, kind));
    }
    *bytes = t;
    return AO_OK;
}

int batch_candidates(int* tiles) {
    if (tiles)
        for (int c = 0; c < kNumCands; ++c) {
            tiles[4 * c] = kCands[c].kind;
            tiles[4 * c + 1] = kCands[c].tx;
            tiles[4 * c + 2] = kCands[c].ty;
            tiles[4 * c + 3] = kCands[c].tz;
        }
    return kNumCands;
}

int batch_set_tiles(ao_batch* b, const int* cand) {
    if (!b || !cand) return fail(AO_EINVAL, "batch or cand is NULL");
    for (int k = 0; k < kBuckets; ++k)
        if (cand[k] < -1 || cand[k] >= kNumCands)
            return fail(AO_EINVAL, "tile candidate index out of range");
    for (int k = 0; k < kBuckets; ++k)
        if (cand[k] >= 0) b->cand[k] = cand[k];
    return rebuild(b);
}

int batch_destroy(ao_batch* b) {
    if (!b) return fail(AO_EINVAL, "batch is NULL");
    delete b;
    return AO_OK;
}

}  // extern "C"
