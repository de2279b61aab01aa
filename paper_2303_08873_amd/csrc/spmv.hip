// GPU variants of the FP64 CSR SpMV region y = A x (gfx950, wave64).
//
// Every variant reproduces one summation order per row -- the canonical
// pairwise tree over the row-local index: products p_r = fl(val * x[col])
// (no fused multiply-add; built with -ffp-contract=off), padded with -0.0
// to a power of two, leaves 2m and 2m+1 added, then pairs of pairs.  -0.0
// is the exact additive identity, so padding to any larger power of two, or
// summing any aligned power-of-two block on its own and combining the block
// sums by the same tree, gives the same bits.  That is what lets the
// variants split rows differently and still agree bit for bit:
//
//  thread-row  one thread per row: fixed 8-leaf trees, combined by a
//              binary-counter stack (completed aligned subtrees wait for
//              their right sibling; the stack collapses right to left).
//  wave-row    W lanes (W = power of two <= 64) per row: each W-leaf block
//              by an xor butterfly (offsets 1, 2, ..., W/2; absent lanes
//              hold -0.0), block sums by the counter.
//  merge-path  rows are cut into row-aligned 64-leaf units; workgroups take
//              equal shares of (units + nonzeros) so long and short rows
//              balance; unit sums of rows that straddle a share are finished
//              by a fix-up pass with the counter.
//
// An empty row gives +0.0 in every variant.
#include "internal.h"

namespace ao {
namespace {

// Binary-counter stack of completed aligned subtrees, levels 0..15 (rows of
// up to 2^16 blocks; longer rows are refused on the host before launch).
constexpr int kCounterLevels = 16;
struct Counter {
    static constexpr int L = kCounterLevels;
    double s[L];
    unsigned cnt;
    __device__ Counter() : cnt(0u) {}
    __device__ __forceinline__ void push(double x) {
        const unsigned z = (unsigned)__builtin_ctz(~cnt);
#pragma unroll
        for (int t = 0; t < L; ++t)
            if ((unsigned)t < z) x = s[t] + x;
#pragma unroll
        for (int t = 0; t < L; ++t)
            if ((unsigned)t == z) s[t] = x;
        ++cnt;
    }
    __device__ __forceinline__ double finish() const {
        if (cnt == 0u) return 0.0;
        double acc = 0.0;
        bool have = false;
#pragma unroll
        for (int t = 0; t < L; ++t) {
            if ((cnt >> t) & 1u) {
                acc = have ? s[t] + acc : s[t];
                have = true;
            }
        }
        return acc;
    }
};

__device__ __forceinline__ double prod(const int32_t* __restrict__ col,
                                       const double* __restrict__ val,
                                       const double* __restrict__ x, int64_t k) {
    return val[k] * x[col[k]];
}

// The value stored for finished row i: the canonical sum, or the
// relaxation update x_i + (omega * (b_i - s)) / d_i rounded step by step.
__device__ __forceinline__ double row_out(const SpmvEpi& ep, const double* __restrict__ x, int i,
                                          double s) {
    if (ep.b == nullptr) return s;
    const double r = ep.b[i] - s;
    const double t = ep.omega * r;
    const double u = t / ep.d[i];
    return x[i] + u;
}

__global__ __launch_bounds__(1024) void k_thread_row(int n, const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ y, SpmvEpi ep) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int32_t b = row_ptr[i], e = row_ptr[i + 1];
    Counter c;
    for (int32_t k0 = b; k0 < e; k0 += 8) {
        double p[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) p[q] = (k0 + q < e) ? prod(col, val, x, k0 + q) : -0.0;
        const double s01 = p[0] + p[1], s23 = p[2] + p[3], s45 = p[4] + p[5], s67 = p[6] + p[7];
        const double s03 = s01 + s23, s47 = s45 + s67;
        c.push(s03 + s47);
    }
    y[i] = row_out(ep, x, i, c.finish());
}

template <int W>
__global__ __launch_bounds__(1024) void k_wave_row(int n, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y, SpmvEpi ep) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i64 = gid / W;
    const int g = (int)(threadIdx.x % W);
    // every lane of a wave runs the same trip count so the shuffles are
    // uniform; lanes of rows past n carry no work
    const int i = (int)(i64 < n ? i64 : n - 1);
    const bool live = i64 < n;
    const int32_t b = row_ptr[i], e = live ? row_ptr[i + 1] : b;
    // trip count of the longest row among the wave's groups
    int32_t trips = (e - b + W - 1) / W;
#pragma unroll
    for (int off = W; off < 64; off <<= 1) trips = max(trips, __shfl_xor(trips, off));
    Counter c;
    for (int32_t t = 0; t < trips; ++t) {
        const int32_t k = b + t * W + g;
        double v = (k < e) ? prod(col, val, x, k) : -0.0;
#pragma unroll
        for (int off = 1; off < W; off <<= 1) v = v + __shfl_xor(v, off);
        if (t * W < e - b) c.push(v);
    }
    if (live && g == 0) y[i] = row_out(ep, x, i, c.finish());
}

// ---- features: one pass over row_ptr, deterministic two-level reduction ----

constexpr int kFeatBlocks = 1024;

__global__ __launch_bounds__(256) void k_feat_partial(int n, const int32_t* __restrict__ row_ptr,
                                                      double mean, double* __restrict__ psum,
                                                      int* __restrict__ pmax) {
    __shared__ double ss[256];
    __shared__ int sm[256];
    double acc = 0.0;
    int mx = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int len = row_ptr[i + 1] - row_ptr[i];
        const double d = (double)len - mean;
        acc += d * d;
        mx = max(mx, len);
    }
    ss[threadIdx.x] = acc;
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            ss[threadIdx.x] += ss[threadIdx.x + off];
            sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        psum[blockIdx.x] = ss[0];
        pmax[blockIdx.x] = sm[0];
    }
}

__global__ void k_feat_final(int nb, const double* __restrict__ psum, const int* __restrict__ pmax,
                             double* __restrict__ out_sum, int* __restrict__ out_max) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    int m = 0;
    for (int b = 0; b < nb; ++b) {
        s += psum[b];
        m = max(m, pmax[b]);
    }
    *out_sum = s;
    *out_max = m;
}

}  // namespace

hipError_t spmv_features(SpmvPlan& p, hipStream_t s) {
    for (int i = 0; i < AO_MAX_FEATURES; ++i) p.features[i] = 0.0f;
    if (p.n <= 0) return hipSuccess;
    int32_t ends[2];
    hipError_t e = hipMemcpyAsync(&ends[0], p.row_ptr, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&ends[1], p.row_ptr + p.n, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const double nnz = (double)(ends[1] - ends[0]);
    const double mean = nnz / p.n;
    const int nb = (int)std::min<int64_t>(kFeatBlocks, ((int64_t)p.n + 255) / 256);
    // one scratch allocation: psum[nb] | osum | pmax[nb] | omax
    char* buf = nullptr;
    e = hipMalloc(&buf, (size_t)nb * 12 + 16);
    if (e != hipSuccess) return e;
    double* psum = (double*)buf;
    double* osum = psum + nb;
    int* pmax = (int*)(osum + 1);
    int* omax = pmax + nb;
    double sum_h = 0.0;
    int max_h = 0;
    hipLaunchKernelGGL(k_feat_partial, dim3(nb), dim3(256), 0, s, p.n, p.row_ptr, mean, psum, pmax);
    e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_feat_final, dim3(1), dim3(64), 0, s, nb, psum, pmax, osum, omax);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&sum_h, osum, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&max_h, omax, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(buf);
    if (e != hipSuccess) return e;
    const double var = sum_h / p.n;
    p.features[0] = (float)log2((double)p.n);
    p.features[1] = nnz > 0 ? (float)log2(nnz) : 0.0f;
    p.features[2] = (float)mean;
    p.features[3] = (float)log2(1.0 + var);
    p.features[4] = max_h > 0 ? (float)log2((double)max_h) : 0.0f;
    p.max_len = max_h;
    return hipSuccess;
}

hipError_t spmv_merge_path(const ao_variant& v, SpmvPlan& p, const int32_t* col, const double* val,
                           const double* x, double* y, hipStream_t s, const SpmvEpi& ep);

hipError_t spmv_gpu(const ao_variant& v, SpmvPlan& p, const int32_t* col, const double* val,
                    const double* x, double* y, hipStream_t s, const SpmvEpi& ep,
                    bool values_ready) {
    if (p.n <= 0) return hipSuccess;
    if (v.family == AO_FAM_SPMV_XSLICE) return spmv_xslice(v, p, val, x, y, s, ep, values_ready);
    const int B = v.bx;
    if (B <= 0 || B > 1024 || B % 64 != 0) return hipErrorInvalidConfiguration;
    if (v.family == AO_FAM_SPMV_THREAD_ROW) {
        if ((int64_t)p.max_len > ((int64_t)8 << kCounterLevels)) return hipErrorInvalidConfiguration;
        const unsigned grid = (unsigned)(((int64_t)p.n + B - 1) / B);
        hipLaunchKernelGGL(k_thread_row, dim3(grid), dim3(B), 0, s, p.n, p.row_ptr, col, val, x, y,
                           ep);
        return hipGetLastError();
    }
    if (v.family == AO_FAM_SPMV_WAVE_ROW) {
        const int W = v.by == 0 ? 64 : v.by;
        if ((int64_t)p.max_len > ((int64_t)W << kCounterLevels)) return hipErrorInvalidConfiguration;
        const int64_t threads = (int64_t)p.n * W;
        const int64_t grid = (threads + B - 1) / B;
        if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
        switch (W) {
#define AO_WR(WW)                                                                                  \
    case WW:                                                                                       \
        hipLaunchKernelGGL(k_wave_row<WW>, dim3((unsigned)grid), dim3(B), 0, s, p.n, p.row_ptr, \
                           col, val, x, y, ep);                                                    \
        break;
            AO_WR(1) AO_WR(2) AO_WR(4) AO_WR(8) AO_WR(16) AO_WR(32) AO_WR(64)
#undef AO_WR
            default:
                return hipErrorInvalidConfiguration;
        }
        return hipGetLastError();
    }
    if (v.family == AO_FAM_SPMV_MERGE_PATH) return spmv_merge_path(v, p, col, val, x, y, s, ep);
    return hipErrorInvalidValue;
}

// ---- merge-path ------------------------------------------------------------
//
// Units: row i is cut into nu_i = max(1, ceil(L_i / 64)) row-aligned units
// of <= 64 leaves (an empty row keeps one empty unit so that y_i is
// written).  Unit (i, j) costs its leaf count + 1; a workgroup takes the
// units whose cumulative cost falls in [b*D, (b+1)*D), D = 4 * block size.
// The cost before unit (i, j) is base_i + 65 j with
// base_i = (row_ptr[i] - row_ptr[0]) + unit_ptr[i].

namespace {

// exclusive scan of per-row unit counts, three passes (1024 rows per block)
__global__ __launch_bounds__(1024) void k_units_block(int n, const int32_t* __restrict__ row_ptr,
                                                       int32_t* __restrict__ unit_ptr,
                                                       int32_t* __restrict__ block_sums) {
    __shared__ int32_t sh[1024];
    const int i = (int)(blockIdx.x * 1024 + threadIdx.x);
    int32_t v = 0;
    if (i < n) {
        const int32_t len = row_ptr[i + 1] - row_ptr[i];
        v = len > 0 ? (len + 63) / 64 : 1;
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele
        const int32_t t = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) unit_ptr[i] = sh[threadIdx.x] - v;  // exclusive within the block
    if (threadIdx.x == 1023) block_sums[blockIdx.x] = sh[1023];
}

__global__ __launch_bounds__(1024) void k_units_top(int nb, int32_t* __restrict__ block_sums,
                                                     int32_t* __restrict__ total) {
    // one block: exclusive scan of nb block sums, 1024-wide pieces in order
    __shared__ int32_t sh[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int32_t v = i < nb ? block_sums[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t t = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) block_sums[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(1024) void k_units_add(int n, int32_t* __restrict__ unit_ptr,
                                                     const int32_t* __restrict__ block_sums,
                                                     const int32_t* __restrict__ total) {
    const int i = (int)(blockIdx.x * 1024 + threadIdx.x);
    if (i < n) unit_ptr[i] += block_sums[blockIdx.x];
    if (i == 0) unit_ptr[n] = *total;
}

__device__ __forceinline__ int64_t unit_base(const int32_t* row_ptr, const int32_t* unit_ptr,
                                             int i) {
    return (int64_t)(row_ptr[i] - row_ptr[0]) + unit_ptr[i];
}

// start unit of block b = first unit whose cost offset is >= b*D
__global__ void k_partition(int n, int nb, int D, const int32_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ unit_ptr, int32_t* __restrict__ srow,
                            int32_t* __restrict__ sunit) {
    const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b > nb) return;
    const int64_t target = (int64_t)b * D;
    // largest row i with base_i <= target (base is nondecreasing, base_0 = 0)
    int lo = 0, hi = n;  // answer in [0, n]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (unit_base(row_ptr, unit_ptr, mid) <= target) lo = mid; else hi = mid - 1;
    }
    int i = lo;
    int32_t j = 0;
    if (i < n) {
        const int64_t base = unit_base(row_ptr, unit_ptr, i);
        const int32_t nu = unit_ptr[i + 1] - unit_ptr[i];
        const int64_t jj = (target - base + 64) / 65;  // ceil((target - base) / 65)
        if (jj >= nu) {
            i += 1;
            j = 0;
        } else {
            j = (int32_t)jj;
        }
    }
    if (b == nb) {
        i = n;
        j = 0;
    }
    srow[b] = i;
    sunit[b] = j;
}

// The partition tables must describe this row_ptr (the runtime keys them on
// the structure id); every index below is nevertheless clamped to its
// buffer, so tables of another matrix give wrong sums, never stray accesses.
template <int B>
__global__ __launch_bounds__(B) void k_merge_path(int n, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col,
                                                  const double* __restrict__ val,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ y,
                                                  const int32_t* __restrict__ srow,
                                                  const int32_t* __restrict__ sunit,
                                                  const int32_t* __restrict__ unit_ptr,
                                                  double* __restrict__ unit_sums, int64_t units,
                                                  SpmvEpi ep) {
    constexpr int D = 4 * B;
    // a unit that starts just below the block's cost limit may extend 64
    // leaves past it: at most D + 64 leaves and D rows per block
    __shared__ double s[D + 64];
    __shared__ int32_t rs[D + 2];  // row starts (global nnz offsets) of the block's rows
    const int b = (int)blockIdx.x;
    const int i0 = min(max(srow[b], 0), n), i1 = min(max(srow[b + 1], 0), n);
    const int j0 = max(sunit[b], 0), j1 = max(sunit[b + 1], 0);
    const int32_t kbeg = row_ptr[0], kend = row_ptr[n];
    const int32_t e0 = (i0 < n ? row_ptr[i0] : kend) + 64 * j0;
    int32_t e1 = (i1 < n ? row_ptr[i1] : kend) + 64 * j1;
    if (i1 < n) e1 = min(e1, row_ptr[i1 + 1]);
    const int cnt = min(max(e1 - e0, 0), D + 64);
    const int ilast = (j1 > 0) ? i1 : i1 - 1;  // last row touched
    const int nrows = min(max(ilast - i0 + 1, 0), min(D, n - i0));
    for (int t = (int)threadIdx.x; t <= nrows && t < D + 2; t += B) rs[t] = row_ptr[i0 + t];
    constexpr int E = 4 + (64 + B - 1) / B;  // leaves per thread: ceil((D + 64) / B)
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = (int)threadIdx.x + e * B;
        if (p < cnt) {
            const int64_t k = (int64_t)e0 + p;
            s[p] = (k >= kbeg && k < kend) ? val[k] * x[col[k]] : 0.0;
        }
    }
    __syncthreads();
    // each leaf's position r in its row and the row length, found once
    int32_t rr[E], ln[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = (int)threadIdx.x + e * B;
        rr[e] = -1;
        ln[e] = 0;
        if (p < cnt) {
            const int32_t g = e0 + p;
            int lo = 0, hi = nrows - 1;  // row t with rs[t] <= g < rs[t + 1]
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (rs[mid] <= g) lo = mid; else hi = mid - 1;
            }
            rr[e] = g - rs[lo];
            ln[e] = rs[lo + 1] - rs[lo];
        }
    }
    // canonical tree inside each 64-leaf unit
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = (int)threadIdx.x + e * B;
            const int32_t r = rr[e], q = r & 63;
            if (r >= 0 && (q & (2 * d - 1)) == 0 && q + d < 64 && r + d < ln[e] && p + d < cnt)
                s[p] = s[p] + s[p + d];
        }
        __syncthreads();
    }
    // rows: complete ones are finished here, split ones leave their unit sums
    constexpr int kMaxUnits = (D + 64) / 64 + 1;  // units of one row inside one block
    for (int t = (int)threadIdx.x; t < nrows; t += B) {
        const int i = i0 + t;
        const int32_t rb = rs[t], re = rs[t + 1];
        const int32_t nu = re > rb ? (re - rb + 63) / 64 : 1;
        const int32_t ja = (t == 0) ? j0 : 0;
        const int32_t jb = min((i == i1) ? j1 : nu, ja + kMaxUnits);  // units [ja, jb) here
        const bool whole = (ja == 0) && (i < i1);
        if (whole) {
            Counter c;
            for (int32_t j = ja; j < jb; ++j) {
                const int32_t g = rb + 64 * j;
                const int32_t o = g - e0;
                if (g < re && o >= 0 && o < cnt) c.push(s[o]);
            }
            y[i] = row_out(ep, x, i, c.finish());
        } else {
            for (int32_t j = ja; j < jb; ++j) {
                const int32_t g = rb + 64 * j;
                const int32_t o = g - e0;
                const int64_t u = (int64_t)unit_ptr[i] + j;
                if (u >= 0 && u < units) unit_sums[u] = (g < re && o >= 0 && o < cnt) ? s[o] : 0.0;
            }
        }
    }
}

// one thread per block boundary: the first boundary inside a row finishes it
__global__ void k_merge_fixup(int n, int nb, const int32_t* __restrict__ row_ptr,
                              const int32_t* __restrict__ srow, const int32_t* __restrict__ sunit,
                              const int32_t* __restrict__ unit_ptr,
                              const double* __restrict__ unit_sums, int64_t units,
                              const double* __restrict__ x, double* __restrict__ y, SpmvEpi ep) {
    const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b <= 0 || b >= nb) return;
    if (sunit[b] == 0) return;
    const int i = srow[b];
    if (i < 0 || i >= n) return;
    if (srow[b - 1] == i && sunit[b - 1] > 0) return;  // an earlier boundary splits this row
    Counter c;
    const int32_t len = row_ptr[i + 1] - row_ptr[i];
    const int32_t nu = (len + 63) / 64;
    for (int32_t j = 0; j < nu; ++j) {
        const int64_t u = (int64_t)unit_ptr[i] + j;
        c.push((u >= 0 && u < units) ? unit_sums[u] : 0.0);
    }
    y[i] = row_out(ep, x, i, c.finish());
}

}  // namespace

hipError_t spmv_prepare_merge(SpmvPlan& p, int B, hipStream_t s) {
    const int D = 4 * B;
    for (const auto& m : p.mp)
        if (m.D == D) return hipSuccess;
    hipError_t e = hipSuccess;
    if (!p.unit_ptr) {
        const int nblk = (p.n + 1023) / 1024;
        int32_t* bs = nullptr;
        e = hipMalloc(&p.unit_ptr, ((size_t)p.n + 1) * 4);
        if (e == hipSuccess) e = hipMalloc(&bs, ((size_t)nblk + 1) * 4);
        if (e != hipSuccess) {
            if (bs) hipFree(bs);
            return e;
        }
        hipLaunchKernelGGL(k_units_block, dim3(nblk), dim3(1024), 0, s, p.n, p.row_ptr, p.unit_ptr,
                           bs);
        hipLaunchKernelGGL(k_units_top, dim3(1), dim3(1024), 0, s, nblk, bs, bs + nblk);
        hipLaunchKernelGGL(k_units_add, dim3(nblk), dim3(1024), 0, s, p.n, p.unit_ptr, bs,
                           bs + nblk);
        e = hipGetLastError();
        int32_t total = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&total, p.unit_ptr + p.n, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        hipFree(bs);
        if (e != hipSuccess) return e;
        p.units = total;
        e = hipMalloc(&p.unit_sums, (size_t)std::max<int64_t>(p.units, 1) * 8);
        if (e != hipSuccess) return e;
    }
    const int64_t cost = p.nnz + p.units;
    const int64_t nb = (cost + D - 1) / D;
    if (nb > 0x7ffffffe) return hipErrorInvalidConfiguration;
    SpmvPlan::MergeSplit m;
    m.D = D;
    m.blocks = (int)std::max<int64_t>(nb, 1);
    e = hipMalloc(&m.srow, ((size_t)m.blocks + 1) * 8);
    if (e != hipSuccess) return e;
    m.sunit = m.srow + m.blocks + 1;
    hipLaunchKernelGGL(k_partition, dim3((m.blocks + 256) / 256), dim3(256), 0, s, p.n, m.blocks,
                       D, p.row_ptr, p.unit_ptr, m.srow, m.sunit);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        hipFree(m.srow);
        return e;
    }
    p.mp.push_back(m);
    return hipSuccess;
}

hipError_t spmv_merge_path(const ao_variant& v, SpmvPlan& p, const int32_t* col, const double* val,
                           const double* x, double* y, hipStream_t s, const SpmvEpi& ep) {
    const int B = v.bx;
    const SpmvPlan::MergeSplit* m = nullptr;
    for (const auto& q : p.mp)
        if (q.D == 4 * B) m = &q;
    if (!m) return hipErrorNotReady;  // plan not prepared (the runtime prepares it)
    switch (B) {
#define AO_MP(BB)                                                                            \
    case BB:                                                                                 \
        hipLaunchKernelGGL((k_merge_path<BB>), dim3(m->blocks), dim3(BB), 0, s, p.n,          \
                           p.row_ptr, col, val, x, y, m->srow, m->sunit, p.unit_ptr,          \
                           p.unit_sums, p.units, ep);                                         \
        break;
        AO_MP(64) AO_MP(128) AO_MP(256) AO_MP(512) AO_MP(1024)
#undef AO_MP
        default:
            return hipErrorInvalidConfiguration;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_fixup, dim3((m->blocks + 255) / 256), dim3(256), 0, s, p.n,
                       m->blocks, p.row_ptr, m->srow, m->sunit, p.unit_ptr, p.unit_sums, p.units,
                       x, y, ep);
    return hipGetLastError();
}


// ---- gather probe ------------------------------------------------------------
//
// The memory access of a gather-per-nonzero SpMV and nothing else: idx[k]
// streamed once (non-temporal), x[idx[k]] gathered, the gathered values
// summed per wave so that no load is dead.  Workgroup g covers the 2048
// entries [2048 g, 2048 g + 2048); on a round-robin dispatch it runs on XCD
// g % 8, so an index array whose chunk g only names columns of one slice
// per XCD measures gathers that stay in that XCD's L2.

namespace {

constexpr int kProbeChunk = 2048;  // entries per workgroup (256 threads x 8)

__global__ __launch_bounds__(256) void k_gather_probe(const int32_t* __restrict__ idx,
                                                      const double* __restrict__ x, int64_t m,
                                                      int64_t nx, double* __restrict__ out) {
    const int64_t lo = (int64_t)blockIdx.x * kProbeChunk;
    constexpr int U = kProbeChunk / 256;
    int32_t c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t j = lo + threadIdx.x + 256 * u;
        const int32_t v = j < m ? __builtin_nontemporal_load(idx + j) : 0;
        c[u] = (v >= 0 && v < nx) ? v : 0;
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t j = lo + threadIdx.x + 256 * u;
        if (j < m) acc += x[c[u]];
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) out[(int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)] = acc;
}

}  // namespace

int64_t gather_probe_out_len(int64_t m) { return 4 * ((m + kProbeChunk - 1) / kProbeChunk); }

hipError_t gather_probe(const int32_t* idx, const double* x, int64_t m, int64_t nx, double* out,
                        hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const int64_t blocks = (m + kProbeChunk - 1) / kProbeChunk;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_gather_probe, dim3((unsigned)blocks), dim3(256), 0, s, idx, x, m, nx, out);
    return hipGetLastError();
}

}  // namespace ao
