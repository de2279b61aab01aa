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

__global__ __launch_bounds__(1024) void k_thread_row(int n, const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ y) {
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
    y[i] = c.finish();
}

template <int W>
__global__ __launch_bounds__(1024) void k_wave_row(int n, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y) {
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
    if (live && g == 0) y[i] = c.finish();
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
                           const double* x, double* y, hipStream_t s);

hipError_t spmv_gpu(const ao_variant& v, SpmvPlan& p, const int32_t* col, const double* val,
                    const double* x, double* y, hipStream_t s) {
    if (p.n <= 0) return hipSuccess;
    const int B = v.bx;
    if (B <= 0 || B > 1024 || B % 64 != 0) return hipErrorInvalidConfiguration;
    if (v.family == AO_FAM_SPMV_THREAD_ROW) {
        if ((int64_t)p.max_len > ((int64_t)8 << kCounterLevels)) return hipErrorInvalidConfiguration;
        const unsigned grid = (unsigned)(((int64_t)p.n + B - 1) / B);
        hipLaunchKernelGGL(k_thread_row, dim3(grid), dim3(B), 0, s, p.n, p.row_ptr, col, val, x, y);
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
                           col, val, x, y);                                                        \
        break;
            AO_WR(1) AO_WR(2) AO_WR(4) AO_WR(8) AO_WR(16) AO_WR(32) AO_WR(64)
#undef AO_WR
            default:
                return hipErrorInvalidConfiguration;
        }
        return hipGetLastError();
    }
    if (v.family == AO_FAM_SPMV_MERGE_PATH) return spmv_merge_path(v, p, col, val, x, y, s);
    return hipErrorInvalidValue;
}

hipError_t spmv_merge_path(const ao_variant&, SpmvPlan&, const int32_t*, const double*,
                           const double*, double*, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace ao
