// SpMV family with x gathered from LDS (gfx950, wave64): x-slice SpMV.
//
// A gather-per-nonzero SpMV over a random sparsity pattern is bound by the
// gathers themselves: each one pulls a 128-byte line of x into L2 from the
// Infinity Cache.  This family makes every gather an LDS read instead.
// Columns are cut into slices of SW = 2^sw columns (8K or 16K: 64 or 128 KB
// of x), rows into blocks of at most DN = 4096 cost units (one per nonzero
// and one per row; at most DCAP = 8192 nonzeros).  A per-matrix plan orders
// the nonzeros slice by slice (slice outer, then block, then CSR order) and
// keeps, per place, the column inside its slice and the position inside its
// block (16 bits each).  One execution:
//
//   permute   (only when the values changed) the values into that order;
//   products  one workgroup per chunk of a slice loads the slice of x into
//             LDS and forms fl(val * x[col]) for its places, streaming;
//   reduce    one workgroup per row block scatters the block's products from
//             their slice pieces into LDS at their CSR positions, sums every
//             row-aligned 64-leaf unit by the canonical tree (one thread per
//             unit), then combines the unit sums of longer rows by the same
//             tree, and stores y (or the relaxation update).
//
// The products are the same rounded products and the tree is the same
// aligned pairwise tree (absent leaves as -0.0, the exact additive
// identity) as in every other family, so the result is bit-identical.
#include "internal.h"

namespace ao {
namespace {

constexpr int kDN = 4096;      // cost units (nonzeros + rows) per row block
constexpr int kDCAP = 8192;    // nonzeros a row block can hold in LDS
constexpr int kMaxSlices = 1024;
constexpr int kRedThreads = 512;
constexpr int kProdThreads = 1024;
constexpr int kProdChunk = 65536;  // places per products workgroup

// ---- plan ----------------------------------------------------------------

// rb[t] = first row i whose cost (row_ptr[i] - row_ptr[0]) + i is >= t * DN
// (the cost is strictly increasing in i); rb[nb] = n
__global__ void k_xs_blocks(int n, int nb, const int32_t* __restrict__ row_ptr,
                            int32_t* __restrict__ rb) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t > nb) return;
    if (t == nb) {
        rb[t] = n;
        return;
    }
    const int64_t target = (int64_t)t * kDN;
    const int32_t k0 = row_ptr[0];
    int lo = 0, hi = n;  // first i in [0, n] with cost(i) >= target (cost(n) = nnz + n)
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)(row_ptr[mid] - k0) + mid >= target) hi = mid; else lo = mid + 1;
    }
    rb[t] = lo;
}

// *out = largest column index (the matrix may be rectangular: x can be
// longer than y); *out must start at 0
__global__ __launch_bounds__(256) void k_xs_colmax(int32_t kb, int32_t ke,
                                                   const int32_t* __restrict__ col,
                                                   int32_t* __restrict__ out) {
    int32_t m = 0;
    for (int64_t k = kb + (int64_t)blockIdx.x * 256 + threadIdx.x; k < ke;
         k += (int64_t)gridDim.x * 256)
        m = max(m, col[k]);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) m = max(m, __shfl_xor(m, d));
    if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// cnt[s * nb + t] = nonzeros of block t in slice s (workgroup per block)
__global__ __launch_bounds__(256) void k_xs_count(int nb, int ns, int sw,
                                                  const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ rb,
                                                  int32_t* __restrict__ cnt) {
    __shared__ int32_t hist[kMaxSlices];
    const int t = (int)blockIdx.x;
    for (int s = (int)threadIdx.x; s < ns; s += 256) hist[s] = 0;
    __syncthreads();
    const int32_t kb = row_ptr[rb[t]], ke = row_ptr[rb[t + 1]];
    for (int32_t k = kb + (int32_t)threadIdx.x; k < ke; k += 256) {
        const int s = min(max(col[k] >> sw, 0), ns - 1);
        atomicAdd(&hist[s], 1);
    }
    __syncthreads();
    for (int s = (int)threadIdx.x; s < ns; s += 256) cnt[(int64_t)s * nb + t] = hist[s];
}

// exclusive scan of count entries, 1024 per block; block sums out
__global__ __launch_bounds__(1024) void k_xs_scan_block(int64_t count,
                                                        const int32_t* __restrict__ in,
                                                        int32_t* __restrict__ out,
                                                        int32_t* __restrict__ sums) {
    __shared__ int32_t sh[1024];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int32_t v = i < count ? in[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t a = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += a;
        __syncthreads();
    }
    if (i < count) out[i] = sh[threadIdx.x] - v;
    if (threadIdx.x == 1023) sums[blockIdx.x] = sh[1023];
}

// one workgroup: exclusive scan of the nblk block sums in place, total out
__global__ __launch_bounds__(1024) void k_xs_scan_top(int nblk, int32_t* __restrict__ sums,
                                                      int32_t* __restrict__ total) {
    __shared__ int32_t sh[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nblk; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int32_t v = i < nblk ? sums[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t a = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < nblk) sums[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(1024) void k_xs_scan_add(int64_t count, int32_t* __restrict__ out,
                                                      const int32_t* __restrict__ sums,
                                                      const int32_t* __restrict__ total) {
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < count) out[i] += sums[blockIdx.x];
    if (i == 0) out[count] = *total;
}

// Places (one wave per block): the block's nonzeros in CSR order, 64 at a
// time; a lane's place is its slice's cursor plus the number of earlier
// lanes of the chunk in the same slice, so each piece keeps CSR order.
__global__ __launch_bounds__(64) void k_xs_place(int nb, int ns, int sw,
                                                 const int32_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col,
                                                 const int32_t* __restrict__ rb,
                                                 const int32_t* __restrict__ off, int64_t places,
                                                 uint16_t* __restrict__ bcol,
                                                 uint16_t* __restrict__ bk) {
    __shared__ int32_t cur[kMaxSlices];
    const int t = (int)blockIdx.x;
    const int lane = (int)threadIdx.x;
    for (int s = lane; s < ns; s += 64) cur[s] = off[(int64_t)s * nb + t];
    __syncthreads();
    const int32_t kb = row_ptr[rb[t]], ke = row_ptr[rb[t + 1]];
    for (int32_t c = kb; c < ke; c += 64) {
        const int32_t k = c + lane;
        const bool live = k < ke;
        const int32_t cc = live ? col[k] : 0;
        const int s = live ? min(max(cc >> sw, 0), ns - 1) : -1;
        int before = 0, same = 0;
        for (int m = 0; m < 64; ++m) {
            const int sm = __shfl(s, m);
            const int eq = (sm == s) ? 1 : 0;
            same += eq;
            before += (m < lane) ? eq : 0;
        }
        int32_t base = 0;
        if (live) base = cur[s];
        __syncthreads();
        if (live) {
            const int64_t j = (int64_t)base + before;
            if (j >= 0 && j < places) {
                bcol[j] = (uint16_t)(cc - (s << sw));
                bk[j] = (uint16_t)(k - kb);
            }
            if (before == same - 1) cur[s] = base + same;  // the slice's last lane
        }
        __syncthreads();
    }
}

// Units: row i holds max(1, ceil(L_i / 64)) row-aligned 64-leaf units.
__global__ __launch_bounds__(1024) void k_xs_unit_counts(int n, const int32_t* __restrict__ row_ptr,
                                                         int32_t* __restrict__ nu) {
    const int i = (int)(blockIdx.x * 1024 + threadIdx.x);
    if (i >= n) return;
    const int32_t len = row_ptr[i + 1] - row_ptr[i];
    nu[i] = len > 0 ? (len + 63) / 64 : 1;
}

// uinfo[u] = (row - rb[t]) << 16 | unit index in the row, for the units of
// row i (its block t = cost(i) / DN)
__global__ __launch_bounds__(256) void k_xs_units(int n, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ unit_ptr,
                                                  const int32_t* __restrict__ rb,
                                                  int64_t units, uint32_t* __restrict__ uinfo) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int t = (int)(((int64_t)(row_ptr[i] - row_ptr[0]) + i) / kDN);
    const uint32_t r = (uint32_t)(i - rb[t]);
    const int32_t u0 = unit_ptr[i], u1 = unit_ptr[i + 1];
    for (int32_t u = u0; u < u1; ++u)
        if (u >= 0 && u < units) uinfo[u] = (r << 16) | (uint32_t)(u - u0);
}

// ---- execution -----------------------------------------------------------

// The pieces of block t: starts (slice-major offsets) and an inclusive
// prefix of their lengths, in LDS; returns the block's place count.
__device__ int load_pieces(int t, int ns, int nb, const int32_t* __restrict__ off, int32_t* start,
                           int32_t* pre) {
    // piece (s, t) = [off[s*nb + t], off[s*nb + t + 1])
    for (int s = (int)threadIdx.x; s < ns; s += (int)blockDim.x) {
        const int64_t q = (int64_t)s * nb + t;
        start[s] = off[q];
        pre[s] = off[q + 1] - off[q];
    }
    __syncthreads();
    // inclusive scan of pre[0..ns) by one wave (ns <= kMaxSlices)
    if (threadIdx.x < 64) {
        int32_t carry = 0;
        for (int base = 0; base < ns; base += 64) {
            const int s = base + (int)threadIdx.x;
            int32_t v = s < ns ? pre[s] : 0;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int32_t a = __shfl_up(v, d);
                if ((int)threadIdx.x >= d) v += a;
            }
            if (s < ns) pre[s] = carry + v;
            carry += __shfl(v, 63);
        }
    }
    __syncthreads();
    return ns > 0 ? pre[ns - 1] : 0;
}

// place of the e-th entry of the block (pieces in slice order)
__device__ __forceinline__ int64_t place_of(int e, int ns, const int32_t* start, const int32_t* pre) {
    int lo = 0, hi = ns - 1;  // first s with pre[s] > e
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] > e) hi = mid; else lo = mid + 1;
    }
    const int32_t before = lo > 0 ? pre[lo - 1] : 0;
    return (int64_t)start[lo] + (e - before);
}

// XCD-aware order: consecutive blocks on one XCD (round-robin dispatch puts
// workgroup g on XCD g % 8), so the line shared by the pieces of adjacent
// blocks is fetched into one L2
__device__ __forceinline__ int xcd_block(int g, int nb) {
    const int per = (nb + 7) / 8;
    return (g & 7) * per + (g >> 3);
}

// bval[place] = val[kb + bk[place]] (workgroup per row block)
__global__ __launch_bounds__(kRedThreads) void k_xs_permute(int nb, int ns, int64_t places,
                                                            const int32_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ rb,
                                                            const int32_t* __restrict__ off,
                                                            const uint16_t* __restrict__ bk,
                                                            const double* __restrict__ val,
                                                            double* __restrict__ bval) {
    __shared__ int32_t start[kMaxSlices], pre[kMaxSlices];
    const int t = xcd_block((int)blockIdx.x, nb);
    if (t >= nb) return;
    const int total = load_pieces(t, ns, nb, off, start, pre);
    const int32_t kb = row_ptr[rb[t]], kend = row_ptr[rb[nb]];
    for (int e = (int)threadIdx.x; e < total; e += kRedThreads) {
        const int64_t j = min(max(place_of(e, ns, start, pre), (int64_t)0), places - 1);
        bval[j] = val[min(kb + (int32_t)bk[j], kend - 1)];
    }
}

// prod[place] = bval[place] * x[slice base + bcol[place]] over one chunk of
// one slice, x of the slice in LDS
template <int SWL>
__global__ __launch_bounds__(kProdThreads) void k_xs_products(int64_t ncols, int ns, int nb,
                                                              const int32_t* __restrict__ off,
                                                              const int32_t* __restrict__ chunk_first,
                                                              const uint16_t* __restrict__ bcol,
                                                              const double* __restrict__ bval,
                                                              const double* __restrict__ x,
                                                              double* __restrict__ prod) {
    constexpr int SW = 1 << SWL;
    __shared__ double xs[SW];
    // chunk g belongs to the slice s with chunk_first[s] <= g < chunk_first[s + 1]
    const int g = (int)blockIdx.x;
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunk_first[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const int s = lo;
    const int64_t base = (int64_t)s << SWL;
    const int w = (int)min((int64_t)SW, ncols - base);
    for (int c = (int)threadIdx.x; c < SW; c += kProdThreads) xs[c] = c < w ? x[base + c] : 0.0;
    __syncthreads();
    const int64_t p0 = off[(int64_t)s * nb], p1 = off[(int64_t)(s + 1) * nb];
    const int64_t lo_j = p0 + (int64_t)(g - chunk_first[s]) * kProdChunk;
    const int64_t hi_j = min(p1, lo_j + kProdChunk);
    constexpr int U = 4;
    for (int64_t j0 = lo_j + threadIdx.x; j0 < hi_j; j0 += (int64_t)kProdThreads * U) {
        uint16_t c[U];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = j0 + (int64_t)u * kProdThreads;
            c[u] = j < hi_j ? __builtin_nontemporal_load(bcol + j) : (uint16_t)0;
            v[u] = j < hi_j ? __builtin_nontemporal_load(bval + j) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = j0 + (int64_t)u * kProdThreads;
            if (j < hi_j) __builtin_nontemporal_store(v[u] * xs[c[u] & (SW - 1)], prod + j);
        }
    }
}

// canonical sum of m (0..64) consecutive leaves s[0..m): eight aligned
// 8-leaf subtrees, then the 8-wide tree over them; absent leaves -0.0
__device__ __forceinline__ double unit_sum(const double* s, int m) {
    double g[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        g[q] = -0.0;
        if (q * 8 < m) {
            double l[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) l[e] = (q * 8 + e < m) ? s[q * 8 + e] : -0.0;
            g[q] = ((l[0] + l[1]) + (l[2] + l[3])) + ((l[4] + l[5]) + (l[6] + l[7]));
        }
    }
    return ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]));
}

// canonical combine of nu unit sums at stride 64: binary counter of
// completed aligned subtrees, collapsed right to left at the end
__device__ __forceinline__ double combine_units(const double* s, int nu) {
    constexpr int L = 8;  // up to 256 units
    double st[L];
    unsigned cnt = 0u;
    for (int j = 0; j < nu; ++j) {
        double v = s[64 * j];
        const unsigned z = (unsigned)__builtin_ctz(~cnt);
#pragma unroll
        for (int q = 0; q < L; ++q)
            if ((unsigned)q < z) v = st[q] + v;
#pragma unroll
        for (int q = 0; q < L; ++q)
            if ((unsigned)q == z) st[q] = v;
        ++cnt;
    }
    double acc = 0.0;
    bool have = false;
#pragma unroll
    for (int q = 0; q < L; ++q) {
        if ((cnt >> q) & 1u) {
            acc = have ? st[q] + acc : st[q];
            have = true;
        }
    }
    return acc;
}

__device__ __forceinline__ double out_value(const SpmvEpi& ep, const double* __restrict__ x, int i,
                                            double s) {
    if (ep.b == nullptr) return s;
    const double r = ep.b[i] - s;
    const double t = ep.omega * r;
    const double u = t / ep.d[i];
    return x[i] + u;
}

__global__ __launch_bounds__(kRedThreads) void k_xs_reduce(int n, int nb, int ns, int64_t places,
                                                           const int32_t* __restrict__ row_ptr,
                                                           const int32_t* __restrict__ rb,
                                                           const int32_t* __restrict__ off,
                                                           const uint16_t* __restrict__ bk,
                                                           const double* __restrict__ prod,
                                                           const int32_t* __restrict__ unit_ptr,
                                                           const uint32_t* __restrict__ uinfo,
                                                           const double* __restrict__ x,
                                                           double* __restrict__ y, SpmvEpi ep) {
    __shared__ double sl[kDCAP];
    __shared__ int32_t start[kMaxSlices], pre[kMaxSlices];
    const int t = xcd_block((int)blockIdx.x, nb);
    if (t >= nb) return;
    const int total = min(load_pieces(t, ns, nb, off, start, pre), kDCAP);
    const int r0 = rb[t], r1 = rb[t + 1];
    const int32_t kb = row_ptr[r0];
    for (int e = (int)threadIdx.x; e < total; e += kRedThreads) {
        const int64_t j = min(max(place_of(e, ns, start, pre), (int64_t)0), places - 1);
        sl[bk[j] & (kDCAP - 1)] = prod[j];
    }
    __syncthreads();
    // one thread per unit: units of a row with one unit finish the row,
    // others leave their sum in the unit's first leaf slot
    const int32_t u0 = unit_ptr[r0], u1 = unit_ptr[r1];
    for (int32_t u = u0 + (int32_t)threadIdx.x; u < u1; u += kRedThreads) {
        const uint32_t info = uinfo[u];
        const int i = min(r0 + (int)(info >> 16), r1 - 1);
        const int jn = (int)(info & 0xffffu);
        const int32_t rs = row_ptr[i] - kb, re = row_ptr[i + 1] - kb;
        const int32_t a = rs + 64 * jn;
        const int m = (int)min(max(re - a, 0), 64);
        const bool in_lds = a >= 0 && a + m <= kDCAP;
        const double v = in_lds ? unit_sum(sl + a, m) : 0.0;
        if (re - rs <= 64) {
            if (i < n) y[i] = out_value(ep, x, i, re > rs ? v : 0.0);
        } else if (in_lds) {
            sl[a] = v;
        }
    }
    __syncthreads();
    for (int i = r0 + (int)threadIdx.x; i < r1; i += kRedThreads) {
        const int32_t rs = row_ptr[i] - kb, re = row_ptr[i + 1] - kb;
        if (re - rs <= 64) continue;
        const int nu = (re - rs + 63) / 64;
        const bool in_lds = rs >= 0 && rs + 64 * (nu - 1) < kDCAP;
        y[i] = out_value(ep, x, i, in_lds ? combine_units(sl + rs, nu) : 0.0);
    }
}

}  // namespace

// Largest row the family takes: a block holds at most DN - 1 cost units
// before its last row starts, plus that row.
int spmv_xslice_max_row() { return kDCAP - kDN + 1; }

hipError_t spmv_prepare_xslice(SpmvPlan& p, int swl, const int32_t* col, hipStream_t s) {
    for (const auto& q : p.xs)
        if (q.swl == swl) return hipSuccess;
    if (swl != 13 && swl != 14) return hipErrorInvalidConfiguration;
    SpmvPlan::XSlice q;
    q.swl = swl;
    if (p.n <= 0) {
        p.xs.push_back(q);
        return hipSuccess;
    }
    if (p.max_len > spmv_xslice_max_row()) return hipErrorInvalidConfiguration;
    // columns: up to the largest index the matrix holds
    int32_t ends[2] = {0, 0};
    int32_t* d_max = nullptr;
    hipError_t e0 = hipMemcpyAsync(&ends[0], p.row_ptr, 4, hipMemcpyDeviceToHost, s);
    if (e0 == hipSuccess) e0 = hipMemcpyAsync(&ends[1], p.row_ptr + p.n, 4, hipMemcpyDeviceToHost, s);
    if (e0 == hipSuccess) e0 = hipStreamSynchronize(s);
    if (e0 == hipSuccess) e0 = hipMalloc(&d_max, 4);
    if (e0 == hipSuccess) e0 = hipMemsetAsync(d_max, 0, 4, s);
    if (e0 == hipSuccess && ends[1] > ends[0]) {
        const int64_t g = std::min<int64_t>(4096, ((int64_t)ends[1] - ends[0] + 255) / 256);
        hipLaunchKernelGGL(k_xs_colmax, dim3((unsigned)g), dim3(256), 0, s, ends[0], ends[1], col,
                           d_max);
        e0 = hipGetLastError();
    }
    int32_t cmax = 0;
    if (e0 == hipSuccess) e0 = hipMemcpyAsync(&cmax, d_max, 4, hipMemcpyDeviceToHost, s);
    if (e0 == hipSuccess) e0 = hipStreamSynchronize(s);
    if (d_max) hipFree(d_max);
    if (e0 != hipSuccess) return e0;
    q.ncols = (int64_t)cmax + 1;
    const int64_t ns = (q.ncols + (1 << swl) - 1) >> swl;
    if (ns > kMaxSlices) return hipErrorInvalidConfiguration;
    const int64_t cost = p.nnz + p.n;
    const int64_t nb = (cost + kDN - 1) / kDN;
    if (nb > 0x3fffffff || (int64_t)ns * nb > 0x7ffffffe) return hipErrorInvalidConfiguration;
    q.ns = (int)ns;
    q.nb = (int)nb;
    const int64_t count = ns * nb;
    const int64_t sblk = (count + 1023) / 1024;
    int32_t* cnt = nullptr;
    int32_t* sums = nullptr;
    int32_t* nu = nullptr;
    auto cleanup = [&]() {
        if (cnt) hipFree(cnt);
        if (sums) hipFree(sums);
        if (nu) hipFree(nu);
        q.release();
    };
    hipError_t e = hipMalloc(&q.rb, (size_t)(nb + 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&q.off, (size_t)(count + 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&cnt, (size_t)count * 4);
    if (e == hipSuccess) e = hipMalloc(&sums, (size_t)(sblk + 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&q.unit_ptr, ((size_t)p.n + 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&nu, (size_t)p.n * 4);
    if (e != hipSuccess) {
        cleanup();
        return e;
    }
    hipLaunchKernelGGL(k_xs_blocks, dim3((unsigned)((nb + 256) / 256)), dim3(256), 0, s, p.n,
                       (int)nb, p.row_ptr, q.rb);
    hipLaunchKernelGGL(k_xs_count, dim3((unsigned)nb), dim3(256), 0, s, (int)nb, (int)ns, swl,
                       p.row_ptr, col, q.rb, cnt);
    hipLaunchKernelGGL(k_xs_scan_block, dim3((unsigned)sblk), dim3(1024), 0, s, count, cnt, q.off,
                       sums);
    hipLaunchKernelGGL(k_xs_scan_top, dim3(1), dim3(1024), 0, s, (int)sblk, sums, sums + sblk);
    hipLaunchKernelGGL(k_xs_scan_add, dim3((unsigned)sblk), dim3(1024), 0, s, count, q.off, sums,
                       sums + sblk);
    // units: counts per row, scanned into unit_ptr
    const int64_t rblk = ((int64_t)p.n + 1023) / 1024;
    hipLaunchKernelGGL(k_xs_unit_counts, dim3((unsigned)rblk), dim3(1024), 0, s, p.n, p.row_ptr, nu);
    e = hipGetLastError();
    hipFree(sums);
    sums = nullptr;
    if (e == hipSuccess) e = hipMalloc(&sums, (size_t)(rblk + 1) * 4);
    if (e != hipSuccess) {
        cleanup();
        return e;
    }
    hipLaunchKernelGGL(k_xs_scan_block, dim3((unsigned)rblk), dim3(1024), 0, s, (int64_t)p.n, nu,
                       q.unit_ptr, sums);
    hipLaunchKernelGGL(k_xs_scan_top, dim3(1), dim3(1024), 0, s, (int)rblk, sums, sums + rblk);
    hipLaunchKernelGGL(k_xs_scan_add, dim3((unsigned)rblk), dim3(1024), 0, s, (int64_t)p.n,
                       q.unit_ptr, sums, sums + rblk);
    e = hipGetLastError();
    int32_t units = 0, places = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&units, q.unit_ptr + p.n, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&places, q.off + count, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        cleanup();
        return e;
    }
    q.units = units;
    q.places = places;
    // chunks of the products pass: slice s takes ceil(places_s / chunk) of them
    std::vector<int32_t> offs((size_t)ns + 1);
    for (int64_t t = 0; t <= ns && e == hipSuccess; ++t)
        e = hipMemcpyAsync(&offs[t], q.off + t * nb, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    std::vector<int32_t> first((size_t)ns + 1, 0);
    for (int64_t t = 0; t < ns; ++t) {
        const int64_t len = offs[t + 1] - offs[t];
        first[t + 1] = first[t] + (int32_t)std::max<int64_t>(1, (len + kProdChunk - 1) / kProdChunk);
    }
    q.chunks = first[ns];
    if (e == hipSuccess) e = hipMalloc(&q.chunk_first, ((size_t)ns + 1) * 4);
    if (e == hipSuccess)
        e = hipMemcpy(q.chunk_first, first.data(), ((size_t)ns + 1) * 4, hipMemcpyHostToDevice);
    const size_t pl = (size_t)std::max<int64_t>(places, 1);
    if (e == hipSuccess) e = hipMalloc(&q.bcol, pl * 2);
    if (e == hipSuccess) e = hipMalloc(&q.bk, pl * 2);
    if (e == hipSuccess) e = hipMalloc(&q.uinfo, (size_t)std::max<int64_t>(units, 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&q.bval, pl * 8);
    if (e == hipSuccess) e = hipMalloc(&q.prod, pl * 8);
    if (e != hipSuccess) {
        cleanup();
        return e;
    }
    hipLaunchKernelGGL(k_xs_place, dim3((unsigned)nb), dim3(64), 0, s, (int)nb, (int)ns, swl,
                       p.row_ptr, col, q.rb, q.off, (int64_t)places, q.bcol, q.bk);
    hipLaunchKernelGGL(k_xs_units, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, s, p.n,
                       p.row_ptr, q.unit_ptr, q.rb, (int64_t)units, q.uinfo);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(cnt);
    hipFree(nu);
    cnt = nu = nullptr;
    if (e != hipSuccess) {
        cleanup();
        return e;
    }
    p.xs.push_back(q);
    return hipSuccess;
}

hipError_t spmv_xslice(const ao_variant& v, SpmvPlan& p, const double* val, const double* x,
                       double* y, hipStream_t s, const SpmvEpi& ep, bool values_ready) {
    const int swl = v.by == 0 ? 14 : v.by;
    SpmvPlan::XSlice* q = nullptr;
    for (auto& c : p.xs)
        if (c.swl == swl) q = &c;
    if (p.n <= 0) return hipSuccess;
    // no plan: the matrix is one the family does not take (the runtime
    // prepares a plan for every other matrix)
    if (!q) return hipErrorInvalidConfiguration;
    const unsigned rgrid = (unsigned)(8 * ((q->nb + 7) / 8));
    if (!values_ready && q->places > 0) {
        hipLaunchKernelGGL(k_xs_permute, dim3(rgrid), dim3(kRedThreads), 0, s, q->nb, q->ns,
                           q->places, p.row_ptr, q->rb, q->off, q->bk, val, q->bval);
    }
    if (q->places > 0) {
        if (swl == 14)
            hipLaunchKernelGGL(k_xs_products<14>, dim3((unsigned)q->chunks), dim3(kProdThreads), 0,
                               s, q->ncols, q->ns, q->nb, q->off, q->chunk_first, q->bcol, q->bval,
                               x, q->prod);
        else
            hipLaunchKernelGGL(k_xs_products<13>, dim3((unsigned)q->chunks), dim3(kProdThreads), 0,
                               s, q->ncols, q->ns, q->nb, q->off, q->chunk_first, q->bcol, q->bval,
                               x, q->prod);
    }
    hipLaunchKernelGGL(k_xs_reduce, dim3(rgrid), dim3(kRedThreads), 0, s, p.n, q->nb, q->ns,
                       (int64_t)std::max<int64_t>(q->places, 1), p.row_ptr, q->rb, q->off, q->bk, q->prod, q->unit_ptr, q->uinfo, x, y, ep);
    return hipGetLastError();
}

void SpmvPlan::XSlice::release() {
    if (rb) hipFree(rb);
    if (off) hipFree(off);
    if (unit_ptr) hipFree(unit_ptr);
    if (chunk_first) hipFree(chunk_first);
    if (bcol) hipFree(bcol);
    if (bk) hipFree(bk);
    if (uinfo) hipFree(uinfo);
    if (bval) hipFree(bval);
    if (prod) hipFree(prod);
    rb = off = unit_ptr = chunk_first = nullptr;
    bcol = bk = nullptr;
    uinfo = nullptr;
    bval = prod = nullptr;
}

}  // namespace ao
