// SpMV family with x gathered from LDS (gfx950, wave64): x-slice SpMV.
//
// A gather-per-nonzero SpMV over a random sparsity pattern is bound by the
// gathers themselves: each one pulls a 128-byte line of x into L2 from the
// Infinity Cache.  This family makes every gather an LDS read instead.
// Columns are cut into slices of SW = 2^sw columns (8K or 16K: 64 or 128 KB
// of x), rows into blocks of at most DN = 4096 cost units (one per nonzero
// and one per row), a block whose last row would carry it past SPEC = 4096
// nonzeros being split before that row (so a block holds at most 4096
// nonzeros, or a single row of at most DCAP = 4608; longer rows are
// refused).  A per-matrix plan orders the nonzeros slice by slice (slice
// outer, then block, then CSR order) and keeps, per place, the column
// inside its slice, and per element slot of a block (a fixed stride of
// DCAP slots) the element's place and its position inside the block.  One
// execution:
//
//   permute   (only when the values changed) the values into that order;
//   products  one workgroup per chunk of a slice loads the slice of x into
//             LDS and forms fl(val * x[col]) for its places, streaming;
//   reduce    one 512-thread workgroup per row block (four per CU) scatters
//             the block's products from their slice pieces into LDS at
//             their CSR positions, sums every row-aligned 64-leaf unit by
//             the canonical tree (one thread per unit), then combines the
//             unit sums of longer rows by the same tree, and stores y (or
//             the relaxation update).
//
// The products are the same rounded products and the tree is the same
// aligned pairwise tree (absent leaves as -0.0, the exact additive
// identity) as in every other family, so the result is bit-identical.
#include "internal.h"

namespace ao {
namespace {

constexpr int kDN = 4096;      // cost units (nonzeros + rows) per cost block
constexpr int kSpec = 4096;    // nonzeros of a row block of several rows
constexpr int kDCAP = 4608;    // nonzeros a row block can hold in LDS (a single long row)
constexpr int kMaxSlices = 1024;
constexpr int kRedThreads = 512;  // 4 reduce workgroups (32 KB of LDS each) per CU
constexpr int kProdThreads = 1024;
constexpr int kProdChunk = 65536;  // places per products workgroup (target)

typedef unsigned short us4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// ---- plan ----------------------------------------------------------------

// Cost blocks: rb[t] = first row i whose cost (row_ptr[i] - row_ptr[0]) + i
// is >= t * DN (the cost is strictly increasing in i); rb[nb] = n
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

// Row blocks from cost blocks: a cost block [a, b) holds fewer than DN cost
// units before its last row b - 1, so fewer than SPEC nonzeros there; when
// the whole block holds more than SPEC nonzeros its last row becomes a block
// of its own (at most DCAP nonzeros: longer rows are refused).  cnt[t] = 1
// or 2 row blocks of cost block t.
__global__ void k_xs_split_count(int nbc, const int32_t* __restrict__ row_ptr,
                                 const int32_t* __restrict__ rbc, int32_t* __restrict__ cnt) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= nbc) return;
    const int32_t a = rbc[t], b = rbc[t + 1];
    cnt[t] = (b > a + 1 && row_ptr[b] - row_ptr[a] > kSpec) ? 2 : 1;
}

// rb (nb + 1 entries) from the cost blocks and the exclusive scan pos of cnt
__global__ void k_xs_split_write(int nbc, int n, int nb, const int32_t* __restrict__ rbc,
                                 const int32_t* __restrict__ cnt,
                                 const int32_t* __restrict__ pos, int32_t* __restrict__ rb) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t > nbc) return;
    if (t == nbc) {
        rb[nb] = n;
        return;
    }
    rb[pos[t]] = rbc[t];
    if (cnt[t] == 2) rb[pos[t] + 1] = rbc[t + 1] - 1;
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

// first place of each slice: starts[s] = off[s * nb]
__global__ __launch_bounds__(256) void k_xs_slice_starts(int nb, int ns,
                                                         const int32_t* __restrict__ off,
                                                         int32_t* __restrict__ starts) {
    const int q = (int)(blockIdx.x * 256 + threadIdx.x);
    if (q < ns) starts[q] = off[(int64_t)q * nb];
}

// Places (one wave per block): the block's nonzeros in CSR order, 64 at a
// time; a lane's place is its slice's cursor plus the number of earlier
// lanes of the chunk in the same slice, so each piece keeps CSR order.
// The block's elements are its places in place order (its pieces one
// after the other): element e of block t sits at index t * DCAP + e of the
// element arrays (a fixed stride, so a workgroup can request its elements
// before it knows how many there are; unused slots hold zeros), which hold
// its place (ej) and its nonzero's index inside the block (bke, the LDS
// slot it is summed in).
__global__ __launch_bounds__(64) void k_xs_place(int nb, int ns, int sw,
                                                 const int32_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col,
                                                 const int32_t* __restrict__ rb,
                                                 const int32_t* __restrict__ off, int64_t places,
                                                 uint16_t* __restrict__ bcol,
                                                 int32_t* __restrict__ ej,
                                                 uint16_t* __restrict__ bke) {
    __shared__ int32_t cur[kMaxSlices];
    __shared__ int32_t ebase[kMaxSlices];  // element index of each piece's first place
    const int t = (int)blockIdx.x;
    const int lane = (int)threadIdx.x;
    int32_t carry = 0;
    for (int base = 0; base < ns; base += 64) {
        const int s = base + lane;
        int32_t len = 0;
        if (s < ns) {
            const int64_t q = (int64_t)s * nb + t;
            cur[s] = off[q];
            len = off[q + 1] - off[q];
        }
        int32_t v = len;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t w = __shfl_up(v, d);
            if (lane >= d) v += w;
        }
        if (s < ns) ebase[s] = carry + v - len;
        carry += __shfl(v, 63);
    }
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
        int32_t base = 0, eb = 0, st = 0;
        if (live) {
            base = cur[s];
            eb = ebase[s];
            st = off[(int64_t)s * nb + t];
        }
        __syncthreads();
        if (live) {
            const int64_t j = (int64_t)base + before;
            const int64_t e = (int64_t)eb + (j - st);   // element index inside the block
            const int64_t x = (int64_t)t * kDCAP + e;   // its slot in the element arrays
            if (j >= 0 && j < places) bcol[j] = (uint16_t)(cc - (s << sw));
            if (e >= 0 && e < kDCAP) {
                ej[x] = (int32_t)j;
                bke[x] = (uint16_t)(k - kb);
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

// Unit descriptors, 64 bits each, for the units of row i (its row block t:
// the first row block of cost block cost(i) / DN, or the second when that
// cost block was split and i is its last row): bits 0-15 the unit's first nonzero inside the block, 16-23
// its nonzero count (0..64), 24-31 the row's unit count, 32-47 the row
// inside the block, 48-63 the unit's index in the row.
__device__ __forceinline__ uint64_t unit_desc(int a, int m, int nu, int r, int jn) {
    return (uint64_t)(uint32_t)a | ((uint64_t)(uint32_t)m << 16) | ((uint64_t)(uint32_t)nu << 24) |
           ((uint64_t)(uint32_t)r << 32) | ((uint64_t)(uint32_t)jn << 48);
}

__global__ __launch_bounds__(256) void k_xs_units(int n, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ unit_ptr,
                                                  const int32_t* __restrict__ rb,
                                                  const int32_t* __restrict__ pos,
                                                  int64_t units, uint64_t* __restrict__ uinfo) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int tc = (int)(((int64_t)(row_ptr[i] - row_ptr[0]) + i) / kDN);
    const int t = pos[tc] + (i >= rb[pos[tc] + 1] ? 1 : 0);
    const int r = i - rb[t];
    const int32_t rs = row_ptr[i] - row_ptr[rb[t]];
    const int32_t len = row_ptr[i + 1] - row_ptr[i];
    const int nu = len > 0 ? (len + 63) / 64 : 1;
    const int32_t u0 = unit_ptr[i];
    for (int jn = 0; jn < nu; ++jn) {
        const int64_t u = (int64_t)u0 + jn;
        const int m = min(max(len - 64 * jn, 0), 64);
        if (u >= 0 && u < units) uinfo[u] = unit_desc(rs + 64 * jn, m, nu, r, jn);
    }
}

// per block t: first unit ub[t] = unit_ptr[rb[t]], first nonzero kbt[t] =
// row_ptr[rb[t]] (t = 0..nb)
__global__ __launch_bounds__(256) void k_xs_block_info(int nb, const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ rb,
                                                       const int32_t* __restrict__ unit_ptr,
                                                       int32_t* __restrict__ ub,
                                                       int32_t* __restrict__ kbt) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t > nb) return;
    ub[t] = unit_ptr[rb[t]];
    kbt[t] = row_ptr[rb[t]];
}

// ---- execution -----------------------------------------------------------

// XCD-aware order: consecutive blocks on one XCD (round-robin dispatch puts
// workgroup g on XCD g % 8), so the line shared by the pieces of adjacent
// blocks is fetched into one L2
__device__ __forceinline__ int xcd_block(int g, int nb) {
    const int per = (nb + 7) / 8;
    return (g & 7) * per + (g >> 3);
}

// A row block holds at most DCAP elements; a thread of a kRedThreads-wide
// workgroup takes elements e = thread + q * kRedThreads, q < kPer.
constexpr int kPer = (kDCAP + kRedThreads - 1) / kRedThreads;
constexpr int kSpecPer = kSpec / kRedThreads;
static_assert(kSpecPer * kRedThreads == kSpec && kPer * kRedThreads == kDCAP, "slot tiling");

// The element slots of row block t a thread takes: the first SPEC slots are
// requested at once at the block's fixed offset, before its bounds arrive;
// the rest only when the block's count (`count()`, which may wait on a
// load) says it is a single row longer than SPEC.  Slots past the count
// hold zeros; the caller discards them.  (The slots' 16-bit fields land in
// 32-bit registers of their own: packing two into one register would make
// the code wait for the loads right here.)
template <typename Count>
__device__ __forceinline__ void load_elements(int t, const int32_t* __restrict__ ej,
                                              const uint16_t* __restrict__ bke, int32_t* j,
                                              int32_t* b, Count count) {
    const int64_t xt = (int64_t)t * kDCAP + threadIdx.x;
#pragma unroll
    for (int q = 0; q < kSpecPer; ++q) {
        j[q] = ej[xt + q * kRedThreads];
        b[q] = bke[xt + q * kRedThreads];
    }
    if (count() > kSpec) {  // workgroup-uniform
#pragma unroll
        for (int q = kSpecPer; q < kPer; ++q) {
            j[q] = ej[xt + q * kRedThreads];
            b[q] = bke[xt + q * kRedThreads];
        }
    } else {
#pragma unroll
        for (int q = kSpecPer; q < kPer; ++q) {
            j[q] = 0;
            b[q] = 0;
        }
    }
}

// bval[ej[x]] = val[kb + bke[x]] over the elements x of each row block
// (workgroup per row block; its first SPEC element slots are requested
// before its bounds)
__global__ __launch_bounds__(kRedThreads) void k_xs_permute(int nb, int64_t places,
                                                            const int32_t* __restrict__ kbt,
                                                            const int32_t* __restrict__ ej,
                                                            const uint16_t* __restrict__ bke,
                                                            const double* __restrict__ val,
                                                            double* __restrict__ bval) {
    const int t = xcd_block((int)blockIdx.x, nb);
    if (t >= nb) return;
    int32_t j[kPer], b[kPer];
    load_elements(t, ej, bke, j, b, [&]() { return kbt[t + 1] - kbt[t]; });
    const int32_t kb = kbt[t], kend = kbt[nb];
    const int total = min(kbt[t + 1] - kb, kDCAP);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int e = (int)threadIdx.x + q * kRedThreads;
        j[q] = e < total ? min(max(j[q], 0), (int32_t)(places - 1)) : -1;
    }
    double v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) v[q] = j[q] >= 0 ? val[min(kb + (int32_t)b[q], kend - 1)] : 0.0;
#pragma unroll
    for (int q = 0; q < kPer; ++q)
        if (j[q] >= 0) bval[j[q]] = v[q];
}

// prod[place] = bval[place] * x[slice base + bcol[place]] over one chunk
// (a range of one slice's places), x of the slice in LDS.  Places go in
// aligned groups of four (8-byte column and 32-byte value and product
// accesses); groups cut by the chunk's ends take the elementwise path.
template <int SWL>
__global__ __launch_bounds__(kProdThreads) void k_xs_products(int64_t ncols,
                                                              const int4* __restrict__ chunks,
                                                              const uint16_t* __restrict__ bcol,
                                                              const double* __restrict__ bval,
                                                              const double* __restrict__ x,
                                                              double* __restrict__ prod) {
    constexpr int SW = 1 << SWL;
    __shared__ double xs[SW];
    const int4 ch = chunks[blockIdx.x];  // slice, first place, end place, unused
    const int64_t base = (int64_t)ch.x << SWL;
    const int w = (int)min((int64_t)SW, ncols - base);
    for (int c = (int)threadIdx.x; c < SW; c += kProdThreads) xs[c] = c < w ? x[base + c] : 0.0;
    __syncthreads();
    const int64_t lo = ch.y, hi = ch.z;
    const int64_t g0 = lo >> 2, g1 = (hi + 3) >> 2;
    // interior groups (all four places inside the chunk) in batches of two
    // per thread, loads first; the (at most two) cut groups elementwise
    const int64_t a = (lo + 3) >> 2, b = hi >> 2;  // groups [a, b) lie inside
    constexpr int G = 2;
    for (int64_t g = a + threadIdx.x; g < b; g += (int64_t)kProdThreads * G) {
        us4 c[G];
        d2 v0[G], v1[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int64_t gg = min(g + (int64_t)u * kProdThreads, b - 1);
            c[u] = __builtin_nontemporal_load(reinterpret_cast<const us4*>(bcol) + gg);
            v0[u] = __builtin_nontemporal_load(reinterpret_cast<const d2*>(bval) + 2 * gg);
            v1[u] = __builtin_nontemporal_load(reinterpret_cast<const d2*>(bval) + 2 * gg + 1);
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int64_t gg = g + (int64_t)u * kProdThreads;
            if (gg < b) {
                d2 p0, p1;
                p0.x = v0[u].x * xs[c[u].x & (SW - 1)];
                p0.y = v0[u].y * xs[c[u].y & (SW - 1)];
                p1.x = v1[u].x * xs[c[u].z & (SW - 1)];
                p1.y = v1[u].y * xs[c[u].w & (SW - 1)];
                __builtin_nontemporal_store(p0, reinterpret_cast<d2*>(prod) + 2 * gg);
                __builtin_nontemporal_store(p1, reinterpret_cast<d2*>(prod) + 2 * gg + 1);
            }
        }
    }
    if (threadIdx.x < 8) {
        // the cut groups at the ends: g0 (if lo is not aligned) and b (if hi is not)
        const int64_t g = threadIdx.x < 4 ? g0 : b;
        const int64_t je = (g << 2) + (threadIdx.x & 3);
        const bool cut = threadIdx.x < 4 ? (g0 < a) : (b < g1 && b >= a);
        if (cut && je >= lo && je < hi) prod[je] = bval[je] * xs[bcol[je] & (SW - 1)];
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

__global__ __launch_bounds__(kRedThreads) void k_xs_reduce(int n, int nb, int64_t places,
                                                           const int32_t* __restrict__ rb,
                                                           const int32_t* __restrict__ ub,
                                                           const int32_t* __restrict__ kbt,
                                                           const int32_t* __restrict__ ej,
                                                           const uint16_t* __restrict__ bke,
                                                           const double* __restrict__ prod,
                                                           const uint64_t* __restrict__ uinfo,
                                                           const double* __restrict__ x,
                                                           double* __restrict__ y, SpmvEpi ep) {
    __shared__ double sl[kDCAP];
    const int t = xcd_block((int)blockIdx.x, nb);
    if (t >= nb) return;
    // everything the block needs that does not depend on its products is
    // requested up front: its elements, its first row and its units
    int32_t j[kPer], b[kPer];
    load_elements(t, ej, bke, j, b, [&]() { return kbt[t + 1] - kbt[t]; });
    const int r0 = rb[t];
    const int32_t u0 = ub[t], u1 = ub[t + 1];
    const int total = min(kbt[t + 1] - kbt[t], kDCAP);
    const int32_t uf = u0 + (int32_t)threadIdx.x;
    const uint64_t first = uf < u1 ? uinfo[uf] : 0;
    {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = (int)threadIdx.x + q * kRedThreads;
            j[q] = e < total ? min(max(j[q], 0), (int32_t)(places - 1)) : -1;
        }
        double v[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) v[q] = j[q] >= 0 ? prod[j[q]] : 0.0;
#pragma unroll
        for (int q = 0; q < kPer; ++q)
            if (j[q] >= 0) sl[min(b[q], kDCAP - 1)] = v[q];
    }
    __syncthreads();
    // one thread per unit: a row of one unit is finished here; the units of
    // longer rows leave their sum in their first nonzero's slot
    for (int32_t u = uf; u < u1; u += kRedThreads) {
        const uint64_t d = u == uf ? first : uinfo[u];
        const int a = (int)(d & 0xffffu), m = (int)((d >> 16) & 0xffu);
        const int nu = (int)((d >> 24) & 0xffu);
        const int i = r0 + (int)((d >> 32) & 0xffffu);
        const bool in_lds = a + m <= kDCAP;
        const double v = in_lds ? unit_sum(sl + a, m) : 0.0;
        if (nu <= 1) {
            if (i < n) y[i] = out_value(ep, x, i, m > 0 ? v : 0.0);
        } else if (in_lds) {
            sl[a] = v;
        }
    }
    __syncthreads();
    // the first unit of each longer row combines the row's unit sums
    for (int32_t u = uf; u < u1; u += kRedThreads) {
        const uint64_t d = u == uf ? first : uinfo[u];
        const int nu = (int)((d >> 24) & 0xffu), jn = (int)(d >> 48);
        if (nu <= 1 || jn != 0) continue;
        const int a = (int)(d & 0xffffu);
        const int i = r0 + (int)((d >> 32) & 0xffffu);
        const bool in_lds = a + 64 * (nu - 1) < kDCAP;
        if (i < n) y[i] = out_value(ep, x, i, in_lds ? combine_units(sl + a, nu) : 0.0);
    }
}

}  // namespace

// Largest row the family takes: a block holds at most DN - 1 cost units
// before its last row starts, plus that row.
int spmv_xslice_max_row() { return kDCAP; }

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
    const int64_t nbc = (cost + kDN - 1) / kDN;  // cost blocks
    if (nbc > 0x3fffffff) return hipErrorInvalidConfiguration;
    // row blocks: the cost blocks, those above DCAP nonzeros split in two
    int32_t* rbc = nullptr;
    int32_t* scnt = nullptr;
    int32_t* spos = nullptr;
    int32_t* ssum = nullptr;
    auto free_split = [&]() {
        if (rbc) hipFree(rbc);
        if (scnt) hipFree(scnt);
        if (spos) hipFree(spos);
        if (ssum) hipFree(ssum);
        rbc = scnt = spos = ssum = nullptr;
    };
    const int64_t cblk = (nbc + 1023) / 1024;
    int32_t nb32 = 0;
    hipError_t es = hipMalloc(&rbc, (size_t)(nbc + 1) * 4);
    if (es == hipSuccess) es = hipMalloc(&scnt, (size_t)nbc * 4);
    if (es == hipSuccess) es = hipMalloc(&spos, (size_t)(nbc + 1) * 4);
    if (es == hipSuccess) es = hipMalloc(&ssum, (size_t)(cblk + 1) * 4);
    if (es == hipSuccess) {
        hipLaunchKernelGGL(k_xs_blocks, dim3((unsigned)((nbc + 256) / 256)), dim3(256), 0, s, p.n,
                           (int)nbc, p.row_ptr, rbc);
        hipLaunchKernelGGL(k_xs_split_count, dim3((unsigned)((nbc + 255) / 256)), dim3(256), 0, s,
                           (int)nbc, p.row_ptr, rbc, scnt);
        hipLaunchKernelGGL(k_xs_scan_block, dim3((unsigned)cblk), dim3(1024), 0, s, nbc, scnt,
                           spos, ssum);
        hipLaunchKernelGGL(k_xs_scan_top, dim3(1), dim3(1024), 0, s, (int)cblk, ssum, ssum + cblk);
        hipLaunchKernelGGL(k_xs_scan_add, dim3((unsigned)cblk), dim3(1024), 0, s, nbc, spos, ssum,
                           ssum + cblk);
        es = hipGetLastError();
    }
    if (es == hipSuccess) es = hipMemcpyAsync(&nb32, spos + nbc, 4, hipMemcpyDeviceToHost, s);
    if (es == hipSuccess) es = hipStreamSynchronize(s);
    if (es != hipSuccess) {
        free_split();
        return es;
    }
    const int64_t nb = nb32;
    if (nb > 0x3fffffff || (int64_t)ns * nb > 0x7ffffffe) {
        free_split();
        return hipErrorInvalidConfiguration;
    }
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
        free_split();
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
    hipLaunchKernelGGL(k_xs_split_write, dim3((unsigned)((nbc + 256) / 256)), dim3(256), 0, s,
                       (int)nbc, p.n, (int)nb, rbc, scnt, spos, q.rb);
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
    // the products pass is cut into chunks: each slice into equal ranges so
    // that the whole pass is a whole number of rounds of the resident
    // workgroups (one per 128 KB slice and CU, two per 64 KB slice)
    std::vector<int32_t> offs((size_t)ns + 1);
    {
        int32_t* starts = nullptr;
        if (e == hipSuccess) e = hipMalloc(&starts, (size_t)ns * 4);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_xs_slice_starts, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0,
                               s, (int)nb, (int)ns, q.off, starts);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(offs.data(), starts, (size_t)ns * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (starts) hipFree(starts);
    }
    offs[ns] = places;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0) {
        (void)hipGetLastError();
        cus = 256;
    }
    const int64_t resident = (int64_t)cus * (swl == 13 ? 2 : 1);
    const int64_t rounds =
        std::max<int64_t>(1, (places + resident * kProdChunk / 2) / (resident * kProdChunk));
    const double per = (double)std::max<int64_t>(places, 1) / (double)(rounds * resident);
    std::vector<int4> chunks;
    for (int64_t t = 0; t < ns; ++t) {
        const int64_t lo = offs[t], hi = offs[t + 1];
        const int64_t k = std::max<int64_t>(1, (int64_t)std::llround((double)(hi - lo) / per));
        for (int64_t c = 0; c < k; ++c) {
            int4 v;
            v.x = (int)t;
            v.y = (int)(lo + (hi - lo) * c / k);
            v.z = (int)(lo + (hi - lo) * (c + 1) / k);
            v.w = 0;
            chunks.push_back(v);
        }
    }
    q.chunks = (int)chunks.size();
    if (e == hipSuccess) e = hipMalloc(&q.chunk_table, chunks.size() * sizeof(int4));
    if (e == hipSuccess)
        e = hipMemcpy(q.chunk_table, chunks.data(), chunks.size() * sizeof(int4),
                      hipMemcpyHostToDevice);
    const size_t pl = (size_t)std::max<int64_t>(places, 1);
    if (e == hipSuccess) e = hipMalloc(&q.bcol, pl * 2);
    const size_t slots = (size_t)nb * kDCAP;  // element slots: DCAP per row block
    if (e == hipSuccess) e = hipMalloc(&q.ej, slots * 4);
    if (e == hipSuccess) e = hipMalloc(&q.bke, slots * 2);
    if (e == hipSuccess) e = hipMemsetAsync(q.ej, 0, slots * 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(q.bke, 0, slots * 2, s);
    if (e == hipSuccess) e = hipMalloc(&q.uinfo, (size_t)std::max<int64_t>(units, 1) * 8);
    if (e == hipSuccess) e = hipMalloc(&q.ub, (size_t)(nb + 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&q.kbt, (size_t)(nb + 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&q.bval, pl * 8);
    if (e == hipSuccess) e = hipMalloc(&q.prod, pl * 8);
    if (e != hipSuccess) {
        cleanup();
        return e;
    }
    hipLaunchKernelGGL(k_xs_place, dim3((unsigned)nb), dim3(64), 0, s, (int)nb, (int)ns, swl,
                       p.row_ptr, col, q.rb, q.off, (int64_t)places, q.bcol, q.ej, q.bke);
    hipLaunchKernelGGL(k_xs_units, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, s, p.n,
                       p.row_ptr, q.unit_ptr, q.rb, spos, (int64_t)units, q.uinfo);
    hipLaunchKernelGGL(k_xs_block_info, dim3((unsigned)((nb + 256) / 256)), dim3(256), 0, s,
                       (int)nb, p.row_ptr, q.rb, q.unit_ptr, q.ub, q.kbt);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(cnt);
    hipFree(nu);
    cnt = nu = nullptr;
    free_split();
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
        hipLaunchKernelGGL(k_xs_permute, dim3(rgrid), dim3(kRedThreads), 0, s, q->nb, q->places,
                           q->kbt, q->ej, q->bke, val, q->bval);
    }
    if (q->places > 0) {
        if (swl == 14)
            hipLaunchKernelGGL(k_xs_products<14>, dim3((unsigned)q->chunks), dim3(kProdThreads), 0,
                               s, q->ncols, q->chunk_table, q->bcol, q->bval, x, q->prod);
        else
            hipLaunchKernelGGL(k_xs_products<13>, dim3((unsigned)q->chunks), dim3(kProdThreads), 0,
                               s, q->ncols, q->chunk_table, q->bcol, q->bval, x, q->prod);
    }
    hipLaunchKernelGGL(k_xs_reduce, dim3(rgrid), dim3(kRedThreads), 0, s, p.n, q->nb,
                       (int64_t)std::max<int64_t>(q->places, 1), q->rb, q->ub, q->kbt, q->ej,
                       q->bke, q->prod, q->uinfo, x, y, ep);
    return hipGetLastError();
}

void SpmvPlan::XSlice::release() {
    if (rb) hipFree(rb);
    if (off) hipFree(off);
    if (unit_ptr) hipFree(unit_ptr);
    if (chunk_table) hipFree(chunk_table);
    if (ej) hipFree(ej);
    if (bke) hipFree(bke);
    if (ub) hipFree(ub);
    if (kbt) hipFree(kbt);
    if (bcol) hipFree(bcol);
    if (uinfo) hipFree(uinfo);
    if (bval) hipFree(bval);
    if (prod) hipFree(prod);
    rb = off = unit_ptr = ub = kbt = ej = nullptr;
    bke = nullptr;
    chunk_table = nullptr;
    bcol = nullptr;
    uinfo = nullptr;
    bval = prod = nullptr;
}

}  // namespace ao
