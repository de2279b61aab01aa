// FP32 MLP cost model 6 -> 64 -> 64 -> 12 (ReLU) on gfx950.
//
// The paper's runtime trains a depth-2 decision-tree classifier on the
// fastest policy per feature tuple (Sec. 2 Apollo paragraph, Sec. 3.1
// model_type, Sec. 4); this library predicts ln(time) of every variant
// instead and selects the argmin.
//
// Dense layers run on the matrix cores: v_mfma_f32_16x16x4_f32, one 16x16
// output tile per wave at a time, operands read from LDS.  Lane layout of
// that instruction (wave64): A[i][k] comes from lane i + 16k, B[k][j] from
// lane j + 16k, and D[i][j] lands in lane j + 16*(i/4), element i%4.
//
// Parameters are one flat array (W1 64x6, b1, W2 64x64, b2, W3 12x64, b3,
// row-major [out][in]), kept in LDS.  A workgroup of 256 threads (4 waves)
// processes samples in chunks of 64.  Weight gradients are accumulated in
// the registers of the lanes that own the corresponding MFMA output element
// across the chunks of a mini-batch, so Adam updates each parameter in
// place without a gradient buffer.
#include "internal.h"

namespace ao {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kIn = 6, kH = 64, kOut = 12;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH,
              oW3 = oB2 + kH, oB3 = oW3 + kOut * kH, kParams = oB3 + kOut;
static_assert(kParams == AO_MLP_PARAMS, "parameter layout");
constexpr int kChunk = 64;
constexpr int kThreads = 256;

struct Smem {
    float p[kParams];
    float X[kChunk * kIn];
    float H1[kChunk * kH];  // activations; later dZ1 in place
    float H2[kChunk * kH];  // activations; later dZ2 in place
    float dO[kChunk * kOut];
    float y[kChunk];
    int var[kChunk];
    float red[kThreads / 64];
};

// One 16x16 tile D = sum_k A(m0 + i, k) * B(k, n0 + j), K a multiple of 4.
template <class FA, class FB>
__device__ __forceinline__ v4f mfma_tile(FA A, FB B, int m0, int n0, int K) {
    const int l = (int)(threadIdx.x & 63);
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 4) {
        const float a = A(m0 + (l & 15), k0 + (l >> 4));
        const float b = B(k0 + (l >> 4), n0 + (l & 15));
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    return acc;
}

__device__ __forceinline__ int lane_row(int r) { return 4 * ((int)(threadIdx.x & 63) >> 4) + r; }
__device__ __forceinline__ int lane_col() { return (int)(threadIdx.x & 15); }

// Forward of one chunk: X -> H1 -> H2 (in LDS); returns nothing, the output
// layer is evaluated by the caller-specific epilogue.
__device__ void forward_hidden(Smem& s) {
    const int w = (int)(threadIdx.x >> 6);
    const float* W1 = s.p + oW1;
    const float* W2 = s.p + oW2;
    for (int t = w; t < 16; t += 4) {
        const int m0 = 16 * (t >> 2), n0 = 16 * (t & 3);
        v4f acc = mfma_tile([&](int b, int k) { return k < kIn ? s.X[b * kIn + k] : 0.0f; },
                            [&](int k, int o) { return k < kIn ? W1[o * kIn + k] : 0.0f; }, m0, n0,
                            8);
        const int o = n0 + lane_col();
        for (int r = 0; r < 4; ++r) {
            const int b = m0 + lane_row(r);
            s.H1[b * kH + o] = fmaxf(acc[r] + s.p[oB1 + o], 0.0f);
        }
    }
    __syncthreads();
    for (int t = w; t < 16; t += 4) {
        const int m0 = 16 * (t >> 2), n0 = 16 * (t & 3);
        v4f acc = mfma_tile([&](int b, int k) { return s.H1[b * kH + k]; },
                            [&](int k, int o) { return W2[o * kH + k]; }, m0, n0, kH);
        const int o = n0 + lane_col();
        for (int r = 0; r < 4; ++r) {
            const int b = m0 + lane_row(r);
            s.H2[b * kH + o] = fmaxf(acc[r] + s.p[oB2 + o], 0.0f);
        }
    }
    __syncthreads();
}

// Output layer tile of wave w (rows 16w..16w+15 of the chunk, 16 columns of
// which 12 are outputs).
__device__ __forceinline__ v4f output_tile(Smem& s) {
    const int w = (int)(threadIdx.x >> 6);
    const float* W3 = s.p + oW3;
    return mfma_tile([&](int b, int k) { return s.H2[b * kH + k]; },
                     [&](int k, int v) { return v < kOut ? W3[v * kH + k] : 0.0f; }, 16 * w, 0,
                     kH);
}

// Gradient accumulators owned by one lane.
struct Grad {
    v4f w1;     // W1 rows 16w + lane_row(r), column lane_col() (< 6 valid)
    v4f w2[4];  // W2 tiles t = w, w+4, w+8, w+12
    v4f w3;     // W3 rows lane_row(r) (< 12 valid), columns 16w + lane_col()
    float bias; // threads 0..63: b1, 64..127: b2, 128..139: b3
    __device__ void zero() {
        w1 = v4f{0, 0, 0, 0};
        for (int t = 0; t < 4; ++t) w2[t] = v4f{0, 0, 0, 0};
        w3 = v4f{0, 0, 0, 0};
        bias = 0.0f;
    }
};

// Backward of one chunk whose dO is in LDS; accumulates into g.
__device__ void backward_chunk(Smem& s, Grad& g) {
    const int w = (int)(threadIdx.x >> 6);
    const int tid = (int)threadIdx.x;
    const float* W2 = s.p + oW2;
    const float* W3 = s.p + oW3;
    // dW3 += dO^T H2 ; db3
    g.w3 += mfma_tile([&](int v, int b) { return v < kOut ? s.dO[b * kOut + v] : 0.0f; },
                      [&](int b, int h) { return s.H2[b * kH + h]; }, 0, 16 * w, kChunk);
    if (tid >= 128 && tid < 128 + kOut) {
        float acc = 0.0f;
        for (int b = 0; b < kChunk; ++b) acc += s.dO[b * kOut + (tid - 128)];
        g.bias += acc;
    }
    __syncthreads();
    // dZ2 = (dO W3) * [H2 > 0], in place of H2
    for (int t = w; t < 16; t += 4) {
        const int m0 = 16 * (t >> 2), n0 = 16 * (t & 3);
        v4f acc = mfma_tile([&](int b, int v) { return v < kOut ? s.dO[b * kOut + v] : 0.0f; },
                            [&](int v, int h) { return v < kOut ? W3[v * kH + h] : 0.0f; }, m0,
                            n0, 16);
        const int h = n0 + lane_col();
        for (int r = 0; r < 4; ++r) {
            const int b = m0 + lane_row(r);
            float* p = &s.H2[b * kH + h];
            *p = (*p > 0.0f) ? acc[r] : 0.0f;
        }
    }
    __syncthreads();
    // dW2 += dZ2^T H1 ; db2
    for (int q = 0; q < 4; ++q) {
        const int t = w + 4 * q;
        const int m0 = 16 * (t >> 2), n0 = 16 * (t & 3);
        g.w2[q] += mfma_tile([&](int o, int b) { return s.H2[b * kH + o]; },
                             [&](int b, int i) { return s.H1[b * kH + i]; }, m0, n0, kChunk);
    }
    if (tid >= 64 && tid < 128) {
        float acc = 0.0f;
        for (int b = 0; b < kChunk; ++b) acc += s.H2[b * kH + (tid - 64)];
        g.bias += acc;
    }
    __syncthreads();
    // dZ1 = (dZ2 W2) * [H1 > 0], in place of H1
    for (int t = w; t < 16; t += 4) {
        const int m0 = 16 * (t >> 2), n0 = 16 * (t & 3);
        v4f acc = mfma_tile([&](int b, int o) { return s.H2[b * kH + o]; },
                            [&](int o, int i) { return W2[o * kH + i]; }, m0, n0, kH);
        const int i = n0 + lane_col();
        for (int r = 0; r < 4; ++r) {
            const int b = m0 + lane_row(r);
            float* p = &s.H1[b * kH + i];
            *p = (*p > 0.0f) ? acc[r] : 0.0f;
        }
    }
    __syncthreads();
    // dW1 += dZ1^T X ; db1
    g.w1 += mfma_tile([&](int o, int b) { return s.H1[b * kH + o]; },
                      [&](int b, int f) { return f < kIn ? s.X[b * kIn + f] : 0.0f; }, 16 * w, 0,
                      kChunk);
    if (tid < 64) {
        float acc = 0.0f;
        for (int b = 0; b < kChunk; ++b) acc += s.H1[b * kH + tid];
        g.bias += acc;
    }
    __syncthreads();
}

// Visit every parameter owned by this lane: fn(param index, gradient value).
template <class F>
__device__ __forceinline__ void for_owned(const Grad& g, F fn) {
    const int w = (int)(threadIdx.x >> 6);
    const int tid = (int)threadIdx.x;
    const int c = lane_col();
    for (int r = 0; r < 4; ++r) {
        const int o = 16 * w + lane_row(r);
        if (c < kIn) fn(oW1 + o * kIn + c, g.w1[r]);
    }
    for (int q = 0; q < 4; ++q) {
        const int t = w + 4 * q;
        const int m0 = 16 * (t >> 2), n0 = 16 * (t & 3);
        for (int r = 0; r < 4; ++r) fn(oW2 + (m0 + lane_row(r)) * kH + n0 + c, g.w2[q][r]);
    }
    for (int r = 0; r < 4; ++r) {
        const int v = lane_row(r);
        if (v < kOut) fn(oW3 + v * kH + 16 * w + c, g.w3[r]);
    }
    if (tid < 64) fn(oB1 + tid, g.bias);
    else if (tid < 128) fn(oB2 + tid - 64, g.bias);
    else if (tid < 128 + kOut) fn(oB3 + tid - 128, g.bias);
}

// Output epilogue for training: dO = mask * (o - y) * invB; returns this
// lane's share of sum 0.5 (o - y)^2 over valid rows.
__device__ float output_grad(Smem& s, int cnt, float invB) {
    const int w = (int)(threadIdx.x >> 6);
    v4f acc = output_tile(s);
    const int v = lane_col();
    float l2 = 0.0f;
    for (int r = 0; r < 4; ++r) {
        const int b = 16 * w + lane_row(r);
        if (v < kOut) {
            float d = 0.0f;
            if (b < cnt && v == s.var[b]) {
                const float diff = acc[r] + s.p[oB3 + v] - s.y[b];
                d = diff * invB;
                l2 += 0.5f * diff * diff;
            }
            s.dO[b * kOut + v] = d;
        }
    }
    __syncthreads();
    return l2;
}

__device__ float block_sum(Smem& s, float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s.red[threadIdx.x >> 6] = v;
    __syncthreads();
    float t = 0.0f;
    for (int i = 0; i < kThreads / 64; ++i) t += s.red[i];
    return t;
}

__device__ void load_params(Smem& s, const float* params) {
    for (int i = (int)threadIdx.x; i < kParams; i += kThreads) s.p[i] = params[i];
}

// Load chunk rows [0, cnt) via a row-index function; zero the rest.
template <class RowF>
__device__ void load_chunk(Smem& s, const float* X, const float* Y, const int32_t* var,
                           const float* mask, int cnt, RowF row) {
    for (int i = (int)threadIdx.x; i < kChunk * kIn; i += kThreads) {
        const int b = i / kIn, f = i % kIn;
        s.X[i] = b < cnt ? X[(size_t)row(b) * kIn + f] : 0.0f;
    }
    for (int b = (int)threadIdx.x; b < kChunk; b += kThreads) {
        if (b < cnt) {
            const int rb = row(b);
            s.y[b] = Y[rb];
            int v = -1;
            if (var) {
                v = var[rb];
            } else {
                for (int q = 0; q < kOut; ++q)
                    if (mask[(size_t)rb * kOut + q] != 0.0f) v = q;
            }
            s.var[b] = v;
        } else {
            s.y[b] = 0.0f;
            s.var[b] = -1;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void adam_update(float* p, float* m, float* v, int idx, float grad,
                                            float lr, float c1, float c2) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mm = b1 * m[idx] + (1.0f - b1) * grad;
    const float vv = b2 * v[idx] + (1.0f - b2) * grad * grad;
    m[idx] = mm;
    v[idx] = vv;
    p[idx] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// -------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_forward(const float* __restrict__ params,
                                                      const float* __restrict__ X, int batch,
                                                      float* __restrict__ out) {
    __shared__ Smem s;
    load_params(s, params);
    const int base = (int)blockIdx.x * kChunk;
    const int cnt = min(kChunk, batch - base);
    for (int i = (int)threadIdx.x; i < kChunk * kIn; i += kThreads) {
        const int b = i / kIn;
        s.X[i] = b < cnt ? X[(size_t)(base + b) * kIn + i % kIn] : 0.0f;
    }
    __syncthreads();
    forward_hidden(s);
    v4f acc = output_tile(s);
    const int w = (int)(threadIdx.x >> 6), v = lane_col();
    for (int r = 0; r < 4; ++r) {
        const int b = 16 * w + lane_row(r);
        if (v < kOut && b < cnt) out[(size_t)(base + b) * kOut + v] = acc[r] + s.p[oB3 + v];
    }
}

__global__ __launch_bounds__(kThreads) void k_grad(const float* __restrict__ params,
                                                   const float* __restrict__ X,
                                                   const float* __restrict__ Y,
                                                   const float* __restrict__ mask, int batch,
                                                   float* __restrict__ grad,
                                                   float* __restrict__ loss) {
    __shared__ Smem s;
    load_params(s, params);
    Grad g;
    g.zero();
    const float invB = 1.0f / (float)batch;
    float l2 = 0.0f;
    for (int c0 = 0; c0 < batch; c0 += kChunk) {
        const int cnt = min(kChunk, batch - c0);
        load_chunk(s, X, Y, nullptr, mask, cnt, [&](int b) { return c0 + b; });
        forward_hidden(s);
        l2 += output_grad(s, cnt, invB);
        backward_chunk(s, g);
    }
    for_owned(g, [&](int idx, float v) { grad[idx] = v; });
    const float tot = block_sum(s, l2);
    if (threadIdx.x == 0 && loss) *loss = tot * invB;
}

__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float c1, float c2) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < kParams) adam_update(p, m, v, i, g[i], lr, c1, c2);
}

// The whole training run: one workgroup, all epochs and mini-batches.
__global__ __launch_bounds__(kThreads) void k_train(float* __restrict__ params,
                                                    const float* __restrict__ X,
                                                    const float* __restrict__ Y,
                                                    const int32_t* __restrict__ var,
                                                    const int32_t* __restrict__ perm, int n,
                                                    int epochs, int batch, float lr,
                                                    float* __restrict__ mv,
                                                    float* __restrict__ epoch_loss) {
    __shared__ Smem s;
    load_params(s, params);
    __syncthreads();
    float* m = mv;
    float* v = mv + kParams;
    double pw1 = 1.0, pw2 = 1.0;
    for (int e = 0; e < epochs; ++e) {
        const int32_t* pe = perm + (size_t)e * n;
        float l2 = 0.0f;
        for (int b0 = 0; b0 < n; b0 += batch) {
            const int cur = min(batch, n - b0);
            const float invB = 1.0f / (float)cur;
            Grad g;
            g.zero();
            for (int c0 = 0; c0 < cur; c0 += kChunk) {
                const int cnt = min(kChunk, cur - c0);
                load_chunk(s, X, Y, var, nullptr, cnt, [&](int b) { return pe[b0 + c0 + b]; });
                forward_hidden(s);
                l2 += output_grad(s, cnt, invB);
                backward_chunk(s, g);
            }
            pw1 *= 0.9;
            pw2 *= 0.999;
            const float c1 = (float)(1.0 - pw1), c2 = (float)(1.0 - pw2);
            for_owned(g, [&](int idx, float gv) { adam_update(s.p, m, v, idx, gv, lr, c1, c2); });
            __syncthreads();
        }
        const float tot = block_sum(s, l2);
        if (threadIdx.x == 0) epoch_loss[e] = tot / (float)n;
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < kParams; i += kThreads) params[i] = s.p[i];
}

// Inference: raw features -> normalised -> forward -> argmin over allowed.
__global__ __launch_bounds__(kThreads) void k_select(const float* __restrict__ params,
                                                     const MlpNorm* __restrict__ norm,
                                                     const float* __restrict__ feats, int batch,
                                                     int nv, int allowed,
                                                     int32_t* __restrict__ ids,
                                                     float* __restrict__ pred) {
    __shared__ Smem s;
    __shared__ float O[kChunk * 16];
    load_params(s, params);
    const int base = (int)blockIdx.x * kChunk;
    const int cnt = min(kChunk, batch - base);
    for (int i = (int)threadIdx.x; i < kChunk * kIn; i += kThreads) {
        const int b = i / kIn, f = i % kIn;
        s.X[i] = b < cnt ? (feats[(size_t)(base + b) * AO_MAX_FEATURES + f] - norm->mu[f]) /
                               norm->sd[f]
                         : 0.0f;
    }
    __syncthreads();
    forward_hidden(s);
    v4f acc = output_tile(s);
    const int w = (int)(threadIdx.x >> 6), v = lane_col();
    for (int r = 0; r < 4; ++r) {
        const int b = 16 * w + lane_row(r);
        O[b * 16 + v] = v < kOut ? acc[r] + s.p[oB3 + v] : 0.0f;
    }
    __syncthreads();
    const int b = (int)threadIdx.x;
    if (b < cnt) {
        int best = -1;
        bool finite = true;
        for (int q = 0; q < nv; ++q) {
            const float o = O[b * 16 + q];
            if (!isfinite(o)) finite = false;
            if (!((allowed >> q) & 1)) continue;
            if (best < 0 || o < O[b * 16 + best]) best = q;
        }
        ids[base + b] = finite ? best : -1;
        if (pred)
            for (int q = 0; q < kOut; ++q) pred[(size_t)(base + b) * kOut + q] = O[b * 16 + q];
    }
}

}  // namespace

hipError_t mlp_forward(const float* params, const float* x, int batch, float* out, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_forward, dim3((batch + kChunk - 1) / kChunk), dim3(kThreads), 0, s,
                       params, x, batch, out);
    return hipGetLastError();
}

hipError_t mlp_grad(const float* params, const float* x, const float* y, const float* mask,
                    int batch, float* grad, float* loss, hipStream_t s) {
    if (batch <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_grad, dim3(1), dim3(kThreads), 0, s, params, x, y, mask, batch, grad,
                       loss);
    return hipGetLastError();
}

hipError_t mlp_adam(float* params, float* m, float* v, const float* grad, int t, float lr,
                    hipStream_t s) {
    if (t < 1) return hipErrorInvalidValue;
    const float c1 = (float)(1.0 - pow(0.9, t)), c2 = (float)(1.0 - pow(0.999, t));
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, params, m, v, grad,
                       lr, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_train_launch(float* params, const float* x, const float* y, const int32_t* var,
                            const int32_t* perm, int n, int epochs, int batch, float lr,
                            float* mv, float* epoch_loss, hipStream_t s) {
    if (n <= 0 || epochs <= 0 || batch <= 0) return hipErrorInvalidValue;
    hipError_t e = hipMemsetAsync(mv, 0, sizeof(float) * 2 * kParams, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_train, dim3(1), dim3(kThreads), 0, s, params, x, y, var, perm, n, epochs,
                       batch, lr, mv, epoch_loss);
    return hipGetLastError();
}

hipError_t mlp_select_launch(const float* params, const MlpNorm* norm, const float* feats,
                             int batch, int num_variants, int allowed_mask, int32_t* ids,
                             float* pred, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3((batch + kChunk - 1) / kChunk), dim3(kThreads), 0, s,
                       params, norm, feats, batch, num_variants, allowed_mask, ids, pred);
    return hipGetLastError();
}

}  // namespace ao
