// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/adaptomp.h"

namespace ao {

// Thread-local error message (ao_last_error).
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

// Launch one Jacobi sweep dst <- J(src) of a GPU variant on `s`.  Checks the
// launch shape on the host first and returns hipErrorInvalidConfiguration
// without launching when it does not fit the kernel.
hipError_t jacobi_gpu_sweep(const ao_variant& v, const double* src, double* dst, int nx, int ny,
                            int nz, hipStream_t s);

// Two sweeps at once (temporal-blocking family): dst <- J(J(src)).
hipError_t jacobi_gpu_double_sweep(const ao_variant& v, const double* src, double* dst, int nx,
                                  int ny, int nz, hipStream_t s);
// Three or four sweeps at once (families ZREG_T3 / ZREG_T4): dst <- J^T(src).
hipError_t jacobi_gpu_multi_sweep(const ao_variant& v, const double* src, double* dst, int nx,
                                 int ny, int nz, hipStream_t s);
// Planes per block of a launch of a register z-march variant (v.bz, or with
// AO_VF_FILL_Z the chunk fill_planes picks) on an nx * ny * nz grid, for
// `cus` CUs holding `per_cu` of its workgroups each (cus <= 0: the kernel's
// residency on the current device); hipErrorInvalidConfiguration for a
// variant that fits no z-march kernel.
hipError_t jacobi_gpu_planes(const ao_variant& v, int nx, int ny, int nz, int cus, int per_cu,
                             int* planes);
// The chunk length, at most bz_max planes, of the fastest launch when
// `columns` columns of blocks are cut into z-chunks and each block marches
// its chunk plus `halo` planes (2(T-1) for T fused sweeps): the blocks
// spread evenly over `cus` CUs, the busiest CU runs n = ceil(blocks / cus)
// of them in rounds of k = per_cu at once and a last round of n mod k, a
// round of j taking (chunk + halo) * j / gain(j) (gain 1, 1.4, 1.5 for 1,
// 2, 3+ at once); the fewest chunks whose cost lies within 3% of the least
// are taken (less halo traffic), cut into equal lengths.
int fill_planes(int64_t columns, int nz, int bz_max, int halo, int cus, int per_cu);
// All `sweeps` sweeps dst <- J^sweeps(src) of a grid of at most 8192 points
// in one launch of one workgroup (the grid held twice in LDS);
// hipErrorInvalidConfiguration for a larger grid.
bool lds_sweeps_fit(int nx, int ny, int nz);
hipError_t jacobi_gpu_lds_sweeps(const double* src, double* dst, int nx, int ny, int nz,
                                 int sweeps, hipStream_t s);
hipError_t hbm_copy(const double* src, double* dst, int64_t n, bool nt, hipStream_t s);

// Host (OpenMP) variant: S sweeps from u0 into out using tmp (N doubles) as
// the second ping-pong buffer.  All three are host memory.
void jacobi_host_sweeps(const ao_variant& v, const double* u0, double* out, double* tmp, int nx,
                        int ny, int nz, int sweeps);

// SpMV: per-matrix plan (features, merge-path partition) built on the GPU.
struct SpmvPlan {
    uint64_t structure_id = 0;
    const int32_t* row_ptr = nullptr;
    int32_t n = 0;
    int64_t nnz = 0;
    float features[AO_MAX_FEATURES] = {0};
    bool have_features = false;
    int32_t max_len = 0;  // longest row
    // merge-path: row-aligned 64-leaf units and one partition per chunk size
    int32_t* unit_ptr = nullptr;  // [n + 1] first unit of each row
    double* unit_sums = nullptr;  // [units] sums of units of rows split across chunks
    int64_t units = 0;
    struct MergeSplit {
        int D = 0;                  // cost per workgroup
        int blocks = 0;
        int32_t* srow = nullptr;    // [blocks + 1] start row of each workgroup (owns the allocation)
        int32_t* sunit = nullptr;   // [blocks + 1] start unit within that row
    };
    std::vector<MergeSplit> mp;
    // x-slice family: columns cut into slices of 2^swl columns, rows into
    // blocks of at most 4096 cost units (nonzeros + rows); places ordered
    // slice, block, CSR order
    struct XSlice {
        int swl = 0;                    // log2 of the slice width
        int ns = 0, nb = 0;             // slices, row blocks
        int64_t ncols = 0;              // columns (largest index + 1)
        int32_t* rb = nullptr;          // [nb + 1] first row of each block
        int32_t* off = nullptr;         // [ns*nb + 1] first place of piece (slice s, block t) at s*nb+t
        int32_t* unit_ptr = nullptr;    // [n + 1] first 64-leaf unit of each row
        int4* chunk_table = nullptr;    // [chunks] (slice, first place, end place, 0) per products workgroup
        int chunks = 0;
        uint16_t* bcol = nullptr;       // [places] column inside the slice
        int32_t* ej = nullptr;          // [nb * DCAP] per element slot (block t's places in place
                                        // order from t * DCAP; unused slots 0): its place
        uint16_t* bke = nullptr;        // [nb * DCAP] per element slot: its nonzero's index inside
                                        // the block
        uint64_t* uinfo = nullptr;      // [units] unit descriptors (first nonzero and count, the
                                        // row's unit count, row inside the block, index in the row)
        int32_t* ub = nullptr;          // [nb + 1] first unit of each block
        int32_t* kbt = nullptr;         // [nb + 1] first nonzero of each block
        double* bval = nullptr;         // [places] values in place order
        double* prod = nullptr;         // [places] products in place order
        int64_t units = 0, places = 0;
        uint64_t values_id = 0;         // values_id of the values bval holds (0: none)
        const double* values_of = nullptr;  // and the array they came from
        void release();
    };
    std::vector<XSlice> xs;
    ~SpmvPlan();
};
// Build the merge-path partition for workgroups of B threads (synchronises).
hipError_t spmv_prepare_merge(SpmvPlan& p, int B, hipStream_t s);
// Build the x-slice plan for slices of 2^swl columns (synchronises); needs
// the plan's col array and the longest row (features); rows longer than
// spmv_xslice_max_row() nonzeros give hipErrorInvalidConfiguration.
hipError_t spmv_prepare_xslice(SpmvPlan& p, int swl, const int32_t* col, hipStream_t s);
int spmv_xslice_max_row();

hipError_t spmv_features(SpmvPlan& p, hipStream_t s);
// What a finished row i with canonical sum s_i stores: y_i = s_i (b ==
// NULL), or the relaxation update y_i = x_i + (omega * (b_i - s_i)) / d_i.
struct SpmvEpi {
    const double* b = nullptr;
    const double* d = nullptr;
    double omega = 0.0;
};
// values_ready: the x-slice family's copy of val in place order already
// holds this val (the caller knows it: the second and later sweeps of one
// execution, or an unchanged values id); other families ignore it.
hipError_t spmv_xslice(const ao_variant& v, SpmvPlan& p, const double* val, const double* x,
                       double* y, hipStream_t s, const SpmvEpi& ep, bool values_ready);
hipError_t spmv_gpu(const ao_variant& v, SpmvPlan& p, const int32_t* col, const double* val,
                    const double* x, double* y, hipStream_t s, const SpmvEpi& ep = SpmvEpi(),
                    bool values_ready = false);

// Gather probe: out[w] = sum of x[idx[k]] over the entries of wave w
// (idx clamped into [0, nx)); out holds gather_probe_out_len(m) doubles.
int64_t gather_probe_out_len(int64_t m);
hipError_t gather_probe(const int32_t* idx, const double* x, int64_t m, int64_t nx, double* out,
                        hipStream_t s);

// Cost model kernels.
struct MlpNorm {
    float mu[AO_MAX_FEATURES];
    float sd[AO_MAX_FEATURES];
    float y_mean;
};
hipError_t mlp_forward(const float* params, const float* x, int batch, float* out, hipStream_t s);
hipError_t mlp_grad(const float* params, const float* x, const float* y, const float* mask,
                    int batch, float* grad, float* loss, hipStream_t s);
hipError_t mlp_adam(float* params, float* m, float* v, const float* grad, int t, float lr,
                    hipStream_t s);
// Whole training run in one launch: epochs over n samples (x[n*6], y[n],
// variant id[n]) in the order perm[epochs*n]; params updated in place,
// mv = Adam moments scratch (2 * AO_MLP_PARAMS floats, zeroed here),
// epoch_loss[epochs] written.
hipError_t mlp_train_launch(float* params, const float* x, const float* y, const int32_t* var,
                            const int32_t* perm, int n, int epochs, int batch, float lr,
                            float* mv, float* epoch_loss, hipStream_t s);
// Batched inference: raw features feats[batch*6] -> argmin over allowed
// variants (bit v of allowed_mask) of the predicted ln-time, and the
// predictions pred[batch*12] (may be null).
hipError_t mlp_select_launch(const float* params, const MlpNorm* norm, const float* feats,
                             int batch, int num_variants, int allowed_mask, int32_t* ids,
                             float* pred, hipStream_t s);

// Decision-tree classifier (host).
struct DTree {
    struct Node {
        int feature = -1;        // -1: leaf
        double threshold = 0.0;  // f <= threshold goes left
        int left = -1, right = -1;
        std::vector<int> counts;  // class counts of the node's samples
    };
    std::vector<Node> nodes;
    void train(const std::vector<std::vector<float>>& feats, const std::vector<int>& labels,
               int max_depth, int num_classes);
    int predict(const float* f, int allowed_mask) const;  // -1 if no allowed class
};

// Batched Jacobi.
struct BatchItem {
    int32_t inst;        // instance index
    int32_t tx0, ty0, tz0;  // tile origin
};
struct BatchInst {
    const double* u0;
    double* out;
    double* tmp;
    int32_t nx, ny, nz, sweeps;
};
hipError_t batch_sweep_launch(const BatchInst* insts, const BatchItem* items, int nitems,
                              const int32_t* item_tile, int sweep, int grid, hipStream_t s);

// SplitMix64 (Steele, Lea, Flood 2014): output i (1-based) of the stream
// seeded with s is mix(s + i * gamma).
static inline uint64_t splitmix_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static inline uint64_t splitmix_at(uint64_t seed, uint64_t i) {
    return splitmix_mix(seed + i * 0x9E3779B97F4A7C15ull);
}

}  // namespace ao
