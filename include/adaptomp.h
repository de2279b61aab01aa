/*
 * adaptomp.h -- C ABI of the adaptive-region library (libadaptomp.so).
 *
 * An adaptive region declares several variants of one data-parallel
 * computation (a launch geometry, a tiling or an execution target).  Each
 * execution is profiled; once enough samples exist a learned cost model
 * picks the variant for the execution's features.  The calls follow the
 * paper's producer-consumer statement of adaptation (Sec. 2, "Prior
 * proposed OpenMP adaptation extensions"; Sec. 3.1 "Usage of adaptation"):
 * the model produces a variant choice from features (selector_select), the
 * region consumes it (region_run), and profiling plus training close the
 * loop (region_profile, selector_train).  The runtime interface it plays
 * the role of is the Apollo API of Table 1.
 *
 * Conventions for every call:
 *   - Status codes: 0 = OK, > 0 = OK with a note, < 0 = error.  Errors never
 *     abort or exit; on error nothing has been enqueued and outputs are
 *     untouched.  ao_last_error() returns a thread-local message describing
 *     the last error of the calling thread.
 *   - Region handles are owned by the library; all data buffers and HIP
 *     streams are owned by the caller and are never freed by the library.
 *   - Device pointers are HIP device memory of the current device; "host"
 *     data buffers must be pinned host memory (hipHostMalloc).
 *   - Work is enqueued on the caller's stream (a hipStream_t passed as
 *     void*; NULL = the null stream).  Calls are thread-safe: each handle
 *     carries its own lock.
 *   - Floating point: region arithmetic is FP64 and every variant returns
 *     bit-identical results (see the region definitions below); the cost
 *     model is FP32.
 */
#ifndef ADAPTOMP_H
#define ADAPTOMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AO_MAX_VARIANTS 12 /* width of the cost model's output layer */
#define AO_MAX_FEATURES 6  /* width of the cost model's input layer */
#define AO_MLP_PARAMS 5388 /* 6*64+64 + 64*64+64 + 64*12+12 FP32 parameters */

enum ao_status {
    AO_OK = 0,
    AO_NOTE_UNTRAINED = 1, /* no trained model: exploration choice returned */
    AO_NOTE_FALLBACK = 2,  /* model output unusable / out of range: fallback used */
    AO_EINVAL = -1,        /* bad argument (sizes, pointers, kinds, variant ids) */
    AO_ENOMEM = -2,        /* library scratch could not be allocated */
    AO_EHIP = -3,          /* a HIP runtime call failed */
    AO_ESTATE = -4,        /* call not valid in the handle's current state */
    AO_EEXIST = -5,        /* model name already declared with a different spec */
    AO_EIO = -6,           /* file missing, unreadable or corrupt */
    AO_ELAUNCH = -7        /* the variant failed to launch; it is masked out */
};

/* Region kinds (the computation a region performs). */
enum ao_kind {
    /* S sweeps of the 7-point FP64 Jacobi stencil on an nx*ny*nz grid (x
     * fastest, index (k*ny + j)*nx + i): each sweep sets every point to
     * (((((xm+xp)+ym)+yp)+zm)+zp) * fl(1/6), neighbours outside the grid read
     * as +0.0, no fused multiply-add.  u0 is read, the S-th sweep lands in
     * out, u0 and out must not overlap.  (Stencil workload: Heat, Table 3.) */
    AO_JACOBI7_F64 = 0,
    /* y = A x for CSR A with int32 row_ptr[n+1] and col[nnz], FP64 val and x,
     * each row summed in the canonical pairwise order: products
     * fl(val*x[col]) indexed by their position in the row, padded with -0.0
     * to a power of two and added pairwise level by level (an empty row
     * gives +0.0).  (Sparse workload: AMGMk relax, Table 3.) */
    AO_CSR_SPMV_F64 = 1,
    /* Weighted Jacobi relaxation, the AMGMk relax kernel (Table 3): S =
     * sweeps applications of x <- x + (omega * (b - A x)) / diag, A x as in
     * AO_CSR_SPMV_F64 (canonical order), then one subtraction,
     * multiplication, division and addition per row, each rounded (no FMA).
     * x (the starting vector) is read, the S-th sweep lands in y; S = 0
     * copies x.  diag[n] is A's diagonal (the caller's; the library does not
     * look it up).  y must not overlap x, b, diag or the matrix arrays.
     * Uses the SpMV variant families; device-resident only. */
    AO_CSR_RELAX_F64 = 2
};

enum ao_target { AO_TARGET_GPU = 0, AO_TARGET_HOST = 1 };

enum ao_family {
    AO_FAM_JACOBI_DIRECT = 0, /* GPU: one thread per point, block bx*by (bx*by a multiple
                                 of 64, at most 1024); with AO_VF_LDS_SWEEPS a grid
                                 of at most 8192 points runs all its sweeps in one
                                 launch of one 1024-thread workgroup that holds the
                                 grid twice in LDS */
    AO_FAM_JACOBI_ZMARCH = 1, /* GPU: bx*by LDS plane tile + halo, marches bz planes */
    AO_FAM_JACOBI_HOST = 2,   /* host CPU (OpenMP): tiles bx (0 = whole row) by by rows */
    AO_FAM_JACOBI_ZREG = 3,   /* GPU: register z-march, strip bx (64|128) wide, by (1|2|4|8)
                                 rows per wave, 4 waves per block, bz planes per block */
    AO_FAM_JACOBI_ZREG_T2 = 4, /* GPU: register z-march with two sweeps fused per pass
                                  (temporal blocking); bx = 64, by (1|2|3|4|6|8|10|12|16)
                                  rows per wave, bz planes; an odd sweep count adds one
                                  single sweep */
    AO_FAM_JACOBI_ZREG_T3 = 5, /* GPU: the same with three sweeps fused per pass; bx = 64,
                                  by (1..6|8) rows per wave, bz planes; S mod 3 sweeps
                                  run first as one single or one two-sweep pass */
    AO_FAM_JACOBI_ZREG_T4 = 6, /* GPU: four sweeps fused per pass; bx = 64, by (1..5),
                                  bz planes; S mod 4 sweeps run first as one single, two-
                                  or three-sweep pass (each with the largest row count not
                                  above by that its family takes) */
    AO_FAM_JACOBI_COSCHED = 7, /* host CPU + GPU together (target AO_TARGET_GPU): the first
                                  round(nz * bx / 10) z-planes sweep on the host (OpenMP,
                                  whole rows in tiles of 8), the rest on the GPU (register
                                  z-march, 2 rows per wave, 16 planes), one halo plane
                                  exchanged each way after every sweep; bx = 0..10 (the
                                  host's share in tenths), by = bz = 0; timed with a
                                  steady clock and synchronous */
    AO_FAM_SPMV_THREAD_ROW = 10, /* GPU: one thread per row, blocks of bx */
    AO_FAM_SPMV_WAVE_ROW = 11,   /* GPU: by lanes (power of 2 <= 64, 0 = 64) per row, blocks of bx */
    AO_FAM_SPMV_MERGE_PATH = 12, /* GPU: nnz-balanced row-aligned chunks, blocks of bx */
    AO_FAM_SPMV_XSLICE = 13      /* GPU: columns cut into slices of 2^by columns (by 13|14;
                                    0 = 14: 64 or 128 KB of x) and rows into blocks of at most
                                    4096 nonzeros + rows (a block whose last row would take
                                    it past 4096 nonzeros is split before that row); a
                                    per-matrix plan orders the
                                    nonzeros slice by slice (about 15 B per nonzero plus 16 B
                                    per nonzero of value and product arrays); per execution
                                    the values are copied into that order when they changed
                                    (see values_id), each slice's products are formed with x
                                    in LDS, and each row block sums its rows from the
                                    products in LDS; bx = 0 (fixed geometry); rows longer
                                    than 4608 nonzeros are refused (AO_ELAUNCH, the variant
                                    is masked for the region) */
};

/* variant flags */
#define AO_VF_NT_STORE 1      /* non-temporal (streaming) stores of the output */
#define AO_VF_HALO_PREFETCH 2 /* register z-marches: issue the next plane's loads a plane
                                 ahead (the halo for one sweep; every load for two; for
                                 three and four, as soon as the first fused sweep has
                                 consumed the current plane) */
#define AO_VF_OCCUPANCY 4     /* two-sweep z-march: registers capped for 4 waves per SIMD */
#define AO_VF_LDS_SWEEPS 16   /* one-point-per-thread family: a grid of at most 8192
                                 points runs all its sweeps in one workgroup's LDS
                                 (larger grids run the family's kernel with the
                                 variant's block shape) */
#define AO_VF_STAGED 8        /* three- and four-sweep z-marches (not with
                                 AO_VF_HALO_PREFETCH): waves receive level 0 through
                                 asynchronous global->LDS copies one plane ahead (32-64
                                 KB of LDS per block); with more than 4 rows per wave
                                 (four sweeps) or 6 (three) only waves inside the grid,
                                 and for odd nx only waves whose 68 staged columns lie
                                 inside it */
#define AO_VF_FILL_Z 32       /* register z-marches of one to four sweeps: bz is an
                                 upper bound; each launch takes the planes per block,
                                 at most bz, that minimise the busiest CU's time:
                                 its blocks (the grid's, spread evenly over the CUs)
                                 each march their planes plus the 2(T-1) halo planes
                                 of T fused sweeps, in rounds of the kernel's
                                 occupancy and a last partial round, two at once
                                 1.4x and three 1.5x as fast as one; the fewest
                                 chunks within 3% of the best are taken, in equal
                                 lengths, so mid-size grids fill the chip */

/* One variant.  Ids are positions in the declaration array (0-based), as
 * categorical variants are numbered in declaration order (Sec. 3.1,
 * model_output clause). */
typedef struct ao_variant {
    int32_t target; /* enum ao_target */
    int32_t family; /* enum ao_family */
    int32_t bx, by, bz;
    int32_t flags;  /* AO_VF_* */
} ao_variant;

/* Arguments of one region execution.  All buffers are caller-owned. */
typedef struct ao_args {
    int32_t kind;     /* enum ao_kind; must match the region's kind */
    int32_t resident; /* 1 = buffers in device memory, 0 = in pinned host memory */
    /* Jacobi */
    const double* u0;
    double* out;
    int32_t nx, ny, nz, sweeps; /* nx <= 2^28, nx * ny * nz <= 2^40; else AO_EINVAL */
    /* SpMV (device-resident only) */
    const int32_t* row_ptr;
    const int32_t* col;
    const double* val;
    const double* x;
    double* y;
    int32_t n;
    int64_t nnz;
    /* Identity of the sparsity structure (the contents of row_ptr): the
     * per-matrix plan (features, merge-path partition) is cached under
     * (structure_id, row_ptr, n, nnz).  The caller gives a matrix a new id
     * whenever row_ptr may hold a different structure (a freed and reused
     * buffer, an edited matrix).  0 = unknown: the plan is rebuilt on every
     * call. */
    uint64_t structure_id;
    /* Identity of the values (the contents of val) under that structure:
     * families that keep the values in an order of their own
     * (AO_FAM_SPMV_XSLICE) reuse that copy while values_id, structure_id
     * and val are unchanged.  The caller gives new values a new id; 0 =
     * unknown: the copy is refreshed on every call (within one relaxation
     * execution it is made once for all sweeps). */
    uint64_t values_id;
    /* Relaxation (AO_CSR_RELAX_F64; x, y, the matrix and sweeps as above):
     * right-hand side b[n], diagonal diag[n], weight omega. */
    const double* b;
    const double* diag;
    double omega;
} ao_args;

typedef struct ao_region ao_region; /* opaque, library-owned */

/* Declare (create once) an adaptive region -- Sec. 3.1 `adaptation`
 * directive clauses model_name / variants / min_train_data / model_type,
 * and Table 1 __apollo_region_create.
 *   model_name     unique id; declaring the same name again with the same
 *                  spec returns the same handle, with a different spec
 *                  AO_EEXIST.
 *   kind           enum ao_kind.
 *   variants       num_variants entries (1..AO_MAX_VARIANTS), copied.
 *   min_train_data unique (features, variant) samples before training is
 *                  triggered; <= 0 means num_variants (Sec. 3.1 default).
 *   model_type     "mlp" (default, NULL), "dtree" / "dtree,D" (the paper's
 *                  decision-tree classifier of depth 2 / D on fastest-variant
 *                  labels, trained and evaluated on the host), "exhaustive"
 *                  (time every variant for each new feature vector) or
 *                  "roundrobin" (explore only, never train).
 *   out            receives the handle. */
int region_declare_variants(const char* model_name, int kind, const ao_variant* variants,
                            int num_variants, int min_train_data, const char* model_type,
                            ao_region** out);

/* Execute the region once (Sec. 3.3 call sequence: begin, set features, get
 * policy, run the variant, end).
 *   features  AO_MAX_FEATURES floats, or NULL to compute them: Jacobi
 *             [log2 nx, log2 ny, log2 nz, sweeps, log2(16*N*sweeps),
 *             resident]; SpMV [log2 n, log2 nnz, mean row length,
 *             log2(1 + row-length variance), log2 max row length] (computed
 *             once per matrix on the GPU and cached); relaxation: the SpMV
 *             features and sweeps.
 *   variant   -1: the producer decides (RoundRobin before training, the
 *             model's argmin after, exhaustive timing for
 *             model_type "exhaustive"); >= 0: run that id.
 *   chosen    receives the variant that ran (may be NULL).
 * GPU variants are enqueued on `stream` and timed with HIP events whose
 * results are collected lazily; host variants synchronise the stream, run on
 * the calling thread's OpenMP team and are timed with a steady clock
 * (including any host<->device copies; on host-resident data with a NULL
 * stream they start at once and never touch the GPU).  The execution is
 * appended to the profile database; if it brings the unique-sample count to
 * min_train_data and the model type is "mlp", training runs before the call
 * returns (a failed training leaves the region untrained, is reported by
 * ao_last_error and region_stats, and is retried once the unique count has
 * doubled; the execution itself still succeeds).
 * Returns AO_NOTE_UNTRAINED when the choice came from exploration,
 * AO_NOTE_FALLBACK when the model's choice was replaced. */
int region_run(ao_region* r, const ao_args* a, const float* features, void* stream, int variant,
               int* chosen);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc:
 * region_run of the named GPU variant (variant >= 0) of a Jacobi region
 * on device-resident buffers that allocates nothing.  The array between
 * the launches of one execution (needed when the variant takes more than
 * one launch: more sweeps than it fuses) is a fixed device array of
 * AO_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends, instead of the region's own scratch.  No
 * selection, profiling record or training takes place.  Enqueued on
 * stream (of the current device); output bit-identical to region_run of
 * the same variant.  AO_EINVAL, with nothing enqueued, for a grid whose
 * execution needs more than AO_NOALLOC_SCRATCH_BYTES of scratch (more than
 * AO_NOALLOC_SCRATCH_BYTES / 8 points and more than one launch), a host or
 * co-scheduled variant, host-resident data, an SpMV region or a variant id
 * < 0.  Every call on one GPU shares its array and leaves its contents
 * behind: calls that overlap in time on one GPU (other streams or threads)
 * race and must be serialised by the caller.  The array needs no clearing:
 * each launch writes all of it before the next one reads it. */
#define AO_NOALLOC_SCRATCH_BYTES 67108864 /* 64 MiB: grids of up to 8,388,608 points */
int region_run_noalloc(ao_region* r, const ao_args* a, void* stream, int variant);

/* Record one execution that the caller ran itself (the consumer side of the
 * producer-consumer pattern: user code ran variant `variant` for these
 * features and took `seconds`) -- Table 1 __apollo_region_end.  Appends to
 * the profile database and applies the same train trigger as region_run. */
int region_record(ao_region* r, const float* features, int variant, double seconds);

/* Compute the feature vector of one execution without running it (Table 1
 * __apollo_region_set_feature values): features[AO_MAX_FEATURES] as listed
 * for region_run.  SpMV features are computed on the GPU once per matrix
 * (row_ptr, n, nnz) and cached; synchronises `stream` in that case. */
int region_features(ao_region* r, const ao_args* a, void* stream, float* features);

#define AO_PROFILE_RECORD 1 /* append the timed runs to the profile database */

/* Time variants in isolation (Table 1 begin/end timing) -- the exhaustive
 * selector and the yardstick of the learned one.  For each variant (all if
 * variant == -1): `warmup` untimed runs, then `reps` timed runs; writes the
 * median seconds to median_seconds[v] (num_variants entries when variant ==
 * -1, else 1 entry; a variant that cannot run gets +inf).  Synchronises.
 * flags: AO_PROFILE_RECORD. */
int region_profile(ao_region* r, const ao_args* a, const float* features, int variant, int warmup,
                   int reps, void* stream, int flags, double* median_seconds);

/* Training options (NULL = defaults in brackets). */
typedef struct ao_train_opts {
    int32_t epochs;     /* [200]; 0 installs the untrained (initial) network */
    int32_t batch;      /* [256] */
    float lr;           /* [1e-3] Adam learning rate; betas 0.9 / 0.999, eps 1e-8 */
    uint64_t seed;      /* [7] SplitMix64 seed of the init and of the shuffles */
} ao_train_opts;

/* Train the cost model on the profile database (Table 1
 * __apollo_region_train).  For a "dtree" region: CART with Gini impurity on
 * one sample per distinct feature tuple labelled with its fastest variant;
 * opts are ignored and final_loss receives the training error rate.  The dataset merges duplicate (features, variant)
 * samples by median time; inputs are z-scored, the target is ln(seconds)
 * minus its mean, the loss is the masked MSE of the measured variant; the
 * FP32 MLP 6-64-64-12 (ReLU) is trained with Adam on the GPU by the
 * library's own kernels.  final_loss (may be NULL) receives the last
 * epoch's mean loss.  Synchronises. */
int selector_train(ao_region* r, const ao_train_opts* opts, double* final_loss);

/* Produce variant choices for `batch` feature vectors (batch *
 * AO_MAX_FEATURES floats, host memory) into variants_out[batch] -- Table 1
 * __apollo_region_get_policy / the model_output clause.  With a trained
 * model: argmin of the predicted ln-times over the region's variants (ties
 * to the lowest id), computed by the inference kernel.  Without one: the
 * next exploration id and AO_NOTE_UNTRAINED.  Synchronises. */
int selector_select(ao_region* r, const float* features, int batch, int* variants_out);

/* ---- batched execution of many uneven Jacobi instances ------------------ */

typedef struct ao_batch ao_batch; /* opaque, library-owned plan */

/* Build a plan for `count` device-resident Jacobi instances (inst[i] as for
 * region_run; sweeps may differ).  Instances are bucketed by their largest
 * dimension ((0,16], (16,32], (32,64], (64,128], (128,inf)); each bucket
 * uses one tile shape (from the autotuner, else a default) and every
 * (instance, tile) pair becomes one work item.  The library allocates the
 * ping-pong scratch (sum of N_i doubles).  The instance buffers must stay
 * valid for the plan's lifetime. */
int batch_create(const ao_args* inst, int count, ao_batch** out);

/* Autotune: for each bucket time each candidate tile shape over the
 * bucket's instances (warmup + reps, median) and keep the fastest; then,
 * largest bucket first, time each candidate again over the whole batch with
 * every other bucket on its current tile and keep the fastest (the buckets
 * share the persistent kernels, so the best tile alone can balance worse
 * beside the others).  Writes the chosen candidate index per bucket to
 * chosen[5] (may be NULL; -1 = empty bucket).  Synchronises; overwrites the
 * instances' outputs. */
int batch_autotune(ao_batch* b, void* stream, int warmup, int reps, int* chosen);

/* Run every instance once: one persistent kernel per pass over the work
 * list -- a pass is one sweep, two sweeps on the two-sweep tiles (the first
 * pass of an odd sweep count is then a single sweep) or three on the
 * three-sweep tiles (the first pass then takes the S mod 3 remaining
 * sweeps), so an instance takes S, ceil(S/2) or ceil(S/3) passes.  The
 * three tile families run in three persistent kernels launched one after
 * the other in each pass; the three-sweep kernel receives level 0 of its
 * two- and three-sweep passes through global->LDS copies a plane ahead
 * (48 KB of LDS per workgroup) wherever the staged columns fit the grid.
 * use_graph != 0
 * launches all passes as one captured HIP graph (captured on first use,
 * re-captured after autotuning or batch_set_tiles).  Enqueued on
 * `stream`. */
int batch_run(ao_batch* b, void* stream, int use_graph);

/* Per-bucket information: number of instances, work items and the tile
 * (tx, ty, tz) in use, 5 buckets each, any pointer may be NULL.  For a
 * two-sweep tile tx = 62, for a three-sweep tile tx = 60 (columns stored
 * per 64-lane strip). */
int batch_info(const ao_batch* b, int* instances, int* items, int* tiles_xyz);

/* The least HBM traffic one batch_run can move with the tiles in use: each
 * pass reads every point of its instance once and writes it once, so
 * 16 B x points x passes summed over the instances (the sweeps fused in a
 * pass stay on chip).  Written to *bytes; the roofline of a batched run is
 * taken against it. */
int batch_min_traffic(const ao_batch* b, double* bytes);

/* The candidate tile table the autotuner searches: returns its length and,
 * when tiles is not NULL, writes (kind, tx, ty, tz) per candidate into
 * tiles[4 * length]; kind 0 = one point per thread, 1|2|4 = register
 * z-march with that many rows per wave, 11|12|14 = fused two-sweep
 * z-march with 1|2|4 rows per wave, 21|22|24 = fused three-sweep z-march
 * with 1|2|4 rows per wave. */
int batch_candidates(int* tiles);

/* Fix the tile of each bucket: cand[5] candidate indices, -1 keeps the
 * bucket's current tile.  AO_EINVAL for an index outside the table (the
 * plan is unchanged). */
int batch_set_tiles(ao_batch* b, const int* cand);

int batch_destroy(ao_batch* b);

/* ---- cost-model kernels on caller buffers (gradient checks) ------------- */

/* Forward pass of the MLP on device buffers: params[AO_MLP_PARAMS] (W1 64x6,
 * b1, W2 64x64, b2, W3 12x64, b3, row-major [out][in]), x[batch*6]
 * (already normalised), out[batch*12].  Enqueued on stream. */
int ao_mlp_forward(const float* params, const float* x, int batch, float* out, void* stream);

/* Gradient of the masked MSE 0.5/B * sum mask*(o - y)^2 on device buffers:
 * y[batch], mask[batch*12], grad[AO_MLP_PARAMS] (overwritten), loss[1]
 * (device, may be NULL).  Enqueued on stream. */
int ao_mlp_grad(const float* params, const float* x, const float* y, const float* mask, int batch,
                float* grad, float* loss, void* stream);

/* One Adam step (step count t >= 1) on device buffers params, m, v (all
 * AO_MLP_PARAMS) with gradient grad.  Enqueued on stream. */
int ao_mlp_adam(float* params, float* m, float* v, const float* grad, int t, float lr, void* stream);

/* ---- database, state, persistence ------------------------------------- */

typedef struct ao_stats {
    int64_t records;      /* profile records held */
    int64_t unique;       /* distinct (features, variant) pairs */
    int32_t trained;      /* 1 when a usable model exists */
    int32_t num_variants;
    int64_t explore_next; /* RoundRobin counter */
    int64_t trainings;    /* number of completed trainings */
    int64_t fallbacks;    /* exhaustive fallbacks taken */
    int32_t failed_mask;  /* bit v set: variant v failed to launch and is masked */
    int32_t min_train;
    int64_t memo_size;    /* memoised feature vectors */
    double last_train_seconds;
    int64_t train_failures; /* automatic trainings that failed */
} ao_stats;

int region_stats(ao_region* r, ao_stats* out);

/* Copy up to max_records profile records, oldest first: features
 * [max_records * AO_MAX_FEATURES], variant ids, seconds (any may be NULL).
 * Returns the number copied (>= 0) or an error. */
int region_records(ao_region* r, float* features, int* variants, double* seconds, int max_records);

/* Save / load the profile database and the model (weights and
 * normalisation) as a versioned binary file with a CRC-32 (Sec. 3:
 * profiling data accumulate across runs, a trained model is available to
 * later runs).  region_load requires the same kind and variants; a corrupt
 * or missing file leaves the region unchanged and returns AO_EIO. */
int region_save(ao_region* r, const char* path);
int region_load(ao_region* r, const char* path);

/* Forget the memoised choices (the next executions query the model again). */
int region_clear_memo(ao_region* r);

int region_destroy(ao_region* r);

const char* ao_last_error(void);

/* Plain FP64 stream copy dst[0..n) = src[0..n) on device memory (16-byte
 * aligned), enqueued on stream: the achievable-bandwidth probe that region
 * bandwidth is compared with, and the calibration kernel of the byte
 * counters.  nontemporal != 0 uses streaming stores. */
int ao_hbm_copy(const double* src, double* dst, int64_t n, int nontemporal, void* stream);

/* Random-gather probe: the memory access of a gather-per-nonzero SpMV
 * (Sec. 4, the irregular AMGMk-style region) and nothing else.  idx[0..m)
 * (int32, device) is streamed once, x[idx[k]] (FP64, device, nx entries;
 * indices outside [0, nx) read x[0]) is gathered, and the gathered values
 * of each wave (512 entries) are summed into one double of out: out holds
 * 4 * ceil(m / 2048) doubles (device, caller-owned); workgroup g covers
 * entries [2048 g, 2048 g + 2048) and lands on XCD g % 8 under round-robin
 * dispatch.  Passing a matrix's column array as idx times the gathers of
 * an SpMV of that matrix without its value stream.  Enqueued on stream;
 * AO_EINVAL for bad arguments, nothing enqueued. */
int ao_gather_probe(const int32_t* idx, const double* x, int64_t m, int64_t nx, double* out,
                    void* stream);

/* Number of compute units of the current device (0 if none). */
int ao_device_cus(void);

/* Planes per block that one launch of GPU Jacobi variant *v (a register
 * z-march family: ZREG, ZREG_T2, ZREG_T3, ZREG_T4) uses on an nx x ny x nz
 * grid: v->bz, or with AO_VF_FILL_Z the chunk length chosen for `cus` CUs
 * that each hold `blocks_per_cu` of the kernel's workgroups at once (cus <=
 * 0: the current device's CU count and the kernel's own occupancy; then a
 * device must be present, and without one the answer is v->bz).  Written to
 * *planes; AO_EINVAL for non-positive dimensions, cus > 0 with
 * blocks_per_cu < 1, a null pointer or a variant that fits no z-march
 * kernel.  Reports the launch geometry a profiled variant actually ran
 * (Sec. 3.1: a variant is its launch configuration). */
int ao_jacobi_planes(const ao_variant* v, int32_t nx, int32_t ny, int32_t nz, int32_t cus,
                     int32_t blocks_per_cu, int32_t* planes);

#ifdef __cplusplus
}
#endif

#endif /* ADAPTOMP_H */
