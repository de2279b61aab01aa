// Adaptive-region runtime: variant registry, profiler, profile database,
// RoundRobin exploration, train trigger, learned / exhaustive selection,
// persistence.  Host control plane of the library; every region variant and
// the cost model run in the kernels of the other translation units.
//
// Lifecycle of one execution (Sec. 3.3 code generation: create once, begin,
// set features, get policy, run, end -> record and maybe train):
//   region_run -> features -> choose() -> run_variant() -> record -> trigger.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "internal.h"

namespace ao {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

namespace {

std::string hip_msg(const char* what, hipError_t e) {
    return std::string(what) + ": " + hipGetErrorString(e);
}

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Record {
    float f[AO_MAX_FEATURES];
    int32_t variant;
    int32_t resident;
    double seconds;  // NaN while a GPU timing is pending
    uint64_t t_ns;
};

struct FeatKey {
    uint32_t b[AO_MAX_FEATURES];
    bool operator==(const FeatKey& o) const { return memcmp(b, o.b, sizeof(b)) == 0; }
};
struct FeatKeyHash {
    size_t operator()(const FeatKey& k) const {
        uint64_t h = 0x243F6A8885A308D3ull;
        for (uint32_t v : k.b) h = splitmix_mix(h ^ v);
        return (size_t)h;
    }
};
FeatKey make_key(const float* f) {
    FeatKey k;
    for (int i = 0; i < AO_MAX_FEATURES; ++i) {
        float v = f[i] == 0.0f ? 0.0f : f[i];  // -0 and +0 are one feature value
        memcpy(&k.b[i], &v, 4);
    }
    return k;
}
struct UKey {
    FeatKey f;
    int v;
    bool operator==(const UKey& o) const { return v == o.v && f == o.f; }
};
struct UKeyHash {
    size_t operator()(const UKey& k) const { return FeatKeyHash()(k.f) ^ ((size_t)k.v * 0x9E37u); }
};

struct Pending {
    hipEvent_t a, b;
    size_t rec;
};

double median_of(std::vector<double> v) {
    if (v.empty()) return INFINITY;
    std::sort(v.begin(), v.end());
    const size_t n = v.size();
    return (n % 2) ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

}  // namespace
}  // namespace ao

using namespace ao;

struct ao_region {
    std::mutex mu;
    std::string name;
    int kind = 0;
    std::vector<ao_variant> variants;
    int min_train = 0;
    std::string model_type;
    int device = 0;

    std::vector<Record> db;
    std::unordered_set<UKey, UKeyHash> uniq;
    std::deque<Pending> pending;
    std::vector<hipEvent_t> pool;
    int64_t rr = 0;
    int failed_mask = 0;
    int64_t trainings = 0, fallbacks = 0, train_failures = 0;
    int64_t retrain_at = 0;  // no automatic training before this unique count
    double last_train_seconds = 0.0;

    // model
    int dtree_depth = 0;  // > 0: model type "dtree[,depth]"
    DTree tree;
    bool trained = false;
    std::vector<float> params;  // host copy
    MlpNorm norm{};
    float fmin[AO_MAX_FEATURES] = {0}, fmax[AO_MAX_FEATURES] = {0};
    float* d_params = nullptr;
    MlpNorm* d_norm = nullptr;
    std::unordered_map<FeatKey, int, FeatKeyHash> memo;

    // selection staging (pinned host, read/written by the inference kernel)
    hipStream_t sel_stream = nullptr;
    float* h_feat = nullptr;
    int32_t* h_ids = nullptr;
    float* m_feat = nullptr;    // device-side addresses of the two buffers
    int32_t* m_ids = nullptr;
    int sel_cap = 0;

    // region scratch
    double* d_a = nullptr;
    double* d_b = nullptr;
    size_t d_cap = 0;
    double* h_a = nullptr;
    double* h_b = nullptr;
    size_t h_cap = 0;
    std::vector<double> host_tmp;  // second buffer of host variants on host data

    std::vector<std::unique_ptr<SpmvPlan>> plans;

    ~ao_region();
};

namespace ao {
namespace {

std::mutex g_reg_mu;
std::map<std::string, ao_region*> g_regions;

bool same_variant(const ao_variant& a, const ao_variant& b) {
    return a.target == b.target && a.family == b.family && a.bx == b.bx && a.by == b.by &&
           a.bz == b.bz && a.flags == b.flags;
}

// rows per wave the two-sweep kernel is compiled for
bool t2_rows_ok(int r) {
    return r == 1 || r == 2 || r == 3 || r == 4 || r == 6 || r == 8 || r == 10 || r == 12 ||
           r == 16;
}

// rows per wave the three-sweep kernel is compiled for
bool t3_rows_ok(int r) { return (r >= 1 && r <= 6) || r == 8; }

int validate_variant(int kind, const ao_variant& v, int id) {
    const std::string at = "variant " + std::to_string(id) + ": ";
    if (kind == AO_JACOBI7_F64) {
        if (v.target == AO_TARGET_HOST) {
            if (v.family != AO_FAM_JACOBI_HOST)
                return fail(AO_EINVAL, at + "host target needs the host Jacobi family");
            if (v.bx < 0 || v.by < 0) return fail(AO_EINVAL, at + "negative tile");
            return AO_OK;
        }
        if (v.target != AO_TARGET_GPU) return fail(AO_EINVAL, at + "unknown target");
        if (v.family != AO_FAM_JACOBI_DIRECT && v.family != AO_FAM_JACOBI_ZMARCH &&
            v.family != AO_FAM_JACOBI_ZREG && v.family != AO_FAM_JACOBI_ZREG_T2 &&
            v.family != AO_FAM_JACOBI_ZREG_T3 && v.family != AO_FAM_JACOBI_ZREG_T4 &&
            v.family != AO_FAM_JACOBI_COSCHED)
            return fail(AO_EINVAL, at + "unknown GPU Jacobi family");
        if (v.family == AO_FAM_JACOBI_ZREG_T2 &&
            (v.bx != 64 || !t2_rows_ok(v.by) || v.bz <= 0))
            return fail(AO_EINVAL,
                        at + "two-sweep z-march needs bx 64, by 1|2|3|4|6|8|10|12|16, bz > 0");
        if ((v.flags & AO_VF_LDS_SWEEPS) && v.family != AO_FAM_JACOBI_DIRECT)
            return fail(AO_EINVAL, at + "all sweeps in LDS is a flag of the one-point-per-thread "
                                        "family");
        if ((v.flags & AO_VF_FILL_Z) &&
            (v.family != AO_FAM_JACOBI_ZREG && v.family != AO_FAM_JACOBI_ZREG_T2 &&
             v.family != AO_FAM_JACOBI_ZREG_T3 && v.family != AO_FAM_JACOBI_ZREG_T4))
            return fail(AO_EINVAL, at + "filling the device by z-chunk length is for the "
                                        "register z-marches");
        if ((v.flags & AO_VF_STAGED) &&
            ((v.family != AO_FAM_JACOBI_ZREG_T3 && v.family != AO_FAM_JACOBI_ZREG_T4) ||
             (v.flags & AO_VF_HALO_PREFETCH)))
            return fail(AO_EINVAL, at + "staged level 0 is for the three- and four-sweep "
                                        "z-marches, without the prefetch flag");
        if (v.family == AO_FAM_JACOBI_ZREG_T3 && (v.bx != 64 || !t3_rows_ok(v.by) || v.bz <= 0))
            return fail(AO_EINVAL, at + "three-sweep z-march needs bx 64, by 1..6|8, bz > 0");
        if (v.family == AO_FAM_JACOBI_COSCHED) {
            if (v.bx < 0 || v.bx > 10 || v.by != 0 || v.bz != 0)
                return fail(AO_EINVAL, at + "co-scheduling needs bx 0..10 (host tenths), by = bz = 0");
            return AO_OK;
        }
        if (v.family == AO_FAM_JACOBI_ZREG_T4 &&
            (v.bx != 64 || v.by < 1 || v.by > 5 || v.bz <= 0))
            return fail(AO_EINVAL, at + "four-sweep z-march needs bx 64, by 1..5, bz > 0");
        if (v.family == AO_FAM_JACOBI_ZREG &&
            ((v.bx != 64 && v.bx != 128) || (v.by != 1 && v.by != 2 && v.by != 4 && v.by != 8) ||
             v.bz <= 0))
            return fail(AO_EINVAL, at + "register z-march needs bx 64|128, by 1|2|4|8, bz > 0");
        if (v.bx <= 0 || v.by <= 0) return fail(AO_EINVAL, at + "block sizes must be positive");
        if (v.family == AO_FAM_JACOBI_ZMARCH && v.bz <= 0)
            return fail(AO_EINVAL, at + "z-march needs bz > 0");
        return AO_OK;
    }
    if (kind == AO_CSR_SPMV_F64 || kind == AO_CSR_RELAX_F64) {
        if (v.target != AO_TARGET_GPU) return fail(AO_EINVAL, at + "SpMV variants run on the GPU");
        if (v.family != AO_FAM_SPMV_THREAD_ROW && v.family != AO_FAM_SPMV_WAVE_ROW &&
            v.family != AO_FAM_SPMV_MERGE_PATH && v.family != AO_FAM_SPMV_XSLICE)
            return fail(AO_EINVAL, at + "unknown SpMV family");
        if (v.family == AO_FAM_SPMV_XSLICE) {
            if (v.bx != 0 || (v.by != 0 && v.by != 13 && v.by != 14))
                return fail(AO_EINVAL, at + "x-slice SpMV needs bx 0, by 0|13|14");
            return AO_OK;
        }
        if (v.bx <= 0) return fail(AO_EINVAL, at + "block size must be positive");
        if (v.family == AO_FAM_SPMV_WAVE_ROW && v.by != 0 &&
            (v.by < 1 || v.by > 64 || (v.by & (v.by - 1))))
            return fail(AO_EINVAL, at + "lanes per row must be a power of two <= 64");
        return AO_OK;
    }
    return fail(AO_EINVAL, "unknown region kind");
}

int validate_args(const ao_region* r, const ao_args* a) {
    if (!a) return fail(AO_EINVAL, "args is NULL");
    if (a->kind != r->kind) return fail(AO_EINVAL, "args kind does not match the region kind");
    if (r->kind == AO_JACOBI7_F64) {
        if (a->nx < 0 || a->ny < 0 || a->nz < 0 || a->sweeps < 0)
            return fail(AO_EINVAL, "negative grid size or sweep count");
        if (a->resident != 0 && a->resident != 1) return fail(AO_EINVAL, "resident must be 0 or 1");
        const int64_t n = (int64_t)a->nx * a->ny * a->nz;
        if (n > ((int64_t)1 << 40)) return fail(AO_EINVAL, "grid too large");
        if (a->nx > (1 << 28)) return fail(AO_EINVAL, "nx above 2^28");
        if (n > 0 && (!a->u0 || !a->out)) return fail(AO_EINVAL, "u0/out is NULL");
        if (n > 0) {
            const char* u = (const char*)a->u0;
            const char* o = (const char*)a->out;
            const size_t bytes = (size_t)n * 8;
            if (u < o + bytes && o < u + bytes) return fail(AO_EINVAL, "u0 and out overlap");
        }
        return AO_OK;
    }
    if (a->resident != 1) return fail(AO_EINVAL, "SpMV regions need device-resident buffers");
    if (a->n < 0 || a->nnz < 0 || a->nnz > 0x7fffffffLL)
        return fail(AO_EINVAL, "bad n / nnz (int32 indices)");
    if (a->n > 0 && (!a->row_ptr || !a->x || !a->y))
        return fail(AO_EINVAL, "row_ptr/x/y is NULL");
    if (a->nnz > 0 && (!a->col || !a->val)) return fail(AO_EINVAL, "col/val is NULL");
    if (r->kind == AO_CSR_RELAX_F64) {
        if (a->sweeps < 0) return fail(AO_EINVAL, "negative sweep count");
        if (!isfinite(a->omega)) return fail(AO_EINVAL, "omega must be finite");
        if (a->n > 0 && (!a->b || !a->diag)) return fail(AO_EINVAL, "b/diag is NULL");
        // y is written while x (every column), b, diag and the matrix are read
        auto overlaps = [&](const void* p, size_t bytes) {
            const char* q = (const char*)p;
            const char* yy = (const char*)a->y;
            const size_t yb = (size_t)a->n * 8;
            return p && bytes > 0 && q < yy + yb && yy < q + bytes;
        };
        const size_t nb = (size_t)a->n * 8;
        if (a->n > 0 && (overlaps(a->x, nb) || overlaps(a->b, nb) || overlaps(a->diag, nb) ||
                         overlaps(a->val, (size_t)a->nnz * 8) ||
                         overlaps(a->col, (size_t)a->nnz * 4) ||
                         overlaps(a->row_ptr, ((size_t)a->n + 1) * 4)))
            return fail(AO_EINVAL, "y overlaps an input of the relaxation");
    }
    return AO_OK;
}

int ensure_dev(ao_region* r, size_t n) {
    if (r->d_cap >= n) return AO_OK;
    if (r->d_a) hipFree(r->d_a);
    if (r->d_b) hipFree(r->d_b);
    r->d_a = r->d_b = nullptr;
    r->d_cap = 0;
    hipError_t e = hipMalloc(&r->d_a, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&r->d_b, n * sizeof(double));
    if (e != hipSuccess) {
        if (r->d_a) hipFree(r->d_a);
        r->d_a = nullptr;
        (void)hipGetLastError();
        return fail(AO_ENOMEM, hip_msg("device scratch", e));
    }
    r->d_cap = n;
    return AO_OK;
}

int ensure_host(ao_region* r, size_t n) {
    if (r->h_cap >= n) return AO_OK;
    if (r->h_a) hipHostFree(r->h_a);
    if (r->h_b) hipHostFree(r->h_b);
    r->h_a = r->h_b = nullptr;
    r->h_cap = 0;
    hipError_t e = hipHostMalloc(&r->h_a, n * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&r->h_b, n * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        if (r->h_a) hipHostFree(r->h_a);
        r->h_a = nullptr;
        (void)hipGetLastError();
        return fail(AO_ENOMEM, hip_msg("pinned host scratch", e));
    }
    r->h_cap = n;
    return AO_OK;
}

hipEvent_t get_event(ao_region* r) {
    if (!r->pool.empty()) {
        hipEvent_t e = r->pool.back();
        r->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Collect finished GPU timings (all of them when block is set).
void harvest(ao_region* r, bool block) {
    for (auto it = r->pending.begin(); it != r->pending.end();) {
        if (block) {
            hipEventSynchronize(it->b);
        } else if (hipEventQuery(it->b) != hipSuccess) {
            ++it;
            continue;
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, it->a, it->b) == hipSuccess)
            r->db[it->rec].seconds = (double)ms * 1e-3;
        else
            r->db[it->rec].seconds = INFINITY;
        r->pool.push_back(it->a);
        r->pool.push_back(it->b);
        it = r->pending.erase(it);
    }
    (void)hipGetLastError();
}

SpmvPlan* get_plan(ao_region* r, const ao_args* a, hipStream_t s, int* rc) {
    if (a->structure_id != 0) {
        for (auto& p : r->plans)
            if (p->structure_id == a->structure_id && p->row_ptr == a->row_ptr &&
                p->n == a->n && p->nnz == a->nnz)
                return p.get();
    }
    // drop plans whose id is unknown or now names other buffers; keep <= 8
    for (auto it = r->plans.begin(); it != r->plans.end();) {
        const bool stale = (*it)->structure_id == 0 ||
                           ((*it)->structure_id == a->structure_id);
        it = stale ? r->plans.erase(it) : it + 1;
    }
    if (r->plans.size() >= 8) r->plans.erase(r->plans.begin());
    auto p = std::make_unique<SpmvPlan>();
    p->structure_id = a->structure_id;
    p->row_ptr = a->row_ptr;
    p->n = a->n;
    p->nnz = a->nnz;
    hipError_t e = spmv_features(*p, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *rc = fail(AO_EHIP, hip_msg("csr features", e));
        return nullptr;
    }
    p->have_features = true;
    // merge-path partitions for the region's merge-path variants and the
    // x-slice variants' plans (a matrix an x-slice plan cannot take -- a row
    // above its limit, too many slices -- leaves that plan out: the variant
    // then fails to launch and is masked)
    for (const ao_variant& v : r->variants) {
        if (p->n <= 0) continue;
        if (v.family == AO_FAM_SPMV_XSLICE) {
            e = spmv_prepare_xslice(*p, v.by == 0 ? 14 : v.by, a->col, s);
            if (e == hipErrorInvalidConfiguration) {
                (void)hipGetLastError();
                continue;
            }
        } else if (v.family == AO_FAM_SPMV_MERGE_PATH) {
            if (v.bx != 64 && v.bx != 128 && v.bx != 256 && v.bx != 512 && v.bx != 1024) continue;
            e = spmv_prepare_merge(*p, v.bx, s);
        } else {
            continue;
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *rc = fail(AO_EHIP, hip_msg("merge-path / x-slice plan", e));
            return nullptr;
        }
    }
    r->plans.push_back(std::move(p));
    return r->plans.back().get();
}

int compute_features(ao_region* r, const ao_args* a, hipStream_t s, float* f) {
    for (int i = 0; i < AO_MAX_FEATURES; ++i) f[i] = 0.0f;
    if (r->kind == AO_JACOBI7_F64) {
        const double n = (double)a->nx * a->ny * a->nz;
        const double bytes = 16.0 * n * a->sweeps;
        f[0] = (float)log2(std::max(1, a->nx));
        f[1] = (float)log2(std::max(1, a->ny));
        f[2] = (float)log2(std::max(1, a->nz));
        f[3] = (float)a->sweeps;
        f[4] = (float)log2(std::max(1.0, bytes));
        f[5] = (float)a->resident;
        return AO_OK;
    }
    int rc = AO_OK;
    SpmvPlan* p = get_plan(r, a, s, &rc);
    if (!p) return rc;
    memcpy(f, p->features, sizeof(p->features));
    if (r->kind == AO_CSR_RELAX_F64) f[5] = (float)a->sweeps;
    return AO_OK;
}

// CPU+GPU co-scheduling of one Jacobi execution (the co-scheduling use
// case, Sec. 3.2): planes [0, kc) sweep on the host, planes [kc, nz) on the
// GPU, kc = round(nz * bx / 10).  Each side sweeps a sub-grid that carries
// the other side's boundary plane as a halo (its own output for that plane
// is discarded), the GPU asynchronously while the host team works; after the
// sweep the new boundary planes cross (one plane each way).  Every plane is
// computed with the region's arithmetic, so the result is bit-identical to
// any single-target variant.  Synchronous; timed with the steady clock.
int run_cosched(ao_region* r, const ao_variant& v, const ao_args* a, hipStream_t s,
                double* secs) {
    const int nx = a->nx, ny = a->ny, nz = a->nz, S = a->sweeps;
    const size_t plane = (size_t)nx * ny, n = plane * nz;
    const int kc = (int)(((int64_t)nz * v.bx + 5) / 10);
    const bool host_part = kc > 0, gpu_part = kc < nz;
    const int gb = host_part ? kc - 1 : 0;           // first plane of the GPU sub-grid
    const int hz = gpu_part ? kc + 1 : nz;           // planes of the host sub-grid
    const ao_variant gin{AO_TARGET_GPU, AO_FAM_JACOBI_ZREG, 64, 2, 16, v.flags & AO_VF_NT_STORE};
    const ao_variant hin{AO_TARGET_HOST, AO_FAM_JACOBI_HOST, 0, 8, 1, 0};
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(AO_EHIP, hip_msg("stream sync", e));
    if (n > 0 && gpu_part) {
        int rc = ensure_dev(r, n);
        if (rc) return rc;
    }
    if (n > 0 && host_part && a->resident) {
        int rc = ensure_host(r, (size_t)hz * plane);
        if (rc) return rc;
    }
    if (n > 0 && !a->resident && S >= 2 && r->host_tmp.size() < n) r->host_tmp.assign(n, 0.0);
    const uint64_t t0 = now_ns();
    auto copy = [&](void* dst, const void* src, size_t bytes, hipMemcpyKind k) {
        if (e == hipSuccess && bytes > 0) e = hipMemcpyAsync(dst, src, bytes, k, s);
    };
    if (n > 0 && S == 0) {
        copy(a->out, a->u0, n * 8, a->resident ? hipMemcpyDeviceToDevice : hipMemcpyHostToHost);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    } else if (n > 0) {
        // sweep-0 sources; the device chain ends in the device result buffer,
        // the host chain in the host one
        const double* dsrc = nullptr;
        const double* hsrc = nullptr;
        if (a->resident) {
            dsrc = a->u0;
            if (host_part) copy(r->h_a, a->u0, (size_t)hz * plane * 8, hipMemcpyDeviceToHost);
            hsrc = r->h_a;
        } else {
            hsrc = a->u0;
            if (gpu_part)
                copy(r->d_a + (size_t)gb * plane, a->u0 + (size_t)gb * plane,
                     (size_t)(nz - gb) * plane * 8, hipMemcpyHostToDevice);
            dsrc = r->d_a;
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        for (int k = 0; k < S && e == hipSuccess; ++k) {
            const bool last = (S - 1 - k) % 2 == 0;
            double* ddst = a->resident ? (last ? a->out : r->d_a) : (k % 2 == 0 ? r->d_b : r->d_a);
            double* hdst = a->resident ? (k % 2 == 0 ? r->h_b : r->h_a)
                                       : (last ? a->out : r->host_tmp.data());
            if (gpu_part)
                e = jacobi_gpu_sweep(gin, dsrc + (size_t)gb * plane, ddst + (size_t)gb * plane, nx,
                                     ny, nz - gb, s);
            if (e == hipSuccess && host_part)
                jacobi_host_sweeps(hin, hsrc, hdst, nullptr, nx, ny, hz, 1);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (host_part && gpu_part) {  // the new boundary planes cross
                copy(ddst + (size_t)(kc - 1) * plane, hdst + (size_t)(kc - 1) * plane, plane * 8,
                     hipMemcpyHostToDevice);
                copy(hdst + (size_t)kc * plane, ddst + (size_t)kc * plane, plane * 8,
                     hipMemcpyDeviceToHost);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
            }
            dsrc = ddst;
            hsrc = hdst;
        }
        // assemble: the other side's planes into the result
        if (a->resident && host_part)
            copy(a->out, hsrc, (size_t)kc * plane * 8, hipMemcpyHostToDevice);
        if (!a->resident && gpu_part)
            copy(a->out + (size_t)kc * plane, dsrc + (size_t)kc * plane,
                 (size_t)(nz - kc) * plane * 8, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(AO_EHIP, hip_msg("co-scheduled variant", e));
    }
    *secs = (double)(now_ns() - t0) * 1e-9;
    return AO_OK;
}

// The GPU launch plan of a Jacobi variant for S sweeps: one launch per
// sweep, or (families fusing P = 2, 3 or 4 sweeps per pass) one per P
// sweeps, the S mod P remaining sweeps first as one single register
// z-march sweep, one two-sweep or one three-sweep pass.  The one-point-per-
// thread family with AO_VF_LDS_SWEEPS runs a grid of at most 8192 points in
// one workgroup's LDS, all S sweeps in one launch (only for a block shape
// its sweep kernel accepts).
struct JacobiPlan {
    int P = 1;            // sweeps per full launch
    int rem = 0;          // sweeps of the first launch when S mod P != 0
    int launches = 0;     // 0 for S = 0
    bool lds_all = false;
};

JacobiPlan jacobi_plan(const ao_variant& v, int nx, int ny, int nz, int S) {
    JacobiPlan p;
    p.P = v.family == AO_FAM_JACOBI_ZREG_T2   ? 2
          : v.family == AO_FAM_JACOBI_ZREG_T3 ? 3
          : v.family == AO_FAM_JACOBI_ZREG_T4 ? 4
                                              : 1;
    p.rem = S % p.P;
    p.lds_all = v.family == AO_FAM_JACOBI_DIRECT && (v.flags & AO_VF_LDS_SWEEPS) && S >= 1 &&
                lds_sweeps_fit(nx, ny, nz) &&
                v.bx > 0 && v.by > 0 && (int64_t)v.bx * v.by <= 1024 && (v.bx * v.by) % 64 == 0;
    p.launches = S == 0 ? 0 : p.lds_all ? 1 : S / p.P + (p.rem ? 1 : 0);
    return p;
}

// Launch l of the plan: src -> dst.
hipError_t jacobi_launch(const ao_variant& v, const JacobiPlan& p, int l, const double* src,
                         double* dst, int nx, int ny, int nz, int S, hipStream_t s) {
    if (p.lds_all) return jacobi_gpu_lds_sweeps(src, dst, nx, ny, nz, S, s);
    if (p.P == 1) return jacobi_gpu_sweep(v, src, dst, nx, ny, nz, s);
    // the first launch of a fused family takes the S mod P remaining sweeps
    // with the largest row count per wave, not above the variant's, that
    // its family is built for
    if (l == 0 && p.rem > 0) {
        if (p.rem == 1) {
            const int rows = v.by >= 8 ? 8 : v.by >= 4 ? 4 : v.by >= 2 ? 2 : 1;
            const ao_variant one{AO_TARGET_GPU, AO_FAM_JACOBI_ZREG, 64, rows, v.bz,
                                 v.flags & (AO_VF_NT_STORE | AO_VF_FILL_Z)};
            return jacobi_gpu_sweep(one, src, dst, nx, ny, nz, s);
        }
        if (p.rem == 2) {
            int rows = v.by;
            while (rows > 1 && !t2_rows_ok(rows)) --rows;
            const ao_variant two{AO_TARGET_GPU, AO_FAM_JACOBI_ZREG_T2, 64, rows, v.bz,
                                 v.flags & (AO_VF_NT_STORE | AO_VF_FILL_Z)};
            return jacobi_gpu_double_sweep(two, src, dst, nx, ny, nz, s);
        }
        int rows = v.by;
        while (rows > 1 && !t3_rows_ok(rows)) --rows;
        const ao_variant three{AO_TARGET_GPU, AO_FAM_JACOBI_ZREG_T3, 64, rows, v.bz,
                               v.flags & (AO_VF_NT_STORE | AO_VF_FILL_Z)};
        return jacobi_gpu_multi_sweep(three, src, dst, nx, ny, nz, s);
    }
    return p.P == 2 ? jacobi_gpu_double_sweep(v, src, dst, nx, ny, nz, s)
                    : jacobi_gpu_multi_sweep(v, src, dst, nx, ny, nz, s);
}

// Enqueue S sweeps of GPU variant v from u0 into out (device buffers of N
// doubles).  Launch k writes out when L-1-k is even and scratch otherwise,
// so the last launch lands in out; scratch (N doubles) is read only after
// a launch has written all of it and is unused when L <= 1.  S = 0 copies.
hipError_t jacobi_gpu_resident(const ao_variant& v, const double* u0, double* out,
                               double* scratch, int nx, int ny, int nz, int S, hipStream_t s) {
    const size_t n = (size_t)nx * ny * nz;
    if (n == 0) return hipSuccess;
    if (S == 0) return hipMemcpyAsync(out, u0, n * 8, hipMemcpyDeviceToDevice, s);
    const JacobiPlan p = jacobi_plan(v, nx, ny, nz, S);
    if (p.launches > 1 && !scratch) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    const double* src = u0;
    for (int k = 0; k < p.launches && e == hipSuccess; ++k) {
        double* dst = ((p.launches - 1 - k) % 2 == 0) ? out : scratch;
        e = jacobi_launch(v, p, k, src, dst, nx, ny, nz, S, s);
        src = dst;
    }
    return e;
}

// The same, alternating between two device buffers a -> b -> a ...: the
// result lands in b when the launch count is odd and in a otherwise (a
// holds the input and is overwritten from the second launch on).
hipError_t jacobi_gpu_swap(const ao_variant& v, double* a, double* b, int nx, int ny, int nz,
                           int S, hipStream_t s, bool* in_b) {
    const JacobiPlan p = jacobi_plan(v, nx, ny, nz, S);
    *in_b = p.launches % 2 == 1;
    hipError_t e = hipSuccess;
    for (int k = 0; k < p.launches && e == hipSuccess; ++k) {
        e = jacobi_launch(v, p, k, a, b, nx, ny, nz, S, s);
        std::swap(a, b);
    }
    return e;
}

// Enqueue / run variant `vid` once.  When `sync` is set the call waits and
// returns the time in *secs; otherwise GPU timings are left pending with
// record index `rec` (host variants always return *secs).
int run_variant(ao_region* r, int vid, const ao_args* a, hipStream_t s, bool sync, double* secs,
                bool* pending_out, hipEvent_t* ev_a, hipEvent_t* ev_b) {
    const ao_variant& v = r->variants[vid];
    *secs = NAN;
    *pending_out = false;
    if (r->kind == AO_JACOBI7_F64) {
        const int nx = a->nx, ny = a->ny, nz = a->nz, S = a->sweeps;
        const size_t n = (size_t)nx * ny * nz;
        if (v.family == AO_FAM_JACOBI_COSCHED) return run_cosched(r, v, a, s, secs);
        if (v.target == AO_TARGET_GPU) {
            int rc = ensure_dev(r, std::max<size_t>(n, 1));
            if (rc) return rc;
            hipEvent_t e0 = get_event(r), e1 = get_event(r);
            if (!e0 || !e1) return fail(AO_EHIP, "event creation failed");
            hipError_t e = hipEventRecord(e0, s);
            if (e == hipSuccess && n > 0) {
                if (a->resident) {
                    e = jacobi_gpu_resident(v, a->u0, a->out, r->d_a, nx, ny, nz, S, s);
                } else {
                    // staged through the region's two device buffers
                    bool in_b = false;
                    e = hipMemcpyAsync(r->d_a, a->u0, n * 8, hipMemcpyHostToDevice, s);
                    if (e == hipSuccess) e = jacobi_gpu_swap(v, r->d_a, r->d_b, nx, ny, nz, S, s,
                                                             &in_b);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(a->out, in_b ? r->d_b : r->d_a, n * 8,
                                           hipMemcpyDeviceToHost, s);
                }
            }
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e != hipSuccess) {
                r->pool.push_back(e0);
                r->pool.push_back(e1);
                (void)hipGetLastError();
                const bool launch = (e == hipErrorInvalidConfiguration ||
                                     e == hipErrorInvalidValue || e == hipErrorLaunchFailure);
                if (launch) {
                    r->failed_mask |= 1 << vid;
                    return fail(AO_ELAUNCH, "variant " + std::to_string(vid) +
                                                " cannot launch (masked out): " +
                                                hipGetErrorString(e));
                }
                return fail(AO_EHIP, hip_msg("GPU variant", e));
            }
            if (sync) {
                hipEventSynchronize(e1);
                float ms = 0.0f;
                hipEventElapsedTime(&ms, e0, e1);
                *secs = (double)ms * 1e-3;
                r->pool.push_back(e0);
                r->pool.push_back(e1);
            } else {
                *pending_out = true;
                *ev_a = e0;
                *ev_b = e1;
            }
            return AO_OK;
        }
        // host variant.  Device-resident data (or an explicit stream): drain
        // the stream first.  Host-resident data on the null stream runs at
        // once, without touching the GPU.
        hipError_t e = hipSuccess;
        if (a->resident || s != nullptr) {
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return fail(AO_EHIP, hip_msg("stream sync", e));
        }
        const uint64_t t0 = now_ns();
        if (n > 0) {
            if (a->resident) {
                int rc = ensure_host(r, n);
                if (rc) return rc;
                e = hipMemcpyAsync(r->h_a, a->u0, n * 8, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return fail(AO_EHIP, hip_msg("D2H", e));
                double* p = r->h_a;
                double* q = r->h_b;
                if (S == 0) {
                    // result is the input itself
                } else {
                    // ping-pong between the two pinned buffers
                    ao_variant hv = v;
                    for (int k = 0; k < S; ++k) {
                        jacobi_host_sweeps(hv, p, q, nullptr, nx, ny, nz, 1);
                        std::swap(p, q);
                    }
                }
                e = hipMemcpyAsync(a->out, p, n * 8, hipMemcpyHostToDevice, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return fail(AO_EHIP, hip_msg("H2D", e));
            } else {
                if (S >= 2 && r->host_tmp.size() < n) r->host_tmp.assign(n, 0.0);
                jacobi_host_sweeps(v, a->u0, a->out, r->host_tmp.data(), nx, ny, nz, S);
            }
        }
        *secs = (double)(now_ns() - t0) * 1e-9;
        return AO_OK;
    }
    // SpMV
    int rc = AO_OK;
    SpmvPlan* p = get_plan(r, a, s, &rc);
    if (!p) return rc;
    hipEvent_t e0 = get_event(r), e1 = get_event(r);
    if (!e0 || !e1) return fail(AO_EHIP, "event creation failed");
    // the x-slice family's reordered values are reused while the caller's
    // values id (nonzero) and value array stay the same
    SpmvPlan::XSlice* xq = nullptr;
    if (v.family == AO_FAM_SPMV_XSLICE)
        for (auto& q : p->xs)
            if (q.swl == (v.by == 0 ? 14 : v.by)) xq = &q;
    const bool cached = xq && a->values_id != 0 && xq->values_id == a->values_id &&
                        xq->values_of == a->val;
    if (xq) {
        xq->values_id = 0;  // until this call's copy is enqueued
        xq->values_of = nullptr;
    }
    hipError_t e = hipEventRecord(e0, s);
    if (r->kind == AO_CSR_SPMV_F64) {
        if (e == hipSuccess) e = spmv_gpu(v, *p, a->col, a->val, a->x, a->y, s, SpmvEpi(), cached);
    } else {
        // relaxation: S sweeps ping-ponging between y and the region's
        // scratch so that the last one lands in y
        const int S = a->sweeps;
        const size_t n = (size_t)std::max(a->n, 0);
        if (S > 1) {
            const int rc2 = ensure_dev(r, std::max<size_t>(n, 1));
            if (rc2) {
                r->pool.push_back(e0);
                r->pool.push_back(e1);
                return rc2;
            }
        }
        SpmvEpi ep;
        ep.b = a->b;
        ep.d = a->diag;
        ep.omega = a->omega;
        if (S == 0 && n > 0 && e == hipSuccess)
            e = hipMemcpyAsync(a->y, a->x, n * 8, hipMemcpyDeviceToDevice, s);
        const double* src = a->x;
        for (int k = 0; k < S && e == hipSuccess; ++k) {
            double* dst = ((S - 1 - k) % 2 == 0) ? a->y : r->d_a;
            e = spmv_gpu(v, *p, a->col, a->val, src, dst, s, ep, cached || k > 0);
            src = dst;
        }
    }
    if (e == hipSuccess && xq && a->values_id != 0) {
        xq->values_id = a->values_id;
        xq->values_of = a->val;
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e != hipSuccess) {
        r->pool.push_back(e0);
        r->pool.push_back(e1);
        (void)hipGetLastError();
        if (e == hipErrorInvalidConfiguration || e == hipErrorInvalidValue) {
            r->failed_mask |= 1 << vid;
            return fail(AO_ELAUNCH, "variant " + std::to_string(vid) +
                                        " cannot launch (masked out): " + hipGetErrorString(e));
        }
        return fail(AO_EHIP, hip_msg("SpMV variant", e));
    }
    if (sync) {
        hipEventSynchronize(e1);
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        *secs = (double)ms * 1e-3;
        r->pool.push_back(e0);
        r->pool.push_back(e1);
    } else {
        *pending_out = true;
        *ev_a = e0;
        *ev_b = e1;
    }
    return AO_OK;
}

size_t append_record(ao_region* r, const float* f, int vid, int resident, double secs) {
    Record rec;
    memcpy(rec.f, f, sizeof(rec.f));
    rec.variant = vid;
    rec.resident = resident;
    rec.seconds = secs;
    rec.t_ns = now_ns();
    r->db.push_back(rec);
    r->uniq.insert(UKey{make_key(f), vid});
    return r->db.size() - 1;
}

// Time each variant in `ids` (warmup + reps, median) -> med[v].
int profile_variants(ao_region* r, const ao_args* a, const float* f, const std::vector<int>& ids,
                     int warmup, int reps, hipStream_t s, bool record, double* med) {
    for (int vid : ids) {
        med[vid] = INFINITY;
        if (r->failed_mask & (1 << vid)) continue;
        bool pend;
        hipEvent_t ea, eb;
        double t;
        int rc = AO_OK;
        for (int w = 0; w < warmup && rc == AO_OK; ++w)
            rc = run_variant(r, vid, a, s, true, &t, &pend, &ea, &eb);
        std::vector<double> ts;
        for (int k = 0; k < reps && rc == AO_OK; ++k) {
            rc = run_variant(r, vid, a, s, true, &t, &pend, &ea, &eb);
            if (rc == AO_OK) {
                ts.push_back(t);
                if (record) append_record(r, f, vid, a->resident, t);
            }
        }
        if (rc == AO_ELAUNCH) continue;  // masked; keep +inf
        if (rc != AO_OK) return rc;
        med[vid] = median_of(ts);
    }
    return AO_OK;
}

int argmin_allowed(const double* med, int V) {
    int best = -1;
    for (int v = 0; v < V; ++v)
        if (std::isfinite(med[v]) && (best < 0 || med[v] < med[best])) best = v;
    return best;
}

int next_explore(ao_region* r, bool advance) {
    const int V = (int)r->variants.size();
    int64_t k = r->rr;
    for (int t = 0; t < V; ++t, ++k) {
        const int v = (int)(k % V);
        if (!(r->failed_mask & (1 << v))) {
            if (advance) r->rr = k + 1;
            return v;
        }
    }
    return -1;
}

int ensure_sel_staging(ao_region* r, int batch) {
    if (!r->sel_stream) {
        hipError_t e = hipStreamCreateWithFlags(&r->sel_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(AO_EHIP, hip_msg("selector stream", e));
    }
    if (r->sel_cap >= batch) return AO_OK;
    if (r->h_feat) hipHostFree(r->h_feat);
    if (r->h_ids) hipHostFree(r->h_ids);
    r->h_feat = nullptr;
    r->h_ids = nullptr;
    const int cap = std::max(batch, 64);
    hipError_t e = hipHostMalloc(&r->h_feat, (size_t)cap * AO_MAX_FEATURES * sizeof(float),
                                 hipHostMallocMapped);
    if (e == hipSuccess) e = hipHostMalloc(&r->h_ids, (size_t)cap * sizeof(int32_t),
                                           hipHostMallocMapped);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&r->m_feat, r->h_feat, 0);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&r->m_ids, r->h_ids, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        r->sel_cap = 0;
        return fail(AO_ENOMEM, hip_msg("selector staging", e));
    }
    r->sel_cap = cap;
    return AO_OK;
}

// Model inference for `batch` feature vectors -> ids (argmin over allowed
// variants); returns AO_OK, or AO_NOTE_FALLBACK if the model produced a
// non-finite prediction (the model is then dropped).
int infer(ao_region* r, const float* feats, int batch, int* ids) {
    int rc = ensure_sel_staging(r, batch);
    if (rc) return rc;
    memcpy(r->h_feat, feats, (size_t)batch * AO_MAX_FEATURES * sizeof(float));
    const int V = (int)r->variants.size();
    const int allowed = ((1 << V) - 1) & ~r->failed_mask;
    hipError_t e = mlp_select_launch(r->d_params, r->d_norm, r->m_feat, batch, V, allowed,
                                     r->m_ids, nullptr, r->sel_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->sel_stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(AO_EHIP, hip_msg("selector inference", e));
    }
    bool bad = false;
    for (int b = 0; b < batch; ++b) {
        ids[b] = r->h_ids[b];
        if (ids[b] < 0 || ids[b] >= V) bad = true;
    }
    if (bad) {
        r->trained = false;
        r->memo.clear();
        set_error("model produced a non-finite prediction; model dropped");
        return AO_NOTE_FALLBACK;
    }
    return AO_OK;
}

bool out_of_range(const ao_region* r, const float* f) {
    for (int i = 0; i < AO_MAX_FEATURES; ++i) {
        const float span = std::max(1.0f, r->fmax[i] - r->fmin[i]);
        if (!std::isfinite(f[i]) || f[i] < r->fmin[i] - 0.25f * span ||
            f[i] > r->fmax[i] + 0.25f * span)
            return true;
    }
    return false;
}

int exhaustive_choice(ao_region* r, const ao_args* a, const float* f, hipStream_t s, int warmup,
                      int reps, int* vid) {
    const int V = (int)r->variants.size();
    std::vector<int> ids(V);
    for (int v = 0; v < V; ++v) ids[v] = v;
    std::vector<double> med(V, INFINITY);
    int rc = profile_variants(r, a, f, ids, warmup, reps, s, true, med.data());
    if (rc) return rc;
    *vid = argmin_allowed(med.data(), V);
    if (*vid < 0) return fail(AO_ELAUNCH, "no variant of the region can run");
    return AO_OK;
}

int train_locked(ao_region* r, const ao_train_opts* opts, double* final_loss);

// Train trigger at the end of an execution (Sec. 3.3): enough unique
// samples and no model yet.  A failed training is retried once the unique
// count has doubled.
void maybe_train(ao_region* r) {
    const int64_t nu = (int64_t)r->uniq.size();
    const bool learns = r->model_type == "mlp" || r->dtree_depth > 0;
    if (learns && !r->trained && nu >= r->min_train && nu >= r->retrain_at) {
        if (train_locked(r, nullptr, nullptr) < 0) {
            r->train_failures += 1;
            r->retrain_at = 2 * nu;
        }
    }
}

}  // namespace
}  // namespace ao

ao_region::~ao_region() {
    harvest(this, true);
    for (hipEvent_t e : pool) hipEventDestroy(e);
    if (d_a) hipFree(d_a);
    if (d_b) hipFree(d_b);
    if (h_a) hipHostFree(h_a);
    if (h_b) hipHostFree(h_b);
    if (d_params) hipFree(d_params);
    if (d_norm) hipFree(d_norm);
    if (h_feat) hipHostFree(h_feat);
    if (h_ids) hipHostFree(h_ids);
    if (sel_stream) hipStreamDestroy(sel_stream);
}

SpmvPlan::~SpmvPlan() {
    for (auto& m : mp)
        if (m.srow) hipFree(m.srow);
    for (auto& q : xs) q.release();
    if (unit_ptr) hipFree(unit_ptr);
    if (unit_sums) hipFree(unit_sums);
}

// --------------------------------------------------------------------------
// Training (selector_train): dataset from the database, GPU trainer kernel
// --------------------------------------------------------------------------
namespace ao {
namespace {

// Decision tree: one sample per distinct feature tuple, labelled with its
// fastest variant (median per variant, ties to the lowest id).
int train_dtree(ao_region* r, double* final_loss) {
    const uint64_t t0 = now_ns();
    std::unordered_map<FeatKey, std::vector<std::vector<double>>, FeatKeyHash> by;
    std::vector<FeatKey> order;
    std::unordered_map<FeatKey, const Record*, FeatKeyHash> first;
    const int V = (int)r->variants.size();
    for (const Record& rec : r->db) {
        if (!std::isfinite(rec.seconds) || rec.seconds <= 0.0) continue;
        const FeatKey k = make_key(rec.f);
        auto it = by.find(k);
        if (it == by.end()) {
            it = by.emplace(k, std::vector<std::vector<double>>(V)).first;
            order.push_back(k);
            first[k] = &rec;
        }
        it->second[rec.variant].push_back(rec.seconds);
    }
    if (order.empty()) return fail(AO_ESTATE, "no usable profile records to train on");
    std::vector<std::vector<float>> feats;
    std::vector<int> labels;
    for (const FeatKey& k : order) {
        int best = -1;
        double bt = INFINITY;
        for (int v = 0; v < V; ++v) {
            const double m = median_of(by[k][v]);
            if (m < bt) {
                bt = m;
                best = v;
            }
        }
        if (best < 0) continue;
        feats.emplace_back(first[k]->f, first[k]->f + AO_MAX_FEATURES);
        labels.push_back(best);
    }
    r->tree.train(feats, labels, r->dtree_depth, V);
    int hits = 0;
    for (size_t q = 0; q < feats.size(); ++q)
        hits += r->tree.predict(feats[q].data(), (1 << V) - 1) == labels[q];
    r->trained = true;
    r->trainings += 1;
    r->memo.clear();
    r->last_train_seconds = (double)(now_ns() - t0) * 1e-9;
    if (final_loss) *final_loss = 1.0 - (double)hits / (double)feats.size();  // training error
    return AO_OK;
}

int train_locked(ao_region* r, const ao_train_opts* opts, double* final_loss) {
    harvest(r, true);
    if (r->dtree_depth > 0) return train_dtree(r, final_loss);
    ao_train_opts o{200, 256, 1e-3f, 7};
    if (opts) o = *opts;
    if (o.epochs < 0 || o.batch <= 0 || !(o.lr > 0.0f))
        return fail(AO_EINVAL, "bad training options");
    // merge duplicate (features, variant) samples by median, first-seen order
    std::unordered_map<UKey, size_t, UKeyHash> idx;
    std::vector<std::vector<double>> times;
    std::vector<const Record*> first;
    for (const Record& rec : r->db) {
        if (!std::isfinite(rec.seconds) || rec.seconds <= 0.0) continue;
        UKey k{make_key(rec.f), rec.variant};
        auto it = idx.find(k);
        if (it == idx.end()) {
            idx.emplace(k, first.size());
            first.push_back(&rec);
            times.push_back({rec.seconds});
        } else {
            times[it->second].push_back(rec.seconds);
        }
    }
    const int n = (int)first.size();
    if (n < 1) return fail(AO_ESTATE, "no usable profile records to train on");
    std::vector<double> F((size_t)n * AO_MAX_FEATURES), lt(n);
    std::vector<int32_t> var(n);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < AO_MAX_FEATURES; ++j) F[(size_t)i * AO_MAX_FEATURES + j] = first[i]->f[j];
        var[i] = first[i]->variant;
        lt[i] = log(median_of(times[i]));
    }
    MlpNorm norm{};
    double ymean = 0.0;
    for (int i = 0; i < n; ++i) ymean += lt[i];
    ymean /= n;
    float fmin[AO_MAX_FEATURES], fmax[AO_MAX_FEATURES];
    for (int j = 0; j < AO_MAX_FEATURES; ++j) {
        double mu = 0.0;
        fmin[j] = INFINITY;
        fmax[j] = -INFINITY;
        for (int i = 0; i < n; ++i) {
            const double v = F[(size_t)i * AO_MAX_FEATURES + j];
            mu += v;
            fmin[j] = std::min(fmin[j], (float)v);
            fmax[j] = std::max(fmax[j], (float)v);
        }
        mu /= n;
        double var2 = 0.0;
        for (int i = 0; i < n; ++i) {
            const double d = F[(size_t)i * AO_MAX_FEATURES + j] - mu;
            var2 += d * d;
        }
        norm.mu[j] = (float)mu;
        norm.sd[j] = (float)std::max(sqrt(var2 / n), 1e-6);
    }
    norm.y_mean = (float)ymean;
    std::vector<float> X((size_t)n * AO_MAX_FEATURES), Y(n);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < AO_MAX_FEATURES; ++j)
            X[(size_t)i * AO_MAX_FEATURES + j] =
                (float)((F[(size_t)i * AO_MAX_FEATURES + j] - norm.mu[j]) / norm.sd[j]);
        Y[i] = (float)(lt[i] - ymean);
    }
    // epoch shuffles: indices ordered by SplitMix64 keys (stable on ties)
    std::vector<int32_t> perm(std::max<size_t>((size_t)o.epochs * n, 1));
    std::vector<std::pair<uint64_t, int32_t>> keyed(n);
    for (int e = 0; e < o.epochs; ++e) {
        const uint64_t es = splitmix_mix(((o.seed << 8) | (uint64_t)(e & 0xFF))) ^ (uint64_t)(e >> 8);
        for (int i = 0; i < n; ++i) keyed[i] = {splitmix_at(es, (uint64_t)i + 1), i};
        std::stable_sort(keyed.begin(), keyed.end(),
                         [](const auto& x, const auto& y) { return x.first < y.first; });
        for (int i = 0; i < n; ++i) perm[(size_t)e * n + i] = keyed[i].second;
    }
    // He-uniform init from SplitMix64(seed), W1, W2, W3 in flat order; zero biases
    std::vector<float> theta(AO_MLP_PARAMS, 0.0f);
    {
        const int sizes[3][2] = {{64, 6}, {64, 64}, {12, 64}};
        const int offs[3] = {0, 6 * 64 + 64, 6 * 64 + 64 + 64 * 64 + 64};
        uint64_t draw = 1;
        for (int l = 0; l < 3; ++l) {
            const double bound = sqrt(6.0 / sizes[l][1]);
            for (int q = 0; q < sizes[l][0] * sizes[l][1]; ++q) {
                const double u = (double)(splitmix_at(o.seed, draw++) >> 11) * 0x1p-53;
                theta[offs[l] + q] = (float)((2.0 * u - 1.0) * bound);
            }
        }
    }
    float *dX = nullptr, *dY = nullptr, *dP = nullptr, *dL = nullptr, *dMV = nullptr;
    int32_t *dV = nullptr, *dPerm = nullptr;
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    auto cleanup = [&]() {
        if (dX) hipFree(dX);
        if (dY) hipFree(dY);
        if (dP) hipFree(dP);
        if (dL) hipFree(dL);
        if (dMV) hipFree(dMV);
        if (dV) hipFree(dV);
        if (dPerm) hipFree(dPerm);
        if (s) hipStreamDestroy(s);
    };
    const uint64_t t0 = now_ns();
    if (e == hipSuccess) e = hipMalloc(&dX, X.size() * 4);
    if (e == hipSuccess) e = hipMalloc(&dY, (size_t)n * 4);
    if (e == hipSuccess) e = hipMalloc(&dV, (size_t)n * 4);
    if (e == hipSuccess) e = hipMalloc(&dPerm, perm.size() * 4);
    if (e == hipSuccess) e = hipMalloc(&dP, AO_MLP_PARAMS * 4);
    if (e == hipSuccess) e = hipMalloc(&dL, (size_t)std::max(o.epochs, 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&dMV, (size_t)2 * AO_MLP_PARAMS * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(dX, X.data(), X.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dY, Y.data(), (size_t)n * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dV, var.data(), (size_t)n * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dPerm, perm.data(), perm.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dP, theta.data(), AO_MLP_PARAMS * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && o.epochs > 0)
        e = mlp_train_launch(dP, dX, dY, dV, dPerm, n, o.epochs, o.batch, o.lr, dMV, dL, s);
    std::vector<float> losses(std::max(o.epochs, 1), NAN);
    if (e == hipSuccess)
        e = hipMemcpyAsync(theta.data(), dP, AO_MLP_PARAMS * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && o.epochs > 0)
        e = hipMemcpyAsync(losses.data(), dL, (size_t)o.epochs * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(AO_EHIP, hip_msg("training", e));
    }
    cleanup();
    bool finite = true;
    for (float v : theta) finite = finite && std::isfinite(v);
    if (!finite || (o.epochs > 0 && !std::isfinite(losses.back()))) {
        r->trained = false;
        return fail(AO_ESTATE, "training diverged (non-finite weights); model not installed");
    }
    if (!r->d_params) {
        e = hipMalloc(&r->d_params, AO_MLP_PARAMS * 4);
        if (e == hipSuccess) e = hipMalloc(&r->d_norm, sizeof(MlpNorm));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(AO_ENOMEM, hip_msg("model buffers", e));
        }
    }
    e = hipMemcpy(r->d_params, theta.data(), AO_MLP_PARAMS * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_norm, &norm, sizeof(MlpNorm), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(AO_EHIP, hip_msg("model upload", e));
    }
    r->params = theta;
    r->norm = norm;
    memcpy(r->fmin, fmin, sizeof(fmin));
    memcpy(r->fmax, fmax, sizeof(fmax));
    r->trained = true;
    r->trainings += 1;
    r->memo.clear();
    r->last_train_seconds = (double)(now_ns() - t0) * 1e-9;
    if (final_loss) *final_loss = losses.back();
    return AO_OK;
}

uint32_t crc32_update(uint32_t crc, const void* data, size_t len) {
    const uint8_t* p = (const uint8_t*)data;
    crc = ~crc;
    for (size_t i = 0; i < len; ++i) {
        crc ^= p[i];
        for (int k = 0; k < 8; ++k) crc = (crc >> 1) ^ (0xEDB88320u & (0u - (crc & 1u)));
    }
    return ~crc;
}

struct Writer {
    std::vector<uint8_t> buf;
    void put(const void* p, size_t n) {
        const uint8_t* b = (const uint8_t*)p;
        buf.insert(buf.end(), b, b + n);
    }
    template <class T>
    void put(const T& v) {
        put(&v, sizeof(T));
    }
};

struct Reader {
    const uint8_t* p;
    size_t n, off = 0;
    bool ok = true;
    void get(void* dst, size_t k) {
        if (!ok || off + k > n) {
            ok = false;
            return;
        }
        memcpy(dst, p + off, k);
        off += k;
    }
    template <class T>
    T get() {
        T v{};
        get(&v, sizeof(T));
        return v;
    }
};

const char kMagic[8] = {'A', 'O', 'M', 'P', 'D', 'B', 0, 1};

}  // namespace
}  // namespace ao

// ==========================================================================
// C ABI
namespace ao {

// Scratch of the allocation-free entry point: the ping-pong array between
// the launches of one region execution.  One copy per GPU, held from the
// library's first use of that GPU until the process ends.  Host code never
// passes this name to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocScratchBytes = (size_t)AO_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int noalloc_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(AO_EHIP, hip_msg("current device", e));
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(AO_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(AO_EHIP, hip_msg("static scratch address", e));
        }
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return AO_OK;
}

}  // namespace
}  // namespace ao

// ==========================================================================
extern "C" {

const char* ao_last_error(void) { return g_err.c_str(); }

int ao_hbm_copy(const double* src, double* dst, int64_t n, int nontemporal, void* stream) {
    if (n < 0 || (n > 0 && (!src || !dst))) return fail(AO_EINVAL, "bad arguments");
    hipError_t e = hbm_copy(src, dst, n, nontemporal != 0, (hipStream_t)stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorInvalidValue ? AO_EINVAL : AO_EHIP,
                    hip_msg("copy (buffers must be 16-byte aligned)", e));
    }
    return AO_OK;
}

int ao_gather_probe(const int32_t* idx, const double* x, int64_t m, int64_t nx, double* out,
                    void* stream) {
    if (m < 0 || nx <= 0 || (m > 0 && (!idx || !x || !out)))
        return fail(AO_EINVAL, "bad arguments");
    hipError_t e = gather_probe(idx, x, m, nx, out, (hipStream_t)stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(AO_EHIP, hip_msg("gather probe", e));
    }
    return AO_OK;
}

int ao_jacobi_planes(const ao_variant* v, int32_t nx, int32_t ny, int32_t nz, int32_t cus,
                     int32_t blocks_per_cu, int32_t* planes) {
    if (!v || !planes || nx <= 0 || ny <= 0 || nz <= 0 || v->target != AO_TARGET_GPU ||
        (cus > 0 && blocks_per_cu < 1))
        return fail(AO_EINVAL, "bad arguments");
    int p = 0;
    const hipError_t e = jacobi_gpu_planes(*v, nx, ny, nz, cus, blocks_per_cu, &p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(AO_EINVAL, "not a register z-march variant that fits its kernels");
    }
    *planes = p;
    return AO_OK;
}

int ao_device_cus(void) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return cus;
}

int region_declare_variants(const char* model_name, int kind, const ao_variant* variants,
                            int num_variants, int min_train_data, const char* model_type,
                            ao_region** out) {
    if (!model_name || !*model_name) return fail(AO_EINVAL, "model_name is required");
    if (!out) return fail(AO_EINVAL, "out is NULL");
    if (kind != AO_JACOBI7_F64 && kind != AO_CSR_SPMV_F64 && kind != AO_CSR_RELAX_F64)
        return fail(AO_EINVAL, "unknown region kind");
    if (!variants || num_variants < 1 || num_variants > AO_MAX_VARIANTS)
        return fail(AO_EINVAL, "need 1..12 variants");
    const std::string mt = model_type ? model_type : "mlp";
    int depth = 0;
    if (mt == "dtree") {
        depth = 2;  // the paper's default depth
    } else if (mt.rfind("dtree,", 0) == 0) {
        depth = atoi(mt.c_str() + 6);
        if (depth < 1 || depth > 16) return fail(AO_EINVAL, "dtree depth must be 1..16");
    } else if (mt != "mlp" && mt != "exhaustive" && mt != "roundrobin") {
        return fail(AO_EINVAL, "model_type must be mlp, dtree[,depth], exhaustive or roundrobin");
    }
    for (int i = 0; i < num_variants; ++i) {
        int rc = validate_variant(kind, variants[i], i);
        if (rc) return rc;
    }
    const int mtd = min_train_data > 0 ? min_train_data : num_variants;
    std::lock_guard<std::mutex> g(g_reg_mu);
    auto it = g_regions.find(model_name);
    if (it != g_regions.end()) {
        ao_region* r = it->second;
        bool same = r->kind == kind && (int)r->variants.size() == num_variants &&
                    r->min_train == mtd && r->model_type == mt;
        for (int i = 0; same && i < num_variants; ++i) same = same_variant(r->variants[i], variants[i]);
        if (!same) return fail(AO_EEXIST, "model name already declared with a different spec");
        *out = r;
        return AO_OK;
    }
    ao_region* r = new (std::nothrow) ao_region();
    if (!r) return fail(AO_ENOMEM, "region allocation");
    r->name = model_name;
    r->kind = kind;
    r->variants.assign(variants, variants + num_variants);
    r->min_train = mtd;
    r->model_type = mt;
    r->dtree_depth = depth;
    if (hipGetDevice(&r->device) != hipSuccess) {
        (void)hipGetLastError();
        r->device = -1;
    }
    g_regions[r->name] = r;
    *out = r;
    return AO_OK;
}

int region_run(ao_region* r, const ao_args* a, const float* features, void* stream, int variant,
               int* chosen) {
    if (!r) return fail(AO_EINVAL, "region is NULL");
    std::lock_guard<std::mutex> g(r->mu);
    int rc = validate_args(r, a);
    if (rc) return rc;
    const int V = (int)r->variants.size();
    if (variant < -1 || variant >= V) return fail(AO_EINVAL, "variant id out of range");
    hipStream_t s = (hipStream_t)stream;
    harvest(r, false);
    float f[AO_MAX_FEATURES];
    if (features) {
        memcpy(f, features, sizeof(f));
    } else {
        rc = compute_features(r, a, s, f);
        if (rc) return rc;
    }
    int status = AO_OK;
    int vid = variant;
    if (vid < 0) {
        const FeatKey key = make_key(f);
        if (r->model_type == "exhaustive") {
            auto it = r->memo.find(key);
            if (it != r->memo.end() && !(r->failed_mask & (1 << it->second))) {
                vid = it->second;
            } else {
                rc = exhaustive_choice(r, a, f, s, 1, 3, &vid);
                if (rc) return rc;
                r->memo[key] = vid;
            }
        } else if (r->dtree_depth > 0 && r->trained) {
            auto it = r->memo.find(key);
            if (it != r->memo.end() && !(r->failed_mask & (1 << it->second))) {
                vid = it->second;
            } else {
                const int V = (int)r->variants.size();
                vid = r->tree.predict(f, ((1 << V) - 1) & ~r->failed_mask);
                if (vid < 0) {
                    rc = exhaustive_choice(r, a, f, s, 0, 1, &vid);
                    if (rc) return rc;
                    r->fallbacks += 1;
                    status = AO_NOTE_FALLBACK;
                }
                r->memo[key] = vid;
            }
        } else if (r->model_type == "mlp" && r->trained) {
            auto it = r->memo.find(key);
            if (it != r->memo.end() && !(r->failed_mask & (1 << it->second))) {
                vid = it->second;
            } else if (out_of_range(r, f)) {
                rc = exhaustive_choice(r, a, f, s, 0, 1, &vid);
                if (rc) return rc;
                r->memo[key] = vid;
                r->fallbacks += 1;
                status = AO_NOTE_FALLBACK;
            } else {
                int q = infer(r, f, 1, &vid);
                if (q < 0) return q;
                if (q == AO_NOTE_FALLBACK) {
                    rc = exhaustive_choice(r, a, f, s, 0, 1, &vid);
                    if (rc) return rc;
                    r->fallbacks += 1;
                    status = AO_NOTE_FALLBACK;
                }
                r->memo[key] = vid;
            }
        } else {
            vid = next_explore(r, true);
            if (vid < 0) return fail(AO_ELAUNCH, "no variant of the region can run");
            status = AO_NOTE_UNTRAINED;
        }
    } else if (r->failed_mask & (1 << vid)) {
        return fail(AO_ELAUNCH, "variant " + std::to_string(vid) + " is masked out (failed launch)");
    }
    double secs;
    bool pend = false;
    hipEvent_t ea = nullptr, eb = nullptr;
    rc = run_variant(r, vid, a, s, false, &secs, &pend, &ea, &eb);
    if (rc) return rc;
    const size_t rec = append_record(r, f, vid, a->resident, pend ? NAN : secs);
    if (pend) r->pending.push_back(Pending{ea, eb, rec});
    if (chosen) *chosen = vid;
    maybe_train(r);
    return status;
}

int region_run_noalloc(ao_region* r, const ao_args* a, void* stream, int variant) {
    if (!r) return fail(AO_EINVAL, "region is NULL");
    std::lock_guard<std::mutex> g(r->mu);
    int rc = validate_args(r, a);
    if (rc) return rc;
    if (r->kind != AO_JACOBI7_F64)
        return fail(AO_EINVAL, "region_run_noalloc runs Jacobi regions only");
    if (variant < 0 || variant >= (int)r->variants.size())
        return fail(AO_EINVAL, "variant id out of range (the caller names the variant)");
    const ao_variant& v = r->variants[variant];
    if (v.target != AO_TARGET_GPU || v.family == AO_FAM_JACOBI_COSCHED)
        return fail(AO_EINVAL, "region_run_noalloc runs GPU variants only");
    if (a->resident != 1) return fail(AO_EINVAL, "region_run_noalloc needs device-resident buffers");
    if (r->failed_mask & (1 << variant))
        return fail(AO_ELAUNCH, "variant " + std::to_string(variant) + " is masked out (failed launch)");
    void* sp = nullptr;
    rc = noalloc_scratch(&sp);
    if (rc) return rc;
    const int nx = a->nx, ny = a->ny, nz = a->nz, S = a->sweeps;
    const size_t n = (size_t)nx * ny * nz;
    if (n == 0) return AO_OK;
    if (jacobi_plan(v, nx, ny, nz, S).launches > 1 && n * 8 > kNoallocScratchBytes)
        return fail(AO_EINVAL, "grid of " + std::to_string(n) + " points needs " +
                                   std::to_string(n * 8) + " bytes of scratch, above the " +
                                   std::to_string(kNoallocScratchBytes) +
                                   "-byte static array of region_run_noalloc");
    hipError_t e = jacobi_gpu_resident(v, a->u0, a->out, (double*)sp, nx, ny, nz, S,
                                       (hipStream_t)stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (e == hipErrorInvalidConfiguration || e == hipErrorInvalidValue ||
            e == hipErrorLaunchFailure) {
            r->failed_mask |= 1 << variant;
            return fail(AO_ELAUNCH, "variant " + std::to_string(variant) +
                                        " cannot launch (masked out): " + hipGetErrorString(e));
        }
        return fail(AO_EHIP, hip_msg("GPU variant", e));
    }
    return AO_OK;
}

int region_features(ao_region* r, const ao_args* a, void* stream, float* features) {
    if (!r || !features) return fail(AO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(r->mu);
    int rc = validate_args(r, a);
    if (rc) return rc;
    return compute_features(r, a, (hipStream_t)stream, features);
}

int region_record(ao_region* r, const float* features, int variant, double seconds) {
    if (!r || !features) return fail(AO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(r->mu);
    if (variant < 0 || variant >= (int)r->variants.size())
        return fail(AO_EINVAL, "variant id out of range");
    if (!(seconds > 0.0) || !std::isfinite(seconds)) return fail(AO_EINVAL, "seconds must be > 0");
    append_record(r, features, variant, -1, seconds);
    maybe_train(r);
    return AO_OK;
}

int region_profile(ao_region* r, const ao_args* a, const float* features, int variant, int warmup,
                   int reps, void* stream, int flags, double* median_seconds) {
    if (!r) return fail(AO_EINVAL, "region is NULL");
    if (!median_seconds) return fail(AO_EINVAL, "median_seconds is NULL");
    if (warmup < 0 || reps < 1) return fail(AO_EINVAL, "need warmup >= 0 and reps >= 1");
    std::lock_guard<std::mutex> g(r->mu);
    int rc = validate_args(r, a);
    if (rc) return rc;
    const int V = (int)r->variants.size();
    if (variant < -1 || variant >= V) return fail(AO_EINVAL, "variant id out of range");
    hipStream_t s = (hipStream_t)stream;
    float f[AO_MAX_FEATURES];
    if (features) {
        memcpy(f, features, sizeof(f));
    } else {
        rc = compute_features(r, a, s, f);
        if (rc) return rc;
    }
    std::vector<int> ids;
    if (variant < 0)
        for (int v = 0; v < V; ++v) ids.push_back(v);
    else
        ids.push_back(variant);
    std::vector<double> med(V, INFINITY);
    rc = profile_variants(r, a, f, ids, warmup, reps, s, (flags & AO_PROFILE_RECORD) != 0,
                          med.data());
    if (rc) return rc;
    if (variant < 0)
        for (int v = 0; v < V; ++v) median_seconds[v] = med[v];
    else
        median_seconds[0] = med[variant];
    return AO_OK;
}

int selector_train(ao_region* r, const ao_train_opts* opts, double* final_loss) {
    if (!r) return fail(AO_EINVAL, "region is NULL");
    std::lock_guard<std::mutex> g(r->mu);
    return train_locked(r, opts, final_loss);
}

int selector_select(ao_region* r, const float* features, int batch, int* variants_out) {
    if (!r) return fail(AO_EINVAL, "region is NULL");
    if (batch < 0 || (batch > 0 && (!features || !variants_out)))
        return fail(AO_EINVAL, "bad batch / buffers");
    std::lock_guard<std::mutex> g(r->mu);
    if (batch == 0) return AO_OK;
    if (r->trained && r->dtree_depth > 0) {
        const int V = (int)r->variants.size();
        const int allowed = ((1 << V) - 1) & ~r->failed_mask;
        bool ok = true;
        for (int b = 0; b < batch; ++b) {
            variants_out[b] = r->tree.predict(features + (size_t)b * AO_MAX_FEATURES, allowed);
            ok = ok && variants_out[b] >= 0;
        }
        if (ok) return AO_OK;
    } else if (r->trained) {
        int rc = infer(r, features, batch, variants_out);
        if (rc <= 0) return rc;
    }
    const int v = next_explore(r, false);
    if (v < 0) return fail(AO_ELAUNCH, "no variant of the region can run");
    for (int b = 0; b < batch; ++b) variants_out[b] = v;
    return r->trained ? AO_NOTE_FALLBACK : AO_NOTE_UNTRAINED;
}

int region_stats(ao_region* r, ao_stats* out) {
    if (!r || !out) return fail(AO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(r->mu);
    harvest(r, false);
    out->records = (int64_t)r->db.size();
    out->unique = (int64_t)r->uniq.size();
    out->trained = r->trained ? 1 : 0;
    out->num_variants = (int)r->variants.size();
    out->explore_next = r->rr;
    out->trainings = r->trainings;
    out->fallbacks = r->fallbacks;
    out->failed_mask = r->failed_mask;
    out->min_train = r->min_train;
    out->memo_size = (int64_t)r->memo.size();
    out->last_train_seconds = r->last_train_seconds;
    out->train_failures = r->train_failures;
    return AO_OK;
}

int region_records(ao_region* r, float* features, int* variants, double* seconds, int max_records) {
    if (!r || max_records < 0) return fail(AO_EINVAL, "bad arguments");
    std::lock_guard<std::mutex> g(r->mu);
    harvest(r, true);
    const int n = (int)std::min<size_t>((size_t)max_records, r->db.size());
    for (int i = 0; i < n; ++i) {
        const Record& rec = r->db[i];
        if (features) memcpy(features + (size_t)i * AO_MAX_FEATURES, rec.f, sizeof(rec.f));
        if (variants) variants[i] = rec.variant;
        if (seconds) seconds[i] = rec.seconds;
    }
    return n;
}

int region_clear_memo(ao_region* r) {
    if (!r) return fail(AO_EINVAL, "region is NULL");
    std::lock_guard<std::mutex> g(r->mu);
    r->memo.clear();
    return AO_OK;
}

int region_save(ao_region* r, const char* path) {
    if (!r || !path) return fail(AO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(r->mu);
    harvest(r, true);
    Writer w;
    w.put(kMagic, 8);
    w.put<uint32_t>(1);
    w.put<int32_t>(r->kind);
    w.put<int32_t>((int32_t)r->variants.size());
    for (const ao_variant& v : r->variants) w.put(v);
    w.put<int32_t>(r->min_train);
    w.put<uint64_t>((uint64_t)r->db.size());
    for (const Record& rec : r->db) {
        w.put(rec.f, sizeof(rec.f));
        w.put<int32_t>(rec.variant);
        w.put<int32_t>(rec.resident);
        w.put<double>(rec.seconds);
        w.put<uint64_t>(rec.t_ns);
    }
    const bool mlp_model = r->trained && r->dtree_depth == 0;
    w.put<uint32_t>(mlp_model ? 1u : 0u);
    if (mlp_model) {
        w.put(r->params.data(), AO_MLP_PARAMS * 4);
        w.put(r->norm);
        w.put(r->fmin, sizeof(r->fmin));
        w.put(r->fmax, sizeof(r->fmax));
    }
    const uint32_t crc = crc32_update(0, w.buf.data(), w.buf.size());
    w.put<uint32_t>(crc);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* fp = fopen(tmp.c_str(), "wb");
    if (!fp) return fail(AO_EIO, "cannot open " + tmp);
    const size_t wr = fwrite(w.buf.data(), 1, w.buf.size(), fp);
    const int cl = fclose(fp);
    if (wr != w.buf.size() || cl != 0 || rename(tmp.c_str(), path) != 0)
        return fail(AO_EIO, "write failed: " + std::string(path));
    return AO_OK;
}

int region_load(ao_region* r, const char* path) {
    if (!r || !path) return fail(AO_EINVAL, "NULL argument");
    FILE* fp = fopen(path, "rb");
    if (!fp) return fail(AO_EIO, "cannot open " + std::string(path));
    std::vector<uint8_t> buf;
    uint8_t tmp[1 << 16];
    size_t k;
    while ((k = fread(tmp, 1, sizeof(tmp), fp)) > 0) buf.insert(buf.end(), tmp, tmp + k);
    fclose(fp);
    if (buf.size() < 12) return fail(AO_EIO, "file too short");
    uint32_t crc_stored;
    memcpy(&crc_stored, buf.data() + buf.size() - 4, 4);
    if (crc32_update(0, buf.data(), buf.size() - 4) != crc_stored)
        return fail(AO_EIO, "CRC mismatch: corrupt file");
    Reader rd{buf.data(), buf.size() - 4};
    char magic[8];
    rd.get(magic, 8);
    if (!rd.ok || memcmp(magic, kMagic, 8) != 0) return fail(AO_EIO, "bad magic");
    if (rd.get<uint32_t>() != 1u) return fail(AO_EIO, "unsupported version");
    std::lock_guard<std::mutex> g(r->mu);
    const int32_t kind = rd.get<int32_t>();
    const int32_t V = rd.get<int32_t>();
    if (!rd.ok || kind != r->kind || V != (int32_t)r->variants.size())
        return fail(AO_EIO, "file was saved by a region of another kind / variant count");
    for (int i = 0; i < V; ++i) {
        ao_variant v = rd.get<ao_variant>();
        if (!rd.ok || !same_variant(v, r->variants[i]))
            return fail(AO_EIO, "file was saved by a region with other variants");
    }
    (void)rd.get<int32_t>();  // min_train of the saving region (the declared one stays)
    const uint64_t nrec = rd.get<uint64_t>();
    if (!rd.ok || nrec > (buf.size() / 32)) return fail(AO_EIO, "bad record count");
    std::vector<Record> db(nrec);
    for (uint64_t i = 0; i < nrec; ++i) {
        rd.get(db[i].f, sizeof(db[i].f));
        db[i].variant = rd.get<int32_t>();
        db[i].resident = rd.get<int32_t>();
        db[i].seconds = rd.get<double>();
        db[i].t_ns = rd.get<uint64_t>();
        if (db[i].variant < 0 || db[i].variant >= V) rd.ok = false;
    }
    const uint32_t has_model = rd.get<uint32_t>();
    std::vector<float> params;
    MlpNorm norm{};
    float fmin[AO_MAX_FEATURES], fmax[AO_MAX_FEATURES];
    if (has_model) {
        params.resize(AO_MLP_PARAMS);
        rd.get(params.data(), AO_MLP_PARAMS * 4);
        norm = rd.get<MlpNorm>();
        rd.get(fmin, sizeof(fmin));
        rd.get(fmax, sizeof(fmax));
        for (float v : params)
            if (!std::isfinite(v)) rd.ok = false;
    }
    if (!rd.ok || rd.off != rd.n) return fail(AO_EIO, "truncated or malformed file");
    if (has_model) {
        hipError_t e = hipSuccess;
        if (!r->d_params) {
            e = hipMalloc(&r->d_params, AO_MLP_PARAMS * 4);
            if (e == hipSuccess) e = hipMalloc(&r->d_norm, sizeof(MlpNorm));
        }
        if (e == hipSuccess)
            e = hipMemcpy(r->d_params, params.data(), AO_MLP_PARAMS * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(r->d_norm, &norm, sizeof(MlpNorm), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(AO_EHIP, hip_msg("model upload", e));
        }
    }
    harvest(r, true);
    r->db = std::move(db);
    r->uniq.clear();
    for (const Record& rec : r->db) r->uniq.insert(UKey{make_key(rec.f), rec.variant});
    r->memo.clear();
    r->trained = has_model != 0 && r->dtree_depth == 0;
    if (r->dtree_depth > 0) r->tree.nodes.clear();  // a tree is rebuilt by selector_train
    if (has_model) {
        r->params = params;
        r->norm = norm;
        memcpy(r->fmin, fmin, sizeof(fmin));
        memcpy(r->fmax, fmax, sizeof(fmax));
    }
    return AO_OK;
}

int region_destroy(ao_region* r) {
    if (!r) return fail(AO_EINVAL, "region is NULL");
    {
        std::lock_guard<std::mutex> g(g_reg_mu);
        auto it = g_regions.find(r->name);
        if (it == g_regions.end() || it->second != r) return fail(AO_EINVAL, "unknown region handle");
        g_regions.erase(it);
    }
    delete r;
    return AO_OK;
}

}  // extern "C"
