// C ABI of libtc.so (declared in include/tc.h): descriptor intake, the plan
// cache, device upload of plan vectors, execution, autotuning and batching.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <queue>
#include <string>
#include <vector>

#include "launch.hpp"
#include "plan.hpp"
#include "tc.h"

struct tc_plan {
    std::unique_ptr<tc::Plan> p;
};

struct tc_batch {
    // tile < 0: every problem runs with its own tile class (one persistent
    // launch per class present); else one class for the whole batch
    int dtype = 0, mode = 0, tile = -1, count = 0, device = 0, grid = 0;
    bool off64 = false;
    int64_t total_items = 0;
    std::vector<tc::BatchItemDev> host;  // per problem that launches work (device pointers filled)
    std::vector<int> host_of;            // per problem: its index in `host`, -1 for an empty problem
    std::vector<int> best;               // per problem: its own regular tile class
    std::vector<double> slow;            // per problem: time per flop relative to one whose k blocks all have a stride
    std::vector<int> order;              // problem index of each table entry
    struct Segment {
        int tile, first, count, grid;
        int64_t items;
        size_t off_pos, ent_pos;  // the launch's work lists inside `assign` (int32 units)
    };
    std::vector<Segment> segs;  // launches, in issue order
    void* table = nullptr;      // device BatchItemDev[count]
    void* vectors = nullptr;    // device arena holding every problem's vectors
    void* assign = nullptr;     // device int32: per launch, workgroup offsets then (problem, tile) entries
    size_t assign_cap = 0;      // bytes allocated for `assign`
};

namespace tc {

static int hipfail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return TC_ERR_HIP;
}

static int make_desc(int ndim, const int64_t* lens, const int64_t* strides, const char* idx, const char* name,
                     TensorDesc* d) {
    if (ndim < 0 || ndim > TC_MAX_NDIM) {
        set_error(std::string(name) + ": ndim outside [0, 16]");
        return TC_ERR_NDIM;
    }
    if (ndim > 0 && (!lens || !strides || !idx)) {
        set_error(std::string(name) + ": NULL descriptor array");
        return TC_ERR_NULL;
    }
    d->ndim = ndim;
    for (int i = 0; i < ndim; ++i) {
        d->lens[i] = lens[i];
        d->strides[i] = strides[i];
        d->idx[i] = idx[i];
    }
    return TC_OK;
}

static std::string desc_key(const TensorDesc& t) {
    std::string s;
    s.reserve(2 + t.ndim * 18);
    s.push_back((char)t.ndim);
    s.append(t.idx, t.ndim);
    s.append((const char*)t.lens, sizeof(int64_t) * t.ndim);
    s.append((const char*)t.strides, sizeof(int64_t) * t.ndim);
    return s;
}

// ---- plan cache and autotuner cache -------------------------------------
static std::mutex g_cache_mu;
static std::map<std::string, std::unique_ptr<tc_plan>> g_plans;       // tc_contract
static std::map<std::string, std::unique_ptr<tc_plan>> g_host_plans;  // tc_contract_noalloc (never uploaded)
static std::map<std::string, int> g_tuned;  // plan signature -> tile

static size_t elt_size(int dtype) { return dtype == TC_F64 ? 8 : 4; }

// Copy the plan's vectors to the current device if not there yet.
static int ensure_uploaded(const Plan& p, DeviceVectors** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hipfail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the library's limit of 16");
        return TC_ERR_ARG;
    }
    std::lock_guard<std::mutex> g(p.dev_mu);
    DeviceVectors& dv = p.dev[dev];
    if (dv.bytes) {
        *out = &dv;
        return TC_OK;
    }
    const std::vector<int64_t>* vecs[8] = {&p.rX, &p.cX, &p.rY, &p.cY, &p.rC, &p.cC, &p.kbsX, &p.kbsY};
    size_t* offs[8] = {&dv.o_rX, &dv.o_cX, &dv.o_rY, &dv.o_cY, &dv.o_rC, &dv.o_cC, &dv.o_kbsX, &dv.o_kbsY};
    size_t total = 0;
    for (int i = 0; i < 8; ++i) {
        *offs[i] = total;
        size_t n = std::max<size_t>(vecs[i]->size(), 1);
        total += (n + 63) & ~(size_t)63;  // 256-byte aligned starts (for int32)
    }
    const size_t w = p.off64 ? 8 : 4;
    std::vector<char> host(total * w, 0);
    for (int i = 0; i < 8; ++i) {
        const std::vector<int64_t>& v = *vecs[i];
        for (size_t j = 0; j < v.size(); ++j) {
            if (p.off64) ((int64_t*)host.data())[*offs[i] + j] = v[j];
            else ((int32_t*)host.data())[*offs[i] + j] = (int32_t)v[j];
        }
    }
    if (dv.buf) {
        hipFree(dv.buf);
        dv.buf = nullptr;
    }
    e = hipMalloc(&dv.buf, host.size());
    if (e != hipSuccess) {
        dv.buf = nullptr;
        set_error("hipMalloc of plan vectors failed");
        return TC_ERR_NOMEM;
    }
    e = hipMemcpy(dv.buf, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hipfail(e, "hipMemcpy of plan vectors");
    dv.bytes = host.size();
    *out = &dv;
    return TC_OK;
}

static void free_device(Plan* p) {
    for (auto& d : p->dev)
        if (d.buf) {
            hipFree(d.buf);
            d.buf = nullptr;
            d.bytes = 0;
        }
    for (auto& per_dev : p->ws) {
        for (auto& w : per_dev)
            if (w.second.first) hipFree(w.second.first);
        per_dev.clear();
    }
}

static bool overlaps(const void* a, int64_t na, const void* b, int64_t nb, size_t w) {
    if (!a || !b || na <= 0 || nb <= 0) return false;
    const char* a0 = (const char*)a;
    const char* b0 = (const char*)b;
    return a0 < b0 + nb * (int64_t)w && b0 < a0 + na * (int64_t)w;
}

// A tensor's data must be device memory of the current device, and its
// element span must lie inside the allocation holding its first element: a
// host pointer or a descriptor reaching past the buffer would otherwise take
// the kernel to an invalid address.  Skipped under graph capture (no runtime
// queries there; plans must have been checked and uploaded beforehand).
static int check_device_span(const void* ptr, int64_t span, size_t w, const char* name) {
    if (!ptr || span <= 0) return TC_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hipfail(e, "hipGetDevice");
    hipPointerAttribute_t at{};
    e = hipPointerGetAttributes(&at, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // do not leave the failed query for a later launch check
        set_error(std::string(name) + " is not device memory (host pointer?)");
        return TC_ERR_ARG;
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged) {
        set_error(std::string(name) + " is not device memory (host pointer?)");
        return TC_ERR_ARG;
    }
    if (at.device != dev) {
        set_error(std::string(name) + " lives on device " + std::to_string(at.device) + ", not on the current device " +
                  std::to_string(dev));
        return TC_ERR_ARG;
    }
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return TC_OK;  // no range information: the type and device checks stand
    }
    const uintptr_t b0 = (uintptr_t)base, p0 = (uintptr_t)ptr;
    if ((uint64_t)span > (uint64_t)((b0 + size - p0) / w)) {
        set_error(std::string(name) + ": the descriptor's element span reaches past the end of its allocation");
        return TC_ERR_ARG;
    }
    return TC_OK;
}

static bool capturing(hipStream_t stream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Checks shared by every execution path: NULL data, C overlapping A or B,
// and (outside capture) device memory holding each span.  *run = false when
// the call is a no-op.
static int check_call(const Plan& p, double alpha, const void* A, const void* B, void* C, hipStream_t stream,
                      bool* run) {
    *run = false;
    if (p.noop || p.m == 0 || p.n == 0) return TC_OK;
    if (!C) {
        set_error("C is NULL");
        return TC_ERR_NULL;
    }
    const bool reads_ab = !(p.k_empty || alpha == 0.0);
    if (reads_ab && (!A || !B)) {
        set_error("A or B is NULL");
        return TC_ERR_NULL;
    }
    const size_t w = elt_size(p.dtype);
    if (overlaps(C, p.spanC, A, p.spanA, w) || overlaps(C, p.spanC, B, p.spanB, w)) {
        set_error("C overlaps A or B");
        return TC_ERR_ALIAS;
    }
    if (!capturing(stream)) {
        int st;
        if ((st = check_device_span(C, p.spanC, w, "C"))) return st;
        if (reads_ab && ((st = check_device_span(A, p.spanA, w, "A")) || (st = check_device_span(B, p.spanB, w, "B"))))
            return st;
    }
    *run = true;
    return TC_OK;
}

// Workspace of the packed split tile for a launch on `stream` (null for every
// other tile): the plan keeps one buffer per (device, stream) it ran on, so
// that calls on different streams never share one, while calls on one stream
// are ordered by the stream.  Allocated (or grown, after the stream's earlier
// work has finished) outside capture; under capture it must already exist.
static int plan_workspace(const Plan& p, hipStream_t stream, void** ws) {
    *ws = nullptr;
    const TileCfg& t = tile_table(p.dtype, p.mode)[p.tile];
    if (p.mode != TC_SPLIT_BF16X3 || t.layout != 4 || p.k_empty || p.k == 0) return TC_OK;
    const size_t need = (size_t)split_pack_bytes(t, p.m, p.n, p.k);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hipfail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the library's limit of 16");
        return TC_ERR_ARG;
    }
    std::lock_guard<std::mutex> g(p.dev_mu);
    std::pair<void*, size_t>& w = p.ws[dev][(void*)stream];
    if (w.first && w.second >= need) {
        *ws = w.first;
        return TC_OK;
    }
    if (capturing(stream)) {
        set_error("the packed split tile's workspace for this stream is made by a first call outside capture");
        return TC_ERR_CAPTURE;
    }
    if (w.first) {
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hipfail(e, "hipStreamSynchronize before growing the split panels");
        hipFree(w.first);
        w = {nullptr, 0};
    }
    e = hipMalloc(&w.first, need);
    if (e != hipSuccess) {
        w = {nullptr, 0};
        set_error("hipMalloc of the split panels (" + std::to_string(need) + " bytes) failed");
        return TC_ERR_NOMEM;
    }
    w.second = need;
    *ws = w.first;
    return TC_OK;
}

static int execute(const tc_plan* plan, double alpha, const void* A, const void* B, double beta, void* C,
                   hipStream_t stream) {
    const Plan& p = *plan->p;
    bool run = false;
    int st = check_call(p, alpha, A, B, C, stream, &run);
    if (st || !run) return st;
    DeviceVectors* dv = nullptr;
    if (capturing(stream)) {
        int dev = 0;
        hipGetDevice(&dev);
        if (dev < 0 || dev >= kMaxDevices || !p.dev[dev].bytes) {
            set_error("plan vectors must be uploaded before graph capture (tc_plan_upload)");
            return TC_ERR_CAPTURE;
        }
        dv = &p.dev[dev];
    } else if ((st = ensure_uploaded(p, &dv))) {
        return st;
    }
    void* ws = nullptr;
    if (alpha != 0.0 && (st = plan_workspace(p, stream, &ws))) return st;
    return launch_plan(p, *dv, alpha, A, B, beta, C, stream, ws);
}

static int create(tc_plan** out, int ndim_A, const int64_t* lens_A, const int64_t* strides_A, const char* idx_A,
                  int ndim_B, const int64_t* lens_B, const int64_t* strides_B, const char* idx_B, int ndim_C,
                  const int64_t* lens_C, const int64_t* strides_C, const char* idx_C, int dtype, int mode) {
    TensorDesc a, b, c;
    int st;
    if ((st = make_desc(ndim_A, lens_A, strides_A, idx_A, "A", &a)) ||
        (st = make_desc(ndim_B, lens_B, strides_B, idx_B, "B", &b)) ||
        (st = make_desc(ndim_C, lens_C, strides_C, idx_C, "C", &c)))
        return st;
    std::unique_ptr<Plan> p;
    if ((st = build_plan(a, b, c, dtype, mode, &p))) return st;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto it = g_tuned.find(plan_signature(*p));
        if (it != g_tuned.end() && it->second != p->tile && !p->off64) set_plan_tile(p.get(), it->second);
    }
    tc_plan* h = new (std::nothrow) tc_plan;
    if (!h) {
        set_error("out of host memory");
        return TC_ERR_NOMEM;
    }
    h->p = std::move(p);
    *out = h;
    return TC_OK;
}

// The plan of a descriptor set from `cache` (created and inserted on first
// use).  The one-shot entry points keep separate caches: tc_contract's plans
// hold device copies of their vectors, the allocation-free path's never do.
static int cached_plan(std::map<std::string, std::unique_ptr<tc_plan>>& cache, int ndim_A, const int64_t* lens_A,
                       const int64_t* strides_A, const char* idx_A, int ndim_B, const int64_t* lens_B,
                       const int64_t* strides_B, const char* idx_B, int ndim_C, const int64_t* lens_C,
                       const int64_t* strides_C, const char* idx_C, int dtype, int mode, tc_plan** out) {
    TensorDesc a, b, c;
    int st;
    if ((st = make_desc(ndim_A, lens_A, strides_A, idx_A, "A", &a)) ||
        (st = make_desc(ndim_B, lens_B, strides_B, idx_B, "B", &b)) ||
        (st = make_desc(ndim_C, lens_C, strides_C, idx_C, "C", &c)))
        return st;
    std::string key;
    key.push_back((char)dtype);
    key.push_back((char)mode);
    key += desc_key(a);
    key += desc_key(b);
    key += desc_key(c);
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *out = it->second.get();
            return TC_OK;
        }
    }
    tc_plan* fresh = nullptr;
    if ((st = create(&fresh, ndim_A, lens_A, strides_A, idx_A, ndim_B, lens_B, strides_B, idx_B, ndim_C, lens_C,
                     strides_C, idx_C, dtype, mode)))
        return st;
    std::lock_guard<std::mutex> g(g_cache_mu);
    auto it = cache.find(key);
    if (it == cache.end()) {
        *out = fresh;
        cache[key].reset(fresh);
    } else {
        *out = it->second.get();
        delete fresh;  // no device copies yet
    }
    return TC_OK;
}

}  // namespace tc

using namespace tc;

extern "C" {

int tc_plan_create(tc_plan** plan, int ndim_A, const int64_t* lens_A, const int64_t* strides_A, const char* idx_A,
                   int ndim_B, const int64_t* lens_B, const int64_t* strides_B, const char* idx_B, int ndim_C,
                   const int64_t* lens_C, const int64_t* strides_C, const char* idx_C, int dtype, int mode) {
    if (!plan) {
        set_error("plan out-pointer is NULL");
        return TC_ERR_NULL;
    }
    *plan = nullptr;
    try {
        return create(plan, ndim_A, lens_A, strides_A, idx_A, ndim_B, lens_B, strides_B, idx_B, ndim_C, lens_C,
                      strides_C, idx_C, dtype, mode);
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return TC_ERR_NOMEM;
    } catch (...) {
        set_error("internal error while planning");
        return TC_ERR_ARG;
    }
}

int tc_plan_upload(tc_plan* plan) {
    if (!plan) {
        set_error("plan is NULL");
        return TC_ERR_NULL;
    }
    DeviceVectors* dv;
    return ensure_uploaded(*plan->p, &dv);
}

int tc_plan_execute(const tc_plan* plan, double alpha, const void* A, const void* B, double beta, void* C,
                    void* stream) {
    if (!plan) {
        set_error("plan is NULL");
        return TC_ERR_NULL;
    }
    return execute(plan, alpha, A, B, beta, C, (hipStream_t)stream);
}

// Device copy of the plan's vectors for a launch on `stream` (uploaded
// outside capture; under capture it must already be there).
static int plan_vectors(const Plan& p, hipStream_t stream, DeviceVectors** dv) {
    if (capturing(stream)) {
        int dev = 0;
        hipGetDevice(&dev);
        if (dev < 0 || dev >= kMaxDevices || !p.dev[dev].bytes) {
            set_error("plan vectors must be uploaded before graph capture (tc_plan_upload)");
            return TC_ERR_CAPTURE;
        }
        *dv = &p.dev[dev];
        return TC_OK;
    }
    return ensure_uploaded(p, dv);
}

int tc_plan_pack_elements(const tc_plan* plan, int operand, int64_t* elems) {
    if (!plan || !elems) {
        set_error("plan or elems is NULL");
        return TC_ERR_NULL;
    }
    if (operand != 0 && operand != 1) {
        set_error("operand must be 0 (A) or 1 (B)");
        return TC_ERR_ARG;
    }
    const Plan& p = *plan->p;
    *elems = (p.noop || p.k_empty) ? 0 : pack_elements(p, operand);
    return TC_OK;
}

int tc_plan_pack(const tc_plan* plan, int operand, const void* src, void* dst, void* stream) {
    int64_t elems = 0;
    int st = tc_plan_pack_elements(plan, operand, &elems);
    if (st) return st;
    if (elems == 0) return TC_OK;
    const Plan& p = *plan->p;
    if (!src || !dst) {
        set_error("src or dst is NULL");
        return TC_ERR_NULL;
    }
    const size_t w = elt_size(p.dtype);
    const int64_t span = operand == 0 ? p.spanA : p.spanB;
    if (overlaps(dst, elems, src, span, w)) {
        set_error("dst overlaps src");
        return TC_ERR_ALIAS;
    }
    hipStream_t s = (hipStream_t)stream;
    if (!capturing(s) && ((st = check_device_span(src, span, w, "src")) || (st = check_device_span(dst, elems, w, "dst"))))
        return st;
    DeviceVectors* dv = nullptr;
    if ((st = plan_vectors(p, s, &dv))) return st;
    return launch_pack(p, *dv, operand, src, dst, s);
}

int tc_plan_store(const tc_plan* plan, double alpha, const void* src, double beta, void* C, void* stream) {
    if (!plan) {
        set_error("plan is NULL");
        return TC_ERR_NULL;
    }
    const Plan& p = *plan->p;
    if (p.noop || p.m == 0 || p.n == 0) return TC_OK;
    if (!src || !C) {
        set_error("src or C is NULL");
        return TC_ERR_NULL;
    }
    const size_t w = elt_size(p.dtype);
    if (overlaps(C, p.spanC, src, p.m * p.n, w)) {
        set_error("C overlaps src");
        return TC_ERR_ALIAS;
    }
    hipStream_t s = (hipStream_t)stream;
    int st;
    if (!capturing(s) && ((st = check_device_span(src, p.m * p.n, w, "src")) || (st = check_device_span(C, p.spanC, w, "C"))))
        return st;
    DeviceVectors* dv = nullptr;
    if ((st = plan_vectors(p, s, &dv))) return st;
    return launch_store(p, *dv, alpha, src, beta, C, s);
}

int tc_plan_destroy(tc_plan* plan) {
    if (!plan) return TC_OK;
    free_device(plan->p.get());
    delete plan;
    return TC_OK;
}

int tc_plan_describe(const tc_plan* plan, char* buf, size_t len) {
    if (!plan) {
        set_error("plan is NULL");
        return TC_ERR_NULL;
    }
    std::string s = describe_plan(*plan->p);
    if (buf && len) {
        size_t n = std::min(len - 1, s.size());
        memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return (int)s.size();
}

int tc_tile_count(int dtype, int mode) {
    int n = tile_count(dtype, mode);
    if (!n) {
        set_error("unsupported dtype/mode combination");
        return TC_ERR_DTYPE;
    }
    return n;
}

int tc_tile_info(int dtype, int mode, int tile, int* MT, int* NT, int* KT, int* waves) {
    int n = tile_count(dtype, mode);
    if (!n) {
        set_error("unsupported dtype/mode combination");
        return TC_ERR_DTYPE;
    }
    if (tile < 0 || tile >= n) {
        set_error("tile id out of range");
        return TC_ERR_ARG;
    }
    const TileCfg& t = tile_table(dtype, mode)[tile];
    if (MT) *MT = t.MT;
    if (NT) *NT = t.NT;
    if (KT) *KT = t.KT;
    if (waves) *waves = t.waves();
    return TC_OK;
}

int tc_plan_set_tile(tc_plan* plan, int tile) {
    if (!plan) {
        set_error("plan is NULL");
        return TC_ERR_NULL;
    }
    Plan* p = plan->p.get();
    if (tile < 0 || tile >= tile_count(p->dtype, p->mode)) {
        set_error("tile id out of range");
        return TC_ERR_ARG;
    }
    std::lock_guard<std::mutex> g(p->dev_mu);
    set_plan_tile(p, tile);
    return TC_OK;
}

int tc_plan_get_tile(const tc_plan* plan) {
    if (!plan) {
        set_error("plan is NULL");
        return TC_ERR_NULL;
    }
    return plan->p->tile;
}

int tc_plan_autotune(tc_plan* plan, const void* A, const void* B, void* C_scratch, int reps, void* stream,
                     double* best_ms) {
    if (!plan) {
        set_error("plan is NULL");
        return TC_ERR_NULL;
    }
    if (reps < 1) reps = 1;
    Plan* p = plan->p.get();
    hipStream_t s = (hipStream_t)stream;
    const int nt = tile_count(p->dtype, p->mode);
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hipfail(e, "hipEventCreate");
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        hipEventDestroy(e0);
        return hipfail(e, "hipEventCreate");
    }
    int best = p->tile;
    float best_t = 1e30f;
    int st = TC_OK;
    for (int t = 0; t < nt && st == TC_OK; ++t) {
        {
            std::lock_guard<std::mutex> g(p->dev_mu);
            set_plan_tile(p, t);
        }
        if ((st = execute(plan, 1.0, A, B, 0.0, C_scratch, s))) break;  // warm-up (uploads)
        hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == TC_OK; ++r) st = execute(plan, 1.0, A, B, 0.0, C_scratch, s);
        hipEventRecord(e1, s);
        e = hipEventSynchronize(e1);
        if (e != hipSuccess) {
            st = hipfail(e, "autotune timing");
            break;
        }
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (ms < best_t) {
            best_t = ms;
            best = t;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> g(p->dev_mu);
        set_plan_tile(p, best);
    }
    if (st) return st;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        g_tuned[plan_signature(*p)] = best;
    }
    if (best_ms) *best_ms = best_t;
    return TC_OK;
}

int tc_contract(double alpha, const void* A, int ndim_A, const int64_t* lens_A, const int64_t* strides_A,
                const char* idx_A, const void* B, int ndim_B, const int64_t* lens_B, const int64_t* strides_B,
                const char* idx_B, double beta, void* C, int ndim_C, const int64_t* lens_C, const int64_t* strides_C,
                const char* idx_C, int dtype, int mode, void* stream) {
    try {
        tc_plan* plan = nullptr;
        int st = cached_plan(g_plans, ndim_A, lens_A, strides_A, idx_A, ndim_B, lens_B, strides_B, idx_B, ndim_C,
                             lens_C, strides_C, idx_C, dtype, mode, &plan);
        if (st) return st;
        return execute(plan, alpha, A, B, beta, C, (hipStream_t)stream);
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return TC_ERR_NOMEM;
    } catch (...) {
        set_error("internal error");
        return TC_ERR_ARG;
    }
}

int tc_contract_noalloc(double alpha, const void* A, int ndim_A, const int64_t* lens_A, const int64_t* strides_A,
                        const char* idx_A, const void* B, int ndim_B, const int64_t* lens_B, const int64_t* strides_B,
                        const char* idx_B, double beta, void* C, int ndim_C, const int64_t* lens_C,
                        const int64_t* strides_C, const char* idx_C, int dtype, int mode, void* stream) {
    try {
        tc_plan* plan = nullptr;
        int st = cached_plan(g_host_plans, ndim_A, lens_A, strides_A, idx_A, ndim_B, lens_B, strides_B, idx_B, ndim_C,
                             lens_C, strides_C, idx_C, dtype, mode, &plan);
        if (st) return st;
        const Plan& p = *plan->p;
        DeviceVectors dv;
        if (!p.noop && noalloc_layout(p, &dv) > (size_t)TC_NOALLOC_SCRATCH_BYTES) {
            set_error("the plan's offset vectors need " + std::to_string(dv.bytes) +
                      " bytes, more than the allocation-free entry point's array of " +
                      std::to_string((long long)TC_NOALLOC_SCRATCH_BYTES) + " bytes");
            return TC_ERR_ARG;
        }
        bool run = false;
        if ((st = check_call(p, alpha, A, B, C, (hipStream_t)stream, &run)) || !run) return st;
        if ((st = noalloc_vectors(p, (hipStream_t)stream, &dv))) return st;
        // no workspace: a packed split tile runs as its in-kernel-split twin
        return launch_plan(p, dv, alpha, A, B, beta, C, (hipStream_t)stream, nullptr);
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return TC_ERR_NOMEM;
    } catch (...) {
        set_error("internal error");
        return TC_ERR_ARG;
    }
}

}  // extern "C"

namespace tc {

// Work-item counts of a batch, the table upload and the workgroups' work
// lists.  The table is grouped by tile class (one persistent launch per class,
// the class with the most work first); inside a class problems are ordered by
// decreasing cost of one tile (k times the problem's relative time per flop),
// the order in which the work lists below hand out their tiles.
static int batch_layout(tc_batch* b) {
    const TileCfg* tab = tile_table(b->dtype, b->mode);
    const std::vector<BatchItemDev>& items = b->host;
    const size_t n = items.size();
    std::vector<int> cls(n);
    for (size_t i = 0; i < n; ++i) cls[i] = b->tile >= 0 ? b->tile : b->best[i];
    const int nt = tile_count(b->dtype, b->mode);
    std::vector<double> work(nt, 0.0);
    for (size_t i = 0; i < n; ++i) {
        const TileCfg& t = tab[cls[i]];
        work[cls[i]] += (double)((items[i].m + t.MT - 1) / t.MT) * (double)((items[i].n + t.NT - 1) / t.NT) *
                        t.MT * t.NT * (double)std::max<int64_t>(items[i].k, 1);
    }
    std::vector<int> rank(nt);
    for (int c = 0; c < nt; ++c) rank[c] = c;
    std::stable_sort(rank.begin(), rank.end(), [&](int x, int y) { return work[x] > work[y]; });
    std::vector<int> pos(nt);
    for (int r = 0; r < nt; ++r) pos[rank[r]] = r;
    std::vector<int> idx(n);
    for (size_t i = 0; i < n; ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
        if (cls[x] != cls[y]) return pos[cls[x]] < pos[cls[y]];
        return (double)items[x].k * b->slow[(size_t)x] > (double)items[y].k * b->slow[(size_t)y];
    });
    std::vector<double> slow_of;  // per table entry
    slow_of.reserve(n);
    for (size_t e = 0; e < n; ++e) slow_of.push_back(b->slow[(size_t)idx[e]]);
    std::vector<BatchItemDev> table;
    table.reserve(n);
    b->segs.clear();
    b->total_items = 0;
    int64_t first = 0;
    for (size_t e = 0; e < n; ++e) {
        const int i = idx[e];
        const TileCfg& t = tab[cls[i]];
        if (b->segs.empty() || b->segs.back().tile != cls[i]) {
            b->segs.push_back({cls[i], (int)e, 0, 0, 0});
            first = 0;
        }
        BatchItemDev it = items[i];
        it.tiles_m = (it.m + t.MT - 1) / t.MT;
        it.tiles_n = (it.n + t.NT - 1) / t.NT;
        it.first_item = first;
        first += it.tiles_m * it.tiles_n;
        b->segs.back().count++;
        b->segs.back().items = first;
        b->total_items += it.tiles_m * it.tiles_n;
        table.push_back(it);
    }
    b->order = idx;
    if (!b->table) {
        hipError_t e = hipMalloc(&b->table, std::max<size_t>(table.size(), 1) * sizeof(BatchItemDev));
        if (e != hipSuccess) {
            b->table = nullptr;
            set_error("hipMalloc of the batch table failed");
            return TC_ERR_NOMEM;
        }
    }
    if (!table.empty()) {
        hipError_t e = hipMemcpy(b->table, table.data(), table.size() * sizeof(BatchItemDev), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hipfail(e, "hipMemcpy of the batch table");
    }
    b->grid = 0;
    for (auto& sg : b->segs) {
        sg.grid = sg.items > 0 ? batch_grid(b->dtype, b->mode, sg.tile, b->off64, sg.items) : 0;
        if (sg.items > 0 && sg.grid <= 0) {
            set_error("could not size the persistent grid");
            return TC_ERR_HIP;
        }
        b->grid = std::max(b->grid, sg.grid);
    }
    // Work lists: within each launch, the (problem, tile) work items in
    // decreasing cost (the table is in that order inside a class; every tile
    // of a problem costs the same), each given to the workgroup with the least
    // work so far, ties to the lower index (longest processing time first).
    // The lists are fixed here, so a launch needs no counter and no reset
    // between graph replays, and the assignment is deterministic.  Cost of a
    // tile: its k plus three stages for the prologue and the C update, times
    // the problem's relative time per flop.
    std::vector<int32_t> host;
    for (auto& sg : b->segs) {
        const TileCfg& t = tab[sg.tile];
        const int G = sg.grid;
        std::vector<std::vector<int32_t>> lists((size_t)std::max(G, 1));
        typedef std::pair<double, int> Load;  // (work so far, workgroup)
        std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
        for (int g = 0; g < G; ++g) heap.push({0.0, g});
        for (int e = 0; e < sg.count; ++e) {
            const BatchItemDev& it = table[(size_t)(sg.first + e)];
            const int64_t tiles = it.tiles_m * it.tiles_n;
            if (tiles > 0x7fffffffLL) {
                set_error("a batch problem has more than 2^31 tiles");
                return TC_ERR_ARG;
            }
            const double cost = ((double)std::max<int64_t>(it.k, 1) + 3.0 * t.KT) * slow_of[(size_t)(sg.first + e)];
            for (int64_t w = 0; w < tiles; ++w) {
                Load l = heap.top();
                heap.pop();
                lists[(size_t)l.second].push_back(e);
                lists[(size_t)l.second].push_back((int32_t)w);
                heap.push({l.first + cost, l.second});
            }
        }
        sg.off_pos = host.size();
        size_t run = 0;
        for (int g = 0; g <= G; ++g) {
            if ((int64_t)run > 0x7fffffffLL) {
                set_error("too many work items in one batched launch");
                return TC_ERR_ARG;
            }
            host.push_back((int32_t)run);
            if (g < G) run += lists[(size_t)g].size() / 2;
        }
        sg.ent_pos = host.size();
        for (int g = 0; g < G; ++g) host.insert(host.end(), lists[(size_t)g].begin(), lists[(size_t)g].end());
    }
    const size_t bytes = std::max<size_t>(host.size(), 1) * sizeof(int32_t);
    if (bytes > b->assign_cap) {
        if (b->assign) hipFree(b->assign);
        b->assign = nullptr;
        b->assign_cap = 0;
        hipError_t e = hipMalloc(&b->assign, bytes);
        if (e != hipSuccess) {
            b->assign = nullptr;
            set_error("hipMalloc of the batch work lists failed");
            return TC_ERR_NOMEM;
        }
        b->assign_cap = bytes;
    }
    if (!host.empty()) {
        hipError_t e = hipMemcpy(b->assign, host.data(), host.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hipfail(e, "hipMemcpy of the batch work lists");
    }
    return TC_OK;
}

// Every problem of a batch runs inside the same persistent launches, so one
// problem's output must not overlap any other problem's output, nor any
// operand another problem reads (address ranges of the element spans).  The
// outputs are sorted by start address: they are pairwise disjoint iff each
// starts at or after the furthest end before it; an operand range then meets
// an output iff the first output ending after the operand's start begins
// before the operand's end.
static int check_batch_aliasing(int count, const tc_plan* const* plans, const double* alpha, const void* const* A,
                                const void* const* B, void* const* C, size_t elt) {
    struct Range {
        uintptr_t lo, hi;
        int prob;
    };
    std::vector<Range> outs;
    for (int i = 0; i < count; ++i) {
        const Plan& p = *plans[i]->p;
        if (p.noop || p.m == 0 || p.n == 0 || p.spanC <= 0) continue;
        outs.push_back({(uintptr_t)C[i], (uintptr_t)C[i] + (uintptr_t)p.spanC * elt, i});
    }
    std::sort(outs.begin(), outs.end(), [](const Range& x, const Range& y) { return x.lo < y.lo; });
    for (size_t e = 1; e < outs.size(); ++e) {
        // outputs before e are disjoint and sorted, so e-1 ends furthest
        if (outs[e].lo < outs[e - 1].hi) {
            set_error("the outputs of batch problems " + std::to_string(outs[e - 1].prob) + " and " +
                      std::to_string(outs[e].prob) + " overlap");
            return TC_ERR_ALIAS;
        }
    }
    auto meets_output = [&](const void* ptr, int64_t span, int* who) {
        if (!ptr || span <= 0) return false;
        const uintptr_t lo = (uintptr_t)ptr, hi = lo + (uintptr_t)span * elt;
        // the first output whose end lies past lo (ends increase with starts)
        auto it = std::upper_bound(outs.begin(), outs.end(), lo, [](uintptr_t v, const Range& r) { return v < r.hi; });
        if (it != outs.end() && it->lo < hi) {
            *who = it->prob;
            return true;
        }
        return false;
    };
    for (int i = 0; i < count; ++i) {
        const Plan& p = *plans[i]->p;
        if (p.noop || p.m == 0 || p.n == 0 || p.k_empty || alpha[i] == 0.0) continue;
        int who = -1;
        if (meets_output(A[i], p.spanA, &who) || meets_output(B[i], p.spanB, &who)) {
            set_error("an operand of batch problem " + std::to_string(i) + " overlaps the output of problem " +
                      std::to_string(who));
            return TC_ERR_ALIAS;
        }
    }
    return TC_OK;
}

static int batch_create(tc_batch** out, int count, const tc_plan* const* plans, const double* alpha,
                        const void* const* A, const void* const* B, const double* beta, void* const* C) {
    if (!out) {
        set_error("batch out-pointer is NULL");
        return TC_ERR_NULL;
    }
    *out = nullptr;
    if (count < 0) {
        set_error("negative problem count");
        return TC_ERR_ARG;
    }
    if (count > 0 && (!plans || !alpha || !A || !B || !beta || !C)) {
        set_error("NULL batch argument array");
        return TC_ERR_NULL;
    }
    int dtype = TC_F64, mode = TC_NATIVE;
    bool off64 = false;
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) {
            set_error("NULL plan in batch");
            return TC_ERR_NULL;
        }
        const Plan& p = *plans[i]->p;
        if (i == 0) {
            dtype = p.dtype;
            mode = p.mode;
        } else if (p.dtype != dtype || p.mode != mode) {
            set_error("all problems of a batch need the same dtype and mode");
            return TC_ERR_DTYPE;
        }
        off64 |= p.off64;
    }
    if (mode != TC_NATIVE) {
        set_error("batched launches support the native modes");
        return TC_ERR_DTYPE;
    }
    const size_t w = off64 ? 8 : 4, elt = elt_size(dtype);
    // per-problem checks (as tc_plan_execute) and arena layout
    std::vector<size_t> base(count, 0);
    size_t total = 0;
    auto al = [](size_t n) { return (std::max<size_t>(n, 1) + 63) & ~(size_t)63; };
    for (int i = 0; i < count; ++i) {
        const Plan& p = *plans[i]->p;
        if (p.noop || p.m == 0 || p.n == 0) continue;
        const bool reads_ab = !(p.k_empty || alpha[i] == 0.0);
        if (!C[i] || (reads_ab && (!A[i] || !B[i]))) {
            set_error("NULL tensor pointer in batch problem " + std::to_string(i));
            return TC_ERR_NULL;
        }
        if (overlaps(C[i], p.spanC, A[i], p.spanA, elt) || overlaps(C[i], p.spanC, B[i], p.spanB, elt)) {
            set_error("C overlaps A or B in batch problem " + std::to_string(i));
            return TC_ERR_ALIAS;
        }
        base[i] = total;
        total += al(p.rX.size()) + al(p.cX.size()) + al(p.rY.size()) + al(p.cY.size()) + al(p.rC.size()) +
                 al(p.cC.size()) + al(p.kbsX.size()) + al(p.kbsY.size());
    }
    int st = check_batch_aliasing(count, plans, alpha, A, B, C, elt);
    if (st) return st;
    for (int i = 0; i < count; ++i) {
        const Plan& p = *plans[i]->p;
        if (p.noop || p.m == 0 || p.n == 0) continue;
        const bool reads_ab = !(p.k_empty || alpha[i] == 0.0);
        if ((st = check_device_span(C[i], p.spanC, elt, "C")) ||
            (reads_ab && ((st = check_device_span(A[i], p.spanA, elt, "A")) ||
                          (st = check_device_span(B[i], p.spanB, elt, "B"))))) {
            set_error(std::string(last_error()) + " (batch problem " + std::to_string(i) + ")");
            return st;
        }
    }
    auto b = std::make_unique<tc_batch>();
    b->dtype = dtype;
    b->mode = mode;
    b->count = count;
    b->off64 = off64;
    b->host_of.assign((size_t)count, -1);
    hipGetDevice(&b->device);
    std::vector<char> host(std::max<size_t>(total, 1) * w, 0);
    if (total) {
        hipError_t e = hipMalloc(&b->vectors, host.size());
        if (e != hipSuccess) {
            b->vectors = nullptr;
            set_error("hipMalloc of the batch vectors failed");
            return TC_ERR_NOMEM;
        }
    }
    const char* dbase = (const char*)b->vectors;
    for (int i = 0; i < count; ++i) {
        const Plan& p = *plans[i]->p;
        if (p.noop || p.m == 0 || p.n == 0) continue;
        const std::vector<int64_t>* vecs[8] = {&p.rX, &p.cX, &p.rY, &p.cY, &p.rC, &p.cC, &p.kbsX, &p.kbsY};
        const void* ptrs[8];
        size_t o = base[i];
        for (int v = 0; v < 8; ++v) {
            for (size_t j = 0; j < vecs[v]->size(); ++j) {
                if (off64) ((int64_t*)host.data())[o + j] = (*vecs[v])[j];
                else ((int32_t*)host.data())[o + j] = (int32_t)(*vecs[v])[j];
            }
            ptrs[v] = dbase + o * w;
            o += al(vecs[v]->size());
        }
        const bool scale_only = p.k_empty || alpha[i] == 0.0;
        BatchItemDev it{};
        it.X = p.swapped ? B[i] : A[i];
        it.Y = p.swapped ? A[i] : B[i];
        it.C = C[i];
        it.rX = ptrs[0];
        it.cX = ptrs[1];
        it.rY = ptrs[2];
        it.cY = ptrs[3];
        it.rC = ptrs[4];
        it.cC = ptrs[5];
        it.kbsX = ptrs[6];
        it.kbsY = ptrs[7];
        it.m = p.m;
        it.n = p.n;
        it.k = scale_only ? 0 : p.k;
        it.spanX = p.swapped ? p.spanB : p.spanA;
        it.spanY = p.swapped ? p.spanA : p.spanB;
        it.alpha = alpha[i];
        it.beta = beta[i];
        it.x_lanes_m = p.x_lanes_m;
        it.y_lanes_n = p.y_lanes_n;
        it.kregX = p.k_blocks_regular_x == (int64_t)p.kbsX.size();
        it.kregY = p.k_blocks_regular_y == (int64_t)p.kbsY.size();
        auto shared_stride = [](const std::vector<int64_t>& kbs) -> int64_t {
            if (kbs.empty() || kbs[0] == 0) return 0;
            for (int64_t v : kbs)
                if (v != kbs[0]) return 0;
            return kbs[0];
        };
        it.ksX = shared_stride(p.kbsX);
        it.ksY = shared_stride(p.kbsY);
        b->host_of[i] = (int)b->host.size();
        b->host.push_back(it);
        b->best.push_back(choose_tile(p, true));  // layouts a batch runs
        // measured in batches: a sub-blocked k order runs at about half the
        // rate, k blocks without a block stride at about 0.8 of it
        b->slow.push_back(p.sub_a >= 0 ? 2.0 : (it.kregX && it.kregY) ? 1.0 : 1.25);
    }
    if (total) {
        hipError_t e = hipMemcpy(b->vectors, host.data(), total * w, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            tc_batch_destroy(b.release());
            return hipfail(e, "hipMemcpy of the batch vectors");
        }
    }
    b->tile = -1;  // every problem with its own tile class until tuned
    st = batch_layout(b.get());
    if (st) {
        tc_batch_destroy(b.release());
        return st;
    }
    *out = b.release();
    return TC_OK;
}

}  // namespace tc

extern "C" {

int tc_batch_create(tc_batch** batch, int count, const tc_plan* const* plans, const double* alpha,
                    const void* const* A, const void* const* B, const double* beta, void* const* C) {
    try {
        return batch_create(batch, count, plans, alpha, A, B, beta, C);
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return TC_ERR_NOMEM;
    } catch (...) {
        set_error("internal error while building the batch");
        return TC_ERR_ARG;
    }
}

int tc_contract_batched(int count, const tc_problem* probs, int dtype, int mode, void* stream) {
    try {
        if (count < 0) {
            set_error("count < 0");
            return TC_ERR_ARG;
        }
        if (count == 0) return TC_OK;
        if (!probs) {
            set_error("problems is NULL");
            return TC_ERR_NULL;
        }
        if (capturing((hipStream_t)stream)) {
            set_error("tc_contract_batched is synchronous and cannot be captured: capture tc_batch_execute instead");
            return TC_ERR_ARG;
        }
        std::vector<const tc_plan*> plans((size_t)count);
        std::vector<double> alpha((size_t)count), beta((size_t)count);
        std::vector<const void*> A((size_t)count), B((size_t)count);
        std::vector<void*> C((size_t)count);
        for (int i = 0; i < count; ++i) {
            const tc_problem& q = probs[i];
            tc_plan* plan = nullptr;
            int st = cached_plan(g_plans, q.ndim_A, q.lens_A, q.strides_A, q.idx_A, q.ndim_B, q.lens_B, q.strides_B,
                                 q.idx_B, q.ndim_C, q.lens_C, q.strides_C, q.idx_C, dtype, mode, &plan);
            if (st) {
                set_error("problem " + std::to_string(i) + ": " + last_error());
                return st;
            }
            plans[(size_t)i] = plan;
            alpha[(size_t)i] = q.alpha;
            beta[(size_t)i] = q.beta;
            A[(size_t)i] = q.A;
            B[(size_t)i] = q.B;
            C[(size_t)i] = q.C;
        }
        tc_batch* b = nullptr;
        int st = batch_create(&b, count, plans.data(), alpha.data(), A.data(), B.data(), beta.data(), C.data());
        if (st) return st;
        st = tc_batch_execute(b, stream);
        const hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        tc_batch_destroy(b);
        if (st) return st;
        return e == hipSuccess ? TC_OK : hipfail(e, "hipStreamSynchronize after the batch");
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return TC_ERR_NOMEM;
    } catch (...) {
        set_error("internal error in the batched contraction");
        return TC_ERR_ARG;
    }
}

int tc_batch_execute(const tc_batch* batch, void* stream) {
    if (!batch) {
        set_error("batch is NULL");
        return TC_ERR_NULL;
    }
    if (batch->total_items == 0) return TC_OK;
    int dev = 0;
    hipGetDevice(&dev);
    if (dev != batch->device) {
        set_error("batch executed on a device other than the one it was created on");
        return TC_ERR_ARG;
    }
    for (const auto& sg : batch->segs) {
        if (sg.items == 0) continue;
        const int32_t* lists = (const int32_t*)batch->assign;
        int st = launch_batch(batch->dtype, batch->mode, sg.tile, batch->off64,
                              (const BatchItemDev*)batch->table + sg.first, lists + sg.off_pos, lists + sg.ent_pos,
                              sg.items, sg.grid, (hipStream_t)stream);
        if (st) return st;
    }
    return TC_OK;
}

int tc_batch_set_tile(tc_batch* batch, int tile) {
    if (!batch) {
        set_error("batch is NULL");
        return TC_ERR_NULL;
    }
    if (tile < -1 || tile >= tile_count(batch->dtype, batch->mode) ||
        (tile >= 0 && tile_table(batch->dtype, batch->mode)[tile].layout == 1)) {
        set_error("not a tile configuration batches run (regular or specialised-wave) of this dtype/mode");
        return TC_ERR_ARG;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(nullptr, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
        set_error("changing a batch's tile uploads its table: not allowed during capture");
        return TC_ERR_CAPTURE;
    }
    batch->tile = tile;
    return batch_layout(batch);
}

int tc_batch_autotune(tc_batch* batch, int reps, void* stream, double* best_ms) {
    if (!batch) {
        set_error("batch is NULL");
        return TC_ERR_NULL;
    }
    if (reps < 1) reps = 1;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hipfail(e, "hipEventCreate");
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        hipEventDestroy(e0);
        return hipfail(e, "hipEventCreate");
    }
    int best = batch->tile, st = TC_OK;
    float best_t = 1e30f;
    const int nt = tile_count(batch->dtype, batch->mode);
    for (int t = -1; t < nt && st == TC_OK; ++t) {  // -1: every problem with its own class
        if (t >= 0 && tile_table(batch->dtype, batch->mode)[t].layout == 1) continue;
        if ((st = tc_batch_set_tile(batch, t))) break;
        if ((st = tc_batch_execute(batch, s))) break;  // warm-up
        hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == TC_OK; ++r) st = tc_batch_execute(batch, s);
        hipEventRecord(e1, s);
        if ((e = hipEventSynchronize(e1)) != hipSuccess) {
            st = hipfail(e, "batch autotune timing");
            break;
        }
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (ms < best_t) {
            best_t = ms;
            best = t;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    int st2 = tc_batch_set_tile(batch, best);
    if (st) return st;
    if (st2) return st2;
    if (best_ms) *best_ms = best_t;
    return TC_OK;
}

int tc_batch_destroy(tc_batch* batch) {
    if (!batch) return TC_OK;
    if (batch->table) hipFree(batch->table);
    if (batch->vectors) hipFree(batch->vectors);
    if (batch->assign) hipFree(batch->assign);
    delete batch;
    return TC_OK;
}

int tc_batch_info(const tc_batch* batch, int64_t* work_items, int* tile, int* grid) {
    if (!batch) {
        set_error("batch is NULL");
        return TC_ERR_NULL;
    }
    if (work_items) *work_items = batch->total_items;
    if (tile) *tile = batch->tile;
    if (grid) *grid = batch->grid;
    return TC_OK;
}

int tc_batch_problem_tile(const tc_batch* batch, int problem, int* tile) {
    if (!batch || !tile) {
        set_error("batch or tile out-pointer is NULL");
        return TC_ERR_NULL;
    }
    if (problem < 0 || problem >= batch->count) {
        set_error("problem index out of range");
        return TC_ERR_ARG;
    }
    const int h = batch->host_of[(size_t)problem];
    *tile = h < 0 ? -1 : (batch->tile >= 0 ? batch->tile : batch->best[(size_t)h]);
    return TC_OK;
}

int tc_scatter_vector(int ndim, const int64_t* lens, const int64_t* strides, int64_t* out) {
    if (ndim < 0 || ndim > TC_MAX_NDIM) {
        set_error("ndim outside [0, 16]");
        return TC_ERR_NDIM;
    }
    if ((ndim && (!lens || !strides)) || !out) {
        set_error("NULL argument");
        return TC_ERR_NULL;
    }
    std::vector<Dim> dims(ndim);
    for (int i = 0; i < ndim; ++i) {
        if (lens[i] < 0) {
            set_error("negative length");
            return TC_ERR_EXTENT;
        }
        dims[i].len = lens[i];
        dims[i].sX = strides[i];
    }
    std::vector<int64_t> v;
    scatter_vector(dims, 0, &v);
    std::copy(v.begin(), v.end(), out);
    return TC_OK;
}

int tc_block_strides(const int64_t* scat, int64_t len, int64_t b, int64_t* out) {
    if (len < 0 || b < 1) {
        set_error("len must be >= 0 and b >= 1");
        return TC_ERR_ARG;
    }
    if (len > 0 && (!scat || !out)) {
        set_error("NULL argument");
        return TC_ERR_NULL;
    }
    block_strides(scat, len, b, out);
    return TC_OK;
}

int tc_permute(const void* src, void* dst, int ndim, const int64_t* lens, const int64_t* src_strides,
               const int64_t* dst_strides, int dtype, void* stream) {
    if (ndim < 0 || ndim > TC_MAX_NDIM) {
        set_error("ndim outside [0, 16]");
        return TC_ERR_NDIM;
    }
    if (ndim && (!lens || !src_strides || !dst_strides)) {
        set_error("NULL descriptor array");
        return TC_ERR_NULL;
    }
    if (dtype != TC_F64 && dtype != TC_F32) {
        set_error("dtype must be TC_F64 or TC_F32");
        return TC_ERR_DTYPE;
    }
    bool empty = false;
    for (int d = 0; d < ndim; ++d) {
        if (lens[d] < 0) {
            set_error("negative length");
            return TC_ERR_EXTENT;
        }
        if (lens[d] == 0) empty = true;
    }
    if (empty) return TC_OK;
    for (int d = 0; d < ndim; ++d) {
        if (lens[d] > 1 && (src_strides[d] <= 0 || dst_strides[d] <= 0)) {
            set_error("stride <= 0 on a dimension of length > 1");
            return TC_ERR_STRIDE;
        }
    }
    if (!src || !dst) {
        set_error("NULL data pointer");
        return TC_ERR_NULL;
    }
    if (!capturing((hipStream_t)stream)) {
        int64_t ss = 1, ds = 1;
        for (int d = 0; d < ndim; ++d) {
            ss += (lens[d] - 1) * (lens[d] > 1 ? src_strides[d] : 0);
            ds += (lens[d] - 1) * (lens[d] > 1 ? dst_strides[d] : 0);
        }
        const size_t w = elt_size(dtype);
        int st;
        if ((st = check_device_span(src, ss, w, "src")) || (st = check_device_span(dst, ds, w, "dst"))) return st;
    }
    return launch_permute(src, dst, ndim, lens, src_strides, dst_strides, dtype, (hipStream_t)stream);
}

const char* tc_status_string(int status) {
    switch (status) {
        case TC_OK: return "ok";
        case TC_ERR_NULL: return "NULL pointer";
        case TC_ERR_NDIM: return "ndim out of range";
        case TC_ERR_LABEL: return "invalid labels";
        case TC_ERR_EXTENT: return "extent mismatch";
        case TC_ERR_STRIDE: return "invalid stride";
        case TC_ERR_ALIAS: return "output aliases itself or an input";
        case TC_ERR_DTYPE: return "unsupported dtype or mode";
        case TC_ERR_HIP: return "HIP runtime error";
        case TC_ERR_NOMEM: return "out of memory";
        case TC_ERR_ARG: return "invalid argument";
        case TC_ERR_CAPTURE: return "not allowed during graph capture";
        default: return "unknown status";
    }
}

const char* tc_last_error(void) { return last_error(); }

}  // extern "C"
