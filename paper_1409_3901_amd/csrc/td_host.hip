// Host side of the C ABI declared in include/td.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/td.h"
#include "td_common.hpp"

extern "C" hipError_t td_launch_prep(const td::Pools* pl, int blocks, hipStream_t s);
extern "C" hipError_t td_launch_finalize(const td::Pools* pl, hipStream_t s);
extern "C" hipError_t td_launch_subset_plain(int P, int K, int blocks, hipStream_t s, const td::Pools* pl);
extern "C" hipError_t td_launch_subset_filt(int P, int K, int blocks, hipStream_t s, const td::Pools* pl);
extern "C" hipError_t td_launch_exact(int P, int K, int blocks, hipStream_t s, const td::Pools* pl, int all_items);
extern "C" uint64_t td_exact_scratch_bytes(int P);

namespace {

using td::Counters;
using td::Deferred;
using td::Pools;
using td::QueryDesc;
using td::QueryState;

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return TD_ERR_HIP;    \
    } while (0)

constexpr int64_t kDefaultDeferCap = 1 << 25;

uint64_t binom_host(int64_t n, int k) {
    if (k < 0 || n < k) return 0;
    unsigned __int128 r = 1;
    for (int i = 1; i <= k; ++i) {
        r = r * (unsigned __int128)(n - k + i) / (unsigned __int128)i;
    }
    if (r > (unsigned __int128)UINT64_MAX) return UINT64_MAX;
    return (uint64_t)r;
}

int next_pow2(int v) {
    int m = 1;
    while (m < v) m <<= 1;
    return m;
}

// One workspace per (device, stream): device pools and a pinned staging
// buffer for the query descriptors.
struct Workspace {
    int device = -1;
    hipStream_t stream = nullptr;
    // device buffers
    double* x64 = nullptr;
    float* x32 = nullptr;
    float* nrm = nullptr;
    uint64_t* xi = nullptr;
    size_t pts_cap = 0;          // capacity in points*p units
    size_t nrm_cap = 0;          // capacity in points
    QueryDesc* qd = nullptr;
    QueryState* qs = nullptr;
    size_t q_cap = 0;
    Deferred* deferred = nullptr;
    int64_t defer_cap = 0;
    Counters* ctr = nullptr;
    uint8_t* wscratch = nullptr;   // per-block scratch of the subset kernels
    size_t wscratch_cap = 0;
    QueryDesc* qd_host = nullptr;  // pinned
    size_t qd_host_cap = 0;
    hipEvent_t staged = nullptr;   // the last descriptor upload has completed
    hipEvent_t ev[6] = {};
};

struct DeviceCtx {
    uint64_t* binom = nullptr;
    int num_cu = 256;
    std::map<hipStream_t, Workspace*> ws;
};

struct LastCall {
    Workspace* ws = nullptr;
    int nq = 0;
    bool timing = false;
};

std::mutex g_mu;
std::map<int, DeviceCtx*> g_dev;
LastCall g_last;

td_status ensure_device(int dev, DeviceCtx** out) {
    auto it = g_dev.find(dev);
    if (it != g_dev.end()) { *out = it->second; return TD_OK; }
    DeviceCtx* c = new DeviceCtx();
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) c->num_cu = prop.multiProcessorCount;
    std::vector<uint64_t> tab((size_t)td::kBinomN * td::kBinomK);
    for (int n = 0; n < td::kBinomN; ++n)
        for (int k = 0; k < td::kBinomK; ++k) tab[(size_t)n * td::kBinomK + k] = binom_host(n, k);
    if (hipMalloc(&c->binom, tab.size() * sizeof(uint64_t)) != hipSuccess) { delete c; return TD_ERR_OUT_OF_MEMORY; }
    if (hipMemcpy(c->binom, tab.data(), tab.size() * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess) {
        delete c;
        return TD_ERR_HIP;
    }
    g_dev[dev] = c;
    *out = c;
    return TD_OK;
}

template <typename T>
td_status grow(T** p, size_t* cap, size_t need) {
    if (*cap >= need && *p) return TD_OK;
    size_t nc = std::max(need, (size_t)(*cap * 3 / 2));
    if (*p) { hipFree(*p); *p = nullptr; }
    if (hipMalloc(p, nc * sizeof(T)) != hipSuccess) { *cap = 0; return TD_ERR_OUT_OF_MEMORY; }
    *cap = nc;
    return TD_OK;
}

td_status get_workspace(DeviceCtx* dc, int dev, hipStream_t s, Workspace** out) {
    auto it = dc->ws.find(s);
    if (it != dc->ws.end()) { *out = it->second; return TD_OK; }
    Workspace* w = new Workspace();
    w->device = dev;
    w->stream = s;
    if (hipMalloc(&w->ctr, sizeof(Counters)) != hipSuccess) { delete w; return TD_ERR_OUT_OF_MEMORY; }
    if (hipEventCreateWithFlags(&w->staged, hipEventDisableTiming) != hipSuccess) return TD_ERR_HIP;
    for (auto& e : w->ev)
        if (hipEventCreate(&e) != hipSuccess) return TD_ERR_HIP;
    dc->ws[s] = w;
    *out = w;
    return TD_OK;
}

void free_workspace(Workspace* w) {
    if (!w) return;
    hipFree(w->x64);
    hipFree(w->x32);
    hipFree(w->nrm);
    hipFree(w->xi);
    hipFree(w->qd);
    hipFree(w->qs);
    hipFree(w->deferred);
    hipFree(w->ctr);
    hipFree(w->wscratch);
    if (w->qd_host) hipHostFree(w->qd_host);
    if (w->staged) hipEventDestroy(w->staged);
    for (auto& e : w->ev)
        if (e) hipEventDestroy(e);
    delete w;
}

td_status ensure_points(Workspace* w, size_t need) {
    if (w->pts_cap >= need && w->x64) return TD_OK;
    size_t nc = std::max(need, w->pts_cap * 3 / 2);
    hipFree(w->x64);
    hipFree(w->x32);
    hipFree(w->xi);
    w->x64 = nullptr;
    w->x32 = nullptr;
    w->xi = nullptr;
    w->pts_cap = 0;
    if (hipMalloc(&w->x64, nc * sizeof(double)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
    if (hipMalloc(&w->x32, nc * sizeof(float)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
    if (hipMalloc(&w->xi, nc * 2 * sizeof(uint64_t)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
    w->pts_cap = nc;
    return TD_OK;
}

td_options defaults() {
    td_options o;
    std::memset(&o, 0, sizeof(o));
    o.precision = TD_PREC_FP32_FILTERED;
    o.autotune = 1;
    o.chunk = 0;
    o.grid_blocks = 0;
    o.filter_scale = 1.0;
    o.force_exact = 0;
    o.timing = 0;
    o.deferred_capacity = 0;
    return o;
}

td_status check_options(const td_options& o) {
    if (o.precision < 0 || o.precision > 2) return TD_ERR_INVALID_ARG;
    if (o.chunk < 0 || (o.chunk % 64) != 0) return TD_ERR_INVALID_ARG;
    if (o.grid_blocks < 0) return TD_ERR_INVALID_ARG;
    if (!(o.filter_scale >= 0.0)) return TD_ERR_INVALID_ARG;   // rejects NaN
    if (o.deferred_capacity < 0) return TD_ERR_INVALID_ARG;
    return TD_OK;
}

struct Problem {
    const double* X;
    int64_t n;
    int32_t p;
    const double* Z;
    int64_t m;
    int32_t* counts;
};

td_status check_problem(const Problem& pr) {
    if (pr.m < 0) return TD_ERR_INVALID_ARG;
    if (pr.m == 0) return TD_OK;
    if (!pr.X || !pr.Z || !pr.counts) return TD_ERR_INVALID_ARG;
    if (pr.p < 1 || pr.p > TD_MAX_P) return TD_ERR_INVALID_ARG;
    if (pr.n < 1 || pr.n > TD_MAX_N) return TD_ERR_INVALID_ARG;
    return TD_OK;
}

// Shape of the launch for one (p, K) class.
int class_K(int64_t n) { return std::max(64, next_pow2((int)n)) / 64; }

int default_chunk(int p, int64_t n) {
    (void)p;
    (void)n;
    return 256;
}

// The engine behind td_depth_ex (single class).
td_status run_single(const Problem& pr, const td_options& o, hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TD_ERR_NO_DEVICE;
    DeviceCtx* dc = nullptr;
    td_status st = ensure_device(dev, &dc);
    if (st != TD_OK) return st;
    Workspace* w = nullptr;
    st = get_workspace(dc, dev, stream, &w);
    if (st != TD_OK) return st;

    const int p = pr.p;
    const int n = (int)pr.n;
    const int m = (int)pr.m;
    const int M = std::max(64, next_pow2(n));
    const int K = M / 64;
    const int ks = p - 2;
    const int chunk = o.chunk > 0 ? o.chunk : default_chunk(p, n);
    const uint64_t nsub = (p >= 2) ? binom_host(n, ks) : 0;
    const uint64_t ipq = (nsub + chunk - 1) / chunk;

    // workspace sizes
    if ((st = ensure_points(w, (size_t)m * M * p)) != TD_OK) return st;
    if ((st = grow(&w->nrm, &w->nrm_cap, (size_t)m * M)) != TD_OK) return st;
    size_t qcap = w->q_cap;
    if ((st = grow(&w->qd, &qcap, (size_t)m)) != TD_OK) return st;
    size_t qcap2 = w->q_cap;
    if ((st = grow(&w->qs, &qcap2, (size_t)m)) != TD_OK) return st;
    w->q_cap = std::min(qcap, qcap2);
    const int64_t dcap = o.deferred_capacity > 0 ? o.deferred_capacity : kDefaultDeferCap;
    if (w->defer_cap < dcap) {
        hipFree(w->deferred);
        w->deferred = nullptr;
        if (hipMalloc(&w->deferred, (size_t)dcap * sizeof(Deferred)) != hipSuccess) { w->defer_cap = 0; return TD_ERR_OUT_OF_MEMORY; }
        w->defer_cap = dcap;
    }
    // descriptors (pinned staging, reused once the previous upload is done)
    HIPCHK(hipEventSynchronize(w->staged));
    if (w->qd_host_cap < (size_t)m) {
        if (w->qd_host) hipHostFree(w->qd_host);
        w->qd_host = nullptr;
        if (hipHostMalloc(&w->qd_host, (size_t)m * sizeof(QueryDesc)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
        w->qd_host_cap = m;
    }
    int ib = 0;
    while ((1 << ib) < M) ++ib;
    for (int q = 0; q < m; ++q) {
        QueryDesc& d = w->qd_host[q];
        d.X = pr.X;
        d.z = pr.Z + (size_t)q * p;
        d.count = pr.counts + q;
        d.n = n;
        d.p = p;
        d.M = M;
        d.idx_bits = ib;
        d.x_off = (uint64_t)q * M;
        d.item_begin = (uint64_t)q * ipq;
        d.items = (uint32_t)ipq;
        d.cls = 0;
    }
    HIPCHK(hipMemcpyAsync(w->qd, w->qd_host, (size_t)m * sizeof(QueryDesc), hipMemcpyHostToDevice, stream));
    HIPCHK(hipEventRecord(w->staged, stream));

    Pools pl;
    pl.x64 = w->x64;
    pl.x32 = w->x32;
    pl.nrm = w->nrm;
    pl.xi = w->xi;
    pl.binom = dc->binom;
    pl.qs = w->qs;
    pl.qd = w->qd;
    pl.deferred = w->deferred;
    pl.ctr = w->ctr;
    pl.defer_cap = (uint64_t)dcap;
    pl.total_items = ipq * (uint64_t)m;
    pl.num_queries = m;
    pl.chunk = chunk;
    pl.filter_scale = std::isinf(o.filter_scale) ? 3.0e38f : (float)o.filter_scale;
    pl.force_exact = o.force_exact;

    int blocks = o.grid_blocks > 0 ? o.grid_blocks : dc->num_cu * 8;
    if ((uint64_t)blocks > pl.total_items) blocks = (int)std::max<uint64_t>(1, pl.total_items);
    const int xblocks = dc->num_cu * 4;   // exact-tier grid
    uint64_t wsb = std::max<uint64_t>(td::wave_scratch_bytes(M), td_exact_scratch_bytes(p));
    wsb = (wsb + 255) & ~(uint64_t)255;
    if ((st = grow(&w->wscratch, &w->wscratch_cap, (size_t)std::max(blocks, xblocks) * wsb)) != TD_OK) return st;
    pl.wscratch = w->wscratch;
    pl.wscratch_bytes = wsb;

    const bool timing = o.timing != 0;
    if (timing) HIPCHK(hipEventRecord(w->ev[0], stream));
    HIPCHK(td_launch_prep(&pl, std::min(m, dc->num_cu * 4), stream));
    if (timing) HIPCHK(hipEventRecord(w->ev[1], stream));
    if (p >= 2 && pl.total_items > 0) {
        hipError_t e;
        if (o.precision == TD_PREC_FP64_PLAIN) e = td_launch_subset_plain(p, K, blocks, stream, &pl);
        else if (o.precision == TD_PREC_FP32_FILTERED) e = td_launch_subset_filt(p, K, blocks, stream, &pl);
        else e = td_launch_exact(p, K, blocks, stream, &pl, 1);
        if (e != hipSuccess) return TD_ERR_HIP;
        if (timing) HIPCHK(hipEventRecord(w->ev[2], stream));
        if (o.precision == TD_PREC_FP32_FILTERED) {
            e = td_launch_exact(p, K, xblocks, stream, &pl, 0);
            if (e != hipSuccess) return TD_ERR_HIP;
        }
    } else if (timing) {
        HIPCHK(hipEventRecord(w->ev[2], stream));
    }
    if (timing) HIPCHK(hipEventRecord(w->ev[3], stream));
    HIPCHK(td_launch_finalize(&pl, stream));
    if (timing) HIPCHK(hipEventRecord(w->ev[4], stream));
    g_last.ws = w;
    g_last.nq = m;
    g_last.timing = timing;
    return TD_OK;
}

}  // namespace

extern "C" {

td_status td_default_options(td_options* out) {
    if (!out) return TD_ERR_INVALID_ARG;
    *out = defaults();
    return TD_OK;
}

td_status td_depth_ex(const double* X, int64_t n, int32_t p, const double* Z, int64_t m, int32_t* counts,
                      const td_options* opt, void* stream) {
    td_options o = opt ? *opt : defaults();
    td_status st = check_options(o);
    if (st != TD_OK) return st;
    Problem pr{X, n, p, Z, m, counts};
    st = check_problem(pr);
    if (st != TD_OK) return st;
    if (m == 0) return TD_OK;
    if (o.precision == TD_PREC_EXACT) return TD_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TD_ERR_NO_DEVICE;
    return run_single(pr, o, (hipStream_t)stream);
}

td_status td_depth(const double* X, int64_t n, int32_t p, const double* Z, int64_t m, int32_t* counts,
                   void* stream) {
    return td_depth_ex(X, n, p, Z, m, counts, nullptr, stream);
}

td_status td_get_stats(td_stats* out) {
    if (!out) return TD_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    std::memset(out, 0, sizeof(*out));
    Workspace* w = g_last.ws;
    if (!w) return TD_OK;
    HIPCHK(hipDeviceSynchronize());
    Counters c;
    HIPCHK(hipMemcpy(&c, w->ctr, sizeof(c), hipMemcpyDeviceToHost));
    out->subsets_swept = c.swept;
    out->fp64_rechecks = c.fp64_rechecks;
    out->deferred_subsets = c.deferred;
    out->exact_predicates = c.exact_preds;
    out->degenerate_subsets = c.degenerate;
    out->invalid_subsets = c.invalid;
    std::vector<QueryState> qs(g_last.nq);
    if (g_last.nq > 0) {
        HIPCHK(hipMemcpy(qs.data(), w->qs, qs.size() * sizeof(QueryState), hipMemcpyDeviceToHost));
    }
    int dst = 0;
    for (auto& s : qs) dst |= (s.status & 0xff);
    out->device_status = dst;
    if (g_last.timing) {
        float a = 0;
        hipEventElapsedTime(&a, w->ev[0], w->ev[1]);
        out->prep_ms = a;
        hipEventElapsedTime(&a, w->ev[1], w->ev[2]);
        out->subset_ms = a;
        hipEventElapsedTime(&a, w->ev[2], w->ev[3]);
        out->exact_ms = a;
        hipEventElapsedTime(&a, w->ev[3], w->ev[4]);
        out->finalize_ms = a;
        hipEventElapsedTime(&a, w->ev[0], w->ev[4]);
        out->total_ms = a;
    }
    return dst ? TD_ERR_DEVICE_STATUS : TD_OK;
}

const char* td_status_string(td_status s) {
    switch (s) {
        case TD_OK: return "ok";
        case TD_ERR_INVALID_ARG: return "invalid argument";
        case TD_ERR_UNSUPPORTED: return "unsupported request";
        case TD_ERR_OUT_OF_MEMORY: return "out of device memory";
        case TD_ERR_HIP: return "HIP runtime error";
        case TD_ERR_DEVICE_STATUS: return "some queries failed (see device_status)";
        case TD_ERR_NO_DEVICE: return "no HIP device";
    }
    return "unknown status";
}

void td_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_dev) {
        hipSetDevice(kv.first);
        hipDeviceSynchronize();
        for (auto& w : kv.second->ws) free_workspace(w.second);
        hipFree(kv.second->binom);
        delete kv.second;
    }
    g_dev.clear();
    g_last = LastCall();
}

int32_t td_version(void) { return 1; }

td_status td_depth_batched(const td_problem* probs, int32_t num, const td_options* opt, void* stream) {
    if (num < 0 || (num > 0 && !probs)) return TD_ERR_INVALID_ARG;
    if (num == 0) return TD_OK;
    (void)opt;
    (void)stream;
    return TD_ERR_UNSUPPORTED;
}

td_status td_autotune(int32_t p, int64_t n, const td_options* base, void* stream) {
    (void)p;
    (void)n;
    (void)base;
    (void)stream;
    return TD_ERR_UNSUPPORTED;
}

}  // extern "C"
