// Host side of the C ABI declared in include/td.h.
//
// One engine serves td_depth_ex and td_depth_batched.  The queries of a call
// are grouped by class (p, Kk): Kk is the number of points each lane of the
// subset kernel holds, K = sort width / 64 except where the bucketed sweep
// runs a narrower kernel (kernel_k).  Every class gets a contiguous range of work items (a work item
// is `chunk` consecutive subset ranks of one query) and its own persistent
// subset kernel; per-call data (query descriptors, class ranges) lives in
// device memory, so kernel arguments do not change between calls and the
// whole call can be captured once in a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/td.h"
#include "td_adia.hpp"
#include "td_common.hpp"
#include "td_rank.hpp"

extern "C" hipError_t td_launch_init(const td::Pools* pl, hipStream_t s);
extern "C" hipError_t td_launch_prep(const td::Pools* pl, int blocks, hipStream_t s);
extern "C" hipError_t td_launch_finalize(const td::Pools* pl, int blocks, hipStream_t s);
extern "C" hipError_t td_launch_subset_plain(int P, int K, int blocks, hipStream_t s, const td::Pools* pl);
extern "C" hipError_t td_launch_subset_filt(int P, int K, int blocks, hipStream_t s, const td::Pools* pl);
extern "C" hipError_t td_launch_subset_bucket(int P, int K, int blocks, hipStream_t s, const td::Pools* pl);
extern "C" hipError_t td_launch_subset_bucket64(int P, int K, int blocks, hipStream_t s, const td::Pools* pl);
extern "C" hipError_t td_launch_vertex(int P, int K, int blocks, hipStream_t s, const td::Pools* pl);
extern "C" int td_resident_blocks_vertex(int P, int K);
extern "C" int td_resident_blocks_plain(int P, int K);
extern "C" int td_resident_blocks_filt(int P, int K);
extern "C" int td_resident_blocks_bucket(int P, int K);
extern "C" hipError_t td_launch_exact(int P, int K, int blocks, hipStream_t s, const td::Pools* pl, int all_items);
extern "C" uint64_t td_exact_scratch_bytes(int P);
extern "C" hipError_t td_launch_adia_seed(const td::Pools* pl, int nq, td::AdiaSeed* seeds, hipStream_t s);
extern "C" hipError_t td_launch_adia_eval(int P, int K, const td::Pools* pl, const td::AdiaJob* jobs, int njobs,
                                          td::AdiaRes* res, hipStream_t s);
extern "C" hipError_t td_launch_adia_cand(const td::Pools* pl, int nq, const td::AdiaNode* nodes, int nnodes,
                                          uint32_t* kmask, int32_t* kmap, int32_t* kcount, hipStream_t s);

// Workspace of the allocation-free entry point td_depth_noalloc: counters,
// call parameters, the binomial table, the per-query arrays, the deferred
// list and the per-block scratch of one call, carved from this array.  Every
// device the library runs on holds it until the process ends.  In host code
// `scratch` names a host-side stand-in: the device address comes from
// hipGetSymbolAddress (per device, at the first call on that device).
constexpr uint64_t kNoAllocBytes = 128ull << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace {

using td::CallParams;
using td::Counters;
using td::Deferred;
using td::Pools;
using td::QueryDesc;
using td::QueryState;
using td::RedoItem;

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return TD_ERR_HIP;    \
    } while (0)

constexpr int64_t kDefaultDeferCap = 1 << 25;
constexpr uint64_t kMaxRedo = 1ull << 22;   // work items of the float64 pass per call
constexpr int64_t kVertexMaxN = 512;        // the vertex check at p >= 5 keeps 8 points per lane

using td::binom_host;

int next_pow2(int v) {
    int m = 1;
    while (m < v) m <<= 1;
    return m;
}

struct Problem {
    const double* X;
    int64_t n;
    int32_t p;
    const double* Z;
    int64_t m;
    int32_t* counts;
};

// Launch shape of one class.
struct Shape {
    int chunk = 256;
    int blocks = 0;   // 0: auto
};

// Device buffers of one (device, stream) pair.
struct Workspace {
    int device = -1;
    hipStream_t stream = nullptr;
    double* x64 = nullptr;
    double* x64lo = nullptr;
    float* x32 = nullptr;
    uint64_t* xi = nullptr;
    size_t val_cap = 0;         // values (points * p)
    float* nrm = nullptr;
    size_t pts_cap = 0;         // points
    QueryDesc* qd = nullptr;
    QueryState* qs = nullptr;
    size_t q_cap = 0;
    CallParams* cp = nullptr;
    Deferred* deferred = nullptr;
    int64_t defer_cap = 0;
    RedoItem* redo = nullptr;
    uint64_t redo_cap = 0;
    Counters* ctr = nullptr;
    uint8_t* wscratch = nullptr;
    size_t wscratch_cap = 0;
    uint8_t* staging = nullptr;  // pinned: CallParams + QueryDesc[]
    size_t staging_cap = 0;
    hipEvent_t staged = nullptr; // the last upload has completed
    hipEvent_t ev[6] = {};
    uint64_t generation = 0;     // bumped whenever a device buffer moves
    // buffers of Algorithm 3 (td_options.method = TD_METHOD_ADIA)
    td::AdiaSeed* a_seeds = nullptr;
    size_t a_seeds_cap = 0;
    td::AdiaJob* a_jobs = nullptr;
    size_t a_jobs_cap = 0;
    td::AdiaRes* a_res = nullptr;
    size_t a_res_cap = 0;
    td::AdiaNode* a_nodes = nullptr;
    size_t a_nodes_cap = 0;
    uint32_t* a_kmask = nullptr;
    size_t a_kmask_cap = 0;
    int32_t* a_kmap = nullptr;
    size_t a_kmap_cap = 0;
    int32_t* a_kcount = nullptr;
    size_t a_kcount_cap = 0;
    // captured graph of the last batched call
    std::string graph_key;
    hipGraphExec_t graph_exec = nullptr;
};

struct DeviceCtx {
    uint64_t* binom = nullptr;
    int num_cu = 256;
    std::map<hipStream_t, Workspace*> ws;
    std::map<std::string, Shape> tuned;   // (tier, p, K) -> shape
    std::map<std::string, int> resident;  // (tier, p, K) -> blocks per CU
};

struct LastCall {
    uint64_t adia_evaluations = 0;  // Algorithm 3: subsets evaluated in Steps 2-4
    uint64_t adia_candidates = 0;   // and candidate points of Step 5 (summed)
    uint64_t adia_rcom = 0;         // and queries Algorithm 1 answered
    Workspace* ws = nullptr;        // null after an allocation-free call
    int device = -1;
    const Counters* ctr = nullptr;  // device counters and query states of the call
    const QueryState* qs = nullptr;
    int nq = 0;
    int timing = 0;   // 1: per stage, 2: whole call only
    uint64_t redo_cap = 0;  // entries of the float64 pass's work list
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
    td::fill_binom_table(tab.data());
    if (hipMalloc(&c->binom, tab.size() * sizeof(uint64_t)) != hipSuccess) { delete c; return TD_ERR_OUT_OF_MEMORY; }
    if (hipMemcpy(c->binom, tab.data(), tab.size() * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(c->binom);
        delete c;
        return TD_ERR_HIP;
    }
    g_dev[dev] = c;
    *out = c;
    return TD_OK;
}

template <typename T>
td_status grow(Workspace* w, T** p, size_t* cap, size_t need) {
    if (*cap >= need && *p) return TD_OK;
    size_t nc = std::max(need, (size_t)(*cap * 3 / 2));
    if (*p) { hipFree(*p); *p = nullptr; }
    *cap = 0;
    ++w->generation;
    if (hipMalloc(p, nc * sizeof(T)) != hipSuccess) { *p = nullptr; return TD_ERR_OUT_OF_MEMORY; }
    *cap = nc;
    return TD_OK;
}

td_status ensure_values(Workspace* w, size_t need) {
    if (w->val_cap >= need && w->x64 && w->x64lo) return TD_OK;
    size_t nc = std::max(need, w->val_cap * 3 / 2);
    hipFree(w->x64);
    hipFree(w->x64lo);
    hipFree(w->x32);
    hipFree(w->xi);
    w->x64 = nullptr;
    w->x64lo = nullptr;
    w->x32 = nullptr;
    w->xi = nullptr;
    w->val_cap = 0;
    ++w->generation;
    if (hipMalloc(&w->x64, nc * sizeof(double)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
    if (hipMalloc(&w->x64lo, nc * sizeof(double)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
    if (hipMalloc(&w->x32, nc * sizeof(float)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
    if (hipMalloc(&w->xi, nc * 2 * sizeof(uint64_t)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
    w->val_cap = nc;
    return TD_OK;
}

td_status get_workspace(DeviceCtx* dc, int dev, hipStream_t s, Workspace** out) {
    auto it = dc->ws.find(s);
    if (it != dc->ws.end()) { *out = it->second; return TD_OK; }
    Workspace* w = new Workspace();
    w->device = dev;
    w->stream = s;
    if (hipMalloc(&w->ctr, sizeof(Counters)) != hipSuccess) { delete w; return TD_ERR_OUT_OF_MEMORY; }
    if (hipMalloc(&w->cp, sizeof(CallParams)) != hipSuccess) { hipFree(w->ctr); delete w; return TD_ERR_OUT_OF_MEMORY; }
    if (hipEventCreateWithFlags(&w->staged, hipEventDisableTiming) != hipSuccess) return TD_ERR_HIP;
    for (auto& e : w->ev)
        if (hipEventCreate(&e) != hipSuccess) return TD_ERR_HIP;
    dc->ws[s] = w;
    *out = w;
    return TD_OK;
}

void free_workspace(Workspace* w) {
    if (!w) return;
    if (w->graph_exec) hipGraphExecDestroy(w->graph_exec);
    hipFree(w->x64);
    hipFree(w->x64lo);
    hipFree(w->x32);
    hipFree(w->xi);
    hipFree(w->nrm);
    hipFree(w->qd);
    hipFree(w->qs);
    hipFree(w->cp);
    hipFree(w->deferred);
    hipFree(w->redo);
    hipFree(w->ctr);
    hipFree(w->wscratch);
    hipFree(w->a_seeds);
    hipFree(w->a_jobs);
    hipFree(w->a_res);
    hipFree(w->a_nodes);
    hipFree(w->a_kmask);
    hipFree(w->a_kmap);
    hipFree(w->a_kcount);
    if (w->staging) hipHostFree(w->staging);
    if (w->staged) hipEventDestroy(w->staged);
    for (auto& e : w->ev)
        if (e) hipEventDestroy(e);
    delete w;
}

td_options defaults() {
    td_options o;
    std::memset(&o, 0, sizeof(o));
    o.precision = TD_PREC_FP32_FILTERED;
    o.autotune = 1;
    o.filter_scale = 1.0;
    o.prune = 1;
    return o;
}

td_status check_options(const td_options& o) {
    if (o.precision < 0 || o.precision > 2) return TD_ERR_INVALID_ARG;
    if (o.chunk < 0 || (o.chunk % 64) != 0) return TD_ERR_INVALID_ARG;
    if (o.grid_blocks < 0) return TD_ERR_INVALID_ARG;
    if (!(o.filter_scale >= 0.0)) return TD_ERR_INVALID_ARG;   // rejects NaN
    if (o.deferred_capacity < 0) return TD_ERR_INVALID_ARG;
    if (o.sweep < 0 || o.sweep > 1) return TD_ERR_INVALID_ARG;
    if (o.prune < 0 || o.prune > 1) return TD_ERR_INVALID_ARG;
    if (o.method < 0 || o.method > 2) return TD_ERR_INVALID_ARG;
    return TD_OK;
}

td_status check_problem(const Problem& pr) {
    if (pr.m < 0) return TD_ERR_INVALID_ARG;
    if (pr.m == 0) return TD_OK;
    if (!pr.X || !pr.Z || !pr.counts) return TD_ERR_INVALID_ARG;
    if (pr.p < 1 || pr.p > TD_MAX_P) return TD_ERR_INVALID_ARG;
    if (pr.n < 1 || pr.n > TD_MAX_N) return TD_ERR_INVALID_ARG;
    return TD_OK;
}

// Tier of the subset kernels: 0 plain float64, 1 filtered with the full sort,
// 3 filtered with the bucketed sweep.  The exact precision runs a filtered
// kernel with every subset deferred to the exact tier.
int subset_tier(const td_options& o) {
    if (o.precision == TD_PREC_FP64_PLAIN) return td::kPlain;
    return o.sweep == TD_SWEEP_BITONIC ? td::kFilt : td::kFiltBucket;
}

// Tier of one class: at p = 2 the default sweep is the full sort.  A query
// has a single sweep there, with no running minimum of other subsets to bound
// it, so the bucket bounds rarely settle its minimum and most sweeps would be
// walked by one lane (measured at n = 1024: 84% walked, 67 us against 38 us
// for the full sort over 1,024 queries).
int class_tier(int tier, int p) { return (tier == td::kFiltBucket && p == 2) ? td::kFilt : tier; }

// Points per lane of the subset kernel for a sample of n points whose sort
// width is M = 64 K.  The bucketed sweep needs no power-of-two width, so a
// sample of 512 < n <= 896 at p <= 6 runs 10, 12 or 14 points per lane
// instead of 16 (padded points cost the same work as real ones, and fewer
// point registers leave fewer spills).
int kernel_k(int tier, int p, int64_t n, int K) {
    if (tier == td::kFiltBucket && K == 16 && p <= 6 && n <= 896) return (int)((n + 127) / 128) * 2;
    return K;
}

std::string tune_key(int tier, int p, int K) {
    return std::to_string(tier) + ":" + std::to_string(p) + ":" + std::to_string(K);
}

// Blocks of a subset kernel one compute unit holds (queried once per
// device and shape; at least 1).
int resident_blocks(DeviceCtx* dc, int tier, int p, int K) {
    const std::string key = tune_key(tier, p, K);
    auto it = dc->resident.find(key);
    if (it != dc->resident.end()) return it->second;
    int n = tier == 0 ? td_resident_blocks_plain(p, K)
            : tier == 1 ? td_resident_blocks_filt(p, K)
                        : td_resident_blocks_bucket(p, K);
    n = std::max(1, std::min(n, 32));
    dc->resident[key] = n;
    return n;
}

struct ClassPlan {
    int p = 0, K = 0, M = 0;
    int tier = 0;             // subset kernel tier of the class (class_tier)
    int Kk = 0;               // points per lane of the subset kernel
    int chunk = 0;            // subsets per work item
    Shape shape;
    int xblocks = 0;          // exact-tier grid
    uint64_t items = 0;
    uint64_t scratch_off = 0; // bytes
    uint64_t scratch_per_block = 0;
};

struct Plan {
    std::vector<QueryDesc> qd;
    std::vector<ClassPlan> cls;
    size_t values = 0, points = 0, scratch = 0;
    int prep_blocks = 1, fin_blocks = 1;
};

// The class set fits CallParams: (p, Kk) with p = 2..TD_MAX_P and Kk one of
// kernel_k's values (1, 2, 4, 8, 16, and 10, 12, 14 at p <= 6).
static_assert(td::kMaxClasses >= (TD_MAX_P - 1) * 5 + 5 * 3, "every (p, Kk) class of one call");

// Per-query restriction of the subsets swept (Algorithm 3, Step 5): only the
// (p-2)-subsets of the kcount points listed at kmap (device memory), and
// zero_term when the query's minimum is known to be 0.
struct QueryPatch {
    const int32_t* kmap = nullptr;
    int32_t kcount = 0;
    int32_t zero_term = 0;
};

// Subsets a query sweeps: C(n, p-2), or C(kcount, p-2) when restricted.
uint64_t query_subsets(const QueryDesc& d) {
    return binom_host(d.kmap ? d.kcount : d.n, d.p - 2);
}

td_status make_plan(DeviceCtx* dc, const Problem* probs, int num, const td_options& o, Plan* plan,
                    const std::vector<QueryPatch>* patch = nullptr) {
    const int tier = subset_tier(o);
    std::map<std::pair<int, int>, int> slot;
    std::vector<int> qcls;
    // chunk per class: the explicit option, else the class's tuned chunk,
    // else the default below
    for (int i = 0; i < num; ++i) {
        const Problem& pr = probs[i];
        if (pr.m == 0) continue;
        const int M = std::max(64, next_pow2((int)pr.n));
        const int K = M / 64;
        const int ct = class_tier(tier, pr.p);
        const int Kk = kernel_k(ct, pr.p, pr.n, K);
        int ib = 0;
        while ((1 << ib) < M) ++ib;
        int c = -1;
        if (pr.p >= 2) {
            // (p, Kk) fixes M as well: Kk differs from K only for M = 1024
            auto key = std::make_pair((int)pr.p, Kk);
            auto it = slot.find(key);
            if (it == slot.end()) {
                if ((int)plan->cls.size() == td::kMaxClasses) return TD_ERR_UNSUPPORTED;
                c = (int)plan->cls.size();
                slot[key] = c;
                ClassPlan cp;
                cp.p = pr.p;
                cp.tier = ct;
                cp.K = K;
                cp.Kk = Kk;
                cp.M = M;
                cp.chunk = o.chunk;
                auto tt = dc->tuned.find(tune_key(ct, pr.p, Kk));
                if (o.autotune && tt != dc->tuned.end()) {
                    cp.shape = tt->second;
                    if (cp.chunk == 0) cp.chunk = tt->second.chunk;
                }
                if (o.grid_blocks > 0) cp.shape.blocks = o.grid_blocks;
                plan->cls.push_back(cp);
            } else {
                c = it->second;
            }
        }
        for (int64_t q = 0; q < pr.m; ++q) {
            QueryDesc d;
            std::memset(&d, 0, sizeof(d));
            d.X = pr.X;
            d.z = pr.Z + (size_t)q * pr.p;
            d.count = pr.counts + q;
            d.n = (int)pr.n;
            d.p = pr.p;
            d.M = M;
            d.idx_bits = ib;
            d.cls = c;
            if (patch) {
                const QueryPatch& qp = (*patch)[plan->qd.size()];
                d.kmap = qp.kmap;
                d.kcount = qp.kcount;
                d.zero_term = qp.zero_term;
            }
            plan->qd.push_back(d);
            qcls.push_back(c);
        }
    }
    for (size_t c = 0; c < plan->cls.size(); ++c) {
        ClassPlan& cp = plan->cls[c];
        if (cp.chunk != 0) continue;
        // default: 256 ranks per item, halved (down to one batch of 64) while
        // the class has fewer than four items per resident wave, so that a
        // class with little work per query (p = 3, or few queries) still
        // spreads over every compute unit
        cp.chunk = 256;
        const uint64_t want = 4ull * (uint64_t)dc->num_cu * (uint64_t)resident_blocks(dc, cp.tier, cp.p, cp.Kk);
        while (cp.chunk > 64) {
            uint64_t it = 0;
            for (const QueryDesc& d : plan->qd)
                if (d.cls == (int)c) it += (query_subsets(d) + cp.chunk - 1) / cp.chunk;
            if (it >= want) break;
            cp.chunk /= 2;
        }
    }
    // group queries by class so that every class owns a contiguous item range
    std::vector<int> order(plan->qd.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int ca = qcls[a] < 0 ? 1 << 20 : qcls[a], cb = qcls[b] < 0 ? 1 << 20 : qcls[b];
        return ca < cb;
    });
    std::vector<QueryDesc> sorted;
    sorted.reserve(order.size());
    for (int i : order) sorted.push_back(plan->qd[i]);
    plan->qd.swap(sorted);
    uint64_t item = 0;
    size_t vals = 0, pts = 0;
    for (size_t i = 0; i < plan->qd.size(); ++i) {
        QueryDesc& d = plan->qd[i];
        d.v_off = vals;
        d.n_off = pts;
        vals += (size_t)d.M * d.p;
        pts += (size_t)d.M;
        d.item_begin = item;
        d.items = 0;
        if (d.cls >= 0) {
            const uint64_t nsub = query_subsets(d);
            const uint64_t chunk = (uint64_t)plan->cls[d.cls].chunk;
            const uint64_t it = (nsub + chunk - 1) / chunk;
            if (it > 0xffffffffull) return TD_ERR_UNSUPPORTED;
            d.items = (uint32_t)it;
            plan->cls[d.cls].items += it;
            item += it;
        }
    }
    plan->values = vals;
    plan->points = pts;
    uint64_t soff = 0;
    for (ClassPlan& cp : plan->cls) {
        // default: every compute unit filled to the kernel's occupancy
        int blocks = cp.shape.blocks > 0 ? cp.shape.blocks : dc->num_cu * resident_blocks(dc, cp.tier, cp.p, cp.Kk);
        if ((uint64_t)blocks > cp.items) blocks = (int)std::max<uint64_t>(1, cp.items);
        cp.shape.blocks = blocks;
        cp.xblocks = dc->num_cu * 8;   // the exact kernel: 2 waves per SIMD
        uint64_t per = std::max<uint64_t>(td::wave_scratch_bytes(cp.M), td_exact_scratch_bytes(cp.p));
        per = (per + 255) & ~(uint64_t)255;
        cp.scratch_per_block = per;
        cp.scratch_off = soff;
        soff += per * (uint64_t)std::max(blocks, cp.xblocks);
    }
    plan->scratch = std::max<uint64_t>(soff, 256);
    const int nq = (int)plan->qd.size();
    plan->prep_blocks = std::max(1, std::min(nq, dc->num_cu * 4));
    plan->fin_blocks = std::max(1, std::min(1024, (nq + 255) / 256));
    return TD_OK;
}

// Enqueues the kernels of a planned call on `s` (capturable: no memsets).
td_status enqueue(const Plan& plan, const Pools& base, const td_options& o, hipStream_t s, Workspace* w,
                  bool timing) {
    if (timing) HIPCHK(hipEventRecord(w->ev[0], s));
    HIPCHK(td_launch_init(&base, s));
    HIPCHK(td_launch_prep(&base, plan.prep_blocks, s));
    if (timing) HIPCHK(hipEventRecord(w->ev[1], s));
    const int tier = subset_tier(o);
    for (size_t c = 0; c < plan.cls.size(); ++c) {
        const ClassPlan& cp = plan.cls[c];
        if (cp.items == 0) continue;
        Pools pl = base;
        pl.cls = (int)c;
        pl.wscratch_bytes = cp.scratch_per_block;
        hipError_t e = cp.tier == td::kPlain ? td_launch_subset_plain(cp.p, cp.K, cp.shape.blocks, s, &pl)
                       : cp.tier == td::kFilt ? td_launch_subset_filt(cp.p, cp.K, cp.shape.blocks, s, &pl)
                                              : td_launch_subset_bucket(cp.p, cp.Kk, cp.shape.blocks, s, &pl);
        if (e != hipSuccess) return TD_ERR_HIP;
        // the float64 pass of the bucketed sweep (p >= 3): the work items the
        // launch above handed over, usually none
        if (cp.tier == td::kFiltBucket && cp.p >= 3 &&
            td_launch_subset_bucket64(cp.p, cp.Kk, cp.shape.blocks, s, &pl) != hipSuccess)
            return TD_ERR_HIP;
    }
    if (timing) HIPCHK(hipEventRecord(w->ev[2], s));
    if (tier != 0) {
        for (size_t c = 0; c < plan.cls.size(); ++c) {
            const ClassPlan& cp = plan.cls[c];
            if (cp.items == 0) continue;
            Pools pl = base;
            pl.cls = (int)c;
            pl.wscratch_bytes = cp.scratch_per_block;
            if (td_launch_exact(cp.p, cp.K, cp.xblocks, s, &pl, 0) != hipSuccess) return TD_ERR_HIP;
        }
    }
    if (timing) HIPCHK(hipEventRecord(w->ev[3], s));
    HIPCHK(td_launch_finalize(&base, plan.fin_blocks, s));
    if (timing) HIPCHK(hipEventRecord(w->ev[4], s));
    return TD_OK;
}

std::string graph_signature(const Plan& plan, const Pools& pl, const td_options& o, const Workspace* w) {
    std::string k = std::to_string(subset_tier(o)) + "|" + std::to_string(w->generation) + "|" +
                     std::to_string(plan.prep_blocks) + "|" + std::to_string(plan.fin_blocks) + "|" +
                     std::to_string(pl.force_exact) + "|" + std::to_string(pl.filter_scale) + "|" +
                     std::to_string(pl.defer_cap) + "|" + std::to_string(pl.redo_cap) + "|" +
                     std::to_string(pl.sweep_mode) + "|" + std::to_string(pl.prune);
    for (const ClassPlan& cp : plan.cls) {
        k += "|" + std::to_string(cp.p) + "," + std::to_string(cp.tier) + "," + std::to_string(cp.K) + "," +
             std::to_string(cp.Kk) + "," +
             std::to_string(cp.shape.blocks) + "," + std::to_string(cp.scratch_per_block) + "," +
             std::to_string(cp.items > 0);
    }
    return k;
}

// Device buffers, the upload of the call's descriptors and the kernels'
// argument block for a planned call (nq > 0).
td_status setup_call(DeviceCtx* dc, Workspace* w, const Plan& plan, const td_options& o, hipStream_t stream,
                     Pools* out) {
    td_status st;
    const int nq = (int)plan.qd.size();
    // device memory
    if ((st = ensure_values(w, std::max<size_t>(plan.values, 1))) != TD_OK) return st;
    if ((st = grow(w, &w->nrm, &w->pts_cap, std::max<size_t>(plan.points, 1))) != TD_OK) return st;
    if (w->q_cap < (size_t)nq || !w->qd || !w->qs) {
        hipFree(w->qd);
        hipFree(w->qs);
        w->qd = nullptr;
        w->qs = nullptr;
        w->q_cap = 0;
        ++w->generation;
        const size_t nc = std::max((size_t)nq, w->q_cap * 3 / 2);
        if (hipMalloc(&w->qd, nc * sizeof(QueryDesc)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&w->qs, nc * sizeof(QueryState)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
        w->q_cap = nc;
    }
    const int64_t dcap = o.deferred_capacity > 0 ? o.deferred_capacity : kDefaultDeferCap;
    if (w->defer_cap < dcap) {
        hipFree(w->deferred);
        w->deferred = nullptr;
        w->defer_cap = 0;
        ++w->generation;
        if (hipMalloc(&w->deferred, (size_t)dcap * sizeof(Deferred)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
        w->defer_cap = dcap;
    }
    // work items the bucketed sweep may hand to its float64 pass: one entry per
    // item of the largest class, at most kMaxRedo (past that, the subsets
    // that need float64 go to the exact tier one by one)
    uint64_t rcap = 64;
    for (const ClassPlan& cp : plan.cls) rcap = std::max<uint64_t>(rcap, cp.items);
    rcap = std::min<uint64_t>(rcap, kMaxRedo);
    if (w->redo_cap < rcap) {
        hipFree(w->redo);
        w->redo = nullptr;
        w->redo_cap = 0;
        ++w->generation;
        if (hipMalloc(&w->redo, (size_t)rcap * sizeof(RedoItem)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
        w->redo_cap = rcap;
    }
    if ((st = grow(w, &w->wscratch, &w->wscratch_cap, plan.scratch)) != TD_OK) return st;

    // per-call data: pinned staging, reused once the previous upload is done
    HIPCHK(hipEventSynchronize(w->staged));
    const size_t bytes = sizeof(CallParams) + (size_t)nq * sizeof(QueryDesc);
    if (w->staging_cap < bytes) {
        if (w->staging) hipHostFree(w->staging);
        w->staging = nullptr;
        w->staging_cap = 0;
        if (hipHostMalloc(&w->staging, bytes) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
        w->staging_cap = bytes;
    }
    CallParams* cph = reinterpret_cast<CallParams*>(w->staging);
    std::memset(cph, 0, sizeof(CallParams));
    cph->num_queries = nq;
    cph->num_classes = (int)plan.cls.size();
    uint64_t acc = 0;
    for (size_t c = 0; c < plan.cls.size(); ++c) {
        cph->cls_begin[c] = acc;
        acc += plan.cls[c].items;
        cph->cls_end[c] = acc;
        cph->cls_scratch[c] = plan.cls[c].scratch_off;
        cph->cls_chunk[c] = (uint32_t)plan.cls[c].chunk;
    }
    std::memcpy(w->staging + sizeof(CallParams), plan.qd.data(), (size_t)nq * sizeof(QueryDesc));
    HIPCHK(hipMemcpyAsync(w->cp, cph, sizeof(CallParams), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(w->qd, w->staging + sizeof(CallParams), (size_t)nq * sizeof(QueryDesc),
                          hipMemcpyHostToDevice, stream));
    HIPCHK(hipEventRecord(w->staged, stream));

    Pools pl;
    std::memset(&pl, 0, sizeof(pl));
    pl.x64 = w->x64;
    pl.x64lo = w->x64lo;
    pl.x32 = w->x32;
    pl.nrm = w->nrm;
    pl.xi = w->xi;
    pl.binom = dc->binom;
    pl.qs = w->qs;
    pl.qd = w->qd;
    pl.cp = w->cp;
    pl.deferred = w->deferred;
    pl.ctr = w->ctr;
    pl.defer_cap = (uint64_t)dcap;
    pl.redo = w->redo;
    pl.redo_cap = w->redo_cap;
    pl.filter_scale = std::isinf(o.filter_scale) ? 3.0e38f : (float)o.filter_scale;
    pl.force_exact = (o.force_exact || o.precision == TD_PREC_EXACT) ? 1 : 0;
    pl.sweep_mode = o.sweep;
    pl.prune = (o.prune && subset_tier(o) != 0) ? 1 : 0;
    pl.wscratch = w->wscratch;
    *out = pl;
    return TD_OK;
}

td_status run(const Problem* probs, int num, const td_options& o, hipStream_t stream, bool use_graph,
              const std::vector<QueryPatch>* patch = nullptr) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TD_ERR_NO_DEVICE;
    DeviceCtx* dc = nullptr;
    td_status st = ensure_device(dev, &dc);
    if (st != TD_OK) return st;
    Workspace* w = nullptr;
    st = get_workspace(dc, dev, stream, &w);
    if (st != TD_OK) return st;
    Plan plan;
    st = make_plan(dc, probs, num, o, &plan, patch);
    if (st != TD_OK) return st;
    const int nq = (int)plan.qd.size();
    if (nq == 0) return TD_OK;
    Pools pl;
    if ((st = setup_call(dc, w, plan, o, stream, &pl)) != TD_OK) return st;

    g_last.adia_evaluations = 0;
    g_last.adia_candidates = 0;
    g_last.adia_rcom = 0;
    g_last.ws = w;
    g_last.device = w->device;
    g_last.ctr = w->ctr;
    g_last.qs = w->qs;
    g_last.nq = nq;
    g_last.redo_cap = pl.redo_cap;
    if (!use_graph) {
        g_last.timing = o.timing ? 1 : 0;
        return enqueue(plan, pl, o, stream, w, o.timing != 0);
    }
    // graph path: capture once per signature, replay afterwards
    const std::string key = graph_signature(plan, pl, o, w);
    if (key != w->graph_key || !w->graph_exec) {
        if (w->graph_exec) {
            hipGraphExecDestroy(w->graph_exec);
            w->graph_exec = nullptr;
        }
        w->graph_key.clear();
        hipStream_t cs = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            hipStreamDestroy(cs);
            return TD_ERR_HIP;
        }
        const td_status es = enqueue(plan, pl, o, cs, w, false);
        const hipError_t ce = hipStreamEndCapture(cs, &g);
        hipStreamDestroy(cs);
        if (es != TD_OK || ce != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return es != TD_OK ? es : TD_ERR_HIP;
        }
        const hipError_t ie = hipGraphInstantiate(&w->graph_exec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (ie != hipSuccess) {
            w->graph_exec = nullptr;
            return TD_ERR_HIP;
        }
        w->graph_key = key;
    }
    g_last.timing = o.timing ? 2 : 0;
    if (o.timing) HIPCHK(hipEventRecord(w->ev[0], stream));
    HIPCHK(hipGraphLaunch(w->graph_exec, stream));
    if (o.timing) HIPCHK(hipEventRecord(w->ev[4], stream));
    return TD_OK;
}

// ------------------------------------------- Algorithm 3 (ADIA), host side
// The queue of critical (p-1)-sets (Steps 3-4) is kept here; every subset is
// evaluated on the device (adia_eval_kernel), and Step 5 runs the certified
// subset kernels restricted to the candidate points.  Up to kAdiaBatch nodes
// of each query are popped per launch; their results are applied in queue
// order with the deletions of Step 4(b) in between, and a popped node that an
// earlier one deleted is passed over, so the iteration is the sequential
// one.  Readings (as in the oracle): a node's (p-2)-subsets are taken by the
// element left out, first element first; new nodes are appended in ascending
// order of the added point; the seed point of Step 2(c) is the smallest
// index next to a minimising state; Step 5's candidates also hold the points
// of the subset that attained d0 in Step 4.
constexpr size_t kAdiaBatch = 256;

td_status adia_eval(Workspace* w, const Pools& pl, int P, int K, const std::vector<td::AdiaJob>& jobs,
                    std::vector<td::AdiaRes>& res, hipStream_t s) {
    res.resize(jobs.size());
    if (jobs.empty()) return TD_OK;
    td_status st;
    if ((st = grow(w, &w->a_jobs, &w->a_jobs_cap, jobs.size())) != TD_OK) return st;
    if ((st = grow(w, &w->a_res, &w->a_res_cap, jobs.size())) != TD_OK) return st;
    HIPCHK(hipMemcpyAsync(w->a_jobs, jobs.data(), jobs.size() * sizeof(td::AdiaJob), hipMemcpyHostToDevice, s));
    HIPCHK(td_launch_adia_eval(P, K, &pl, w->a_jobs, (int)jobs.size(), w->a_res, s));
    HIPCHK(hipMemcpyAsync(res.data(), w->a_res, jobs.size() * sizeof(td::AdiaRes), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return TD_OK;
}

// Points reported next to a minimising state, ascending.
std::vector<int> adia_points(const td::AdiaRes& r) {
    std::vector<int> t(r.t, r.t + std::min(r.tcount, td::kAdiaTMax));
    std::sort(t.begin(), t.end());
    return t;
}

td_status run_adia(const Problem& pr, const td_options& o, hipStream_t stream) {
    // the paper uses Algorithm 1 for n <= 2p; p < 3 has no descent
    if (pr.p < 3 || pr.n <= 2 * pr.p) {
        const td_status s1 = run(&pr, 1, o, stream, false);
        g_last.adia_rcom = (uint64_t)pr.m;
        return s1;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TD_ERR_NO_DEVICE;
    DeviceCtx* dc = nullptr;
    td_status st = ensure_device(dev, &dc);
    if (st != TD_OK) return st;
    Workspace* w = nullptr;
    if ((st = get_workspace(dc, dev, stream, &w)) != TD_OK) return st;
    // ADIA's value is its own: no bound from the directions +-x_j
    td_options po = o;
    po.prune = 0;
    Plan plan;
    if ((st = make_plan(dc, &pr, 1, po, &plan)) != TD_OK) return st;
    const int nq = (int)plan.qd.size();
    if (nq == 0 || plan.cls.empty()) return TD_OK;
    Pools pl;
    if ((st = setup_call(dc, w, plan, po, stream, &pl)) != TD_OK) return st;
    const int P = pr.p, ks = P - 2, K = plan.cls[0].K;
    // Step 2
    HIPCHK(td_launch_init(&pl, stream));
    HIPCHK(td_launch_prep(&pl, plan.prep_blocks, stream));
    if ((st = grow(w, &w->a_seeds, &w->a_seeds_cap, (size_t)nq)) != TD_OK) return st;
    HIPCHK(td_launch_adia_seed(&pl, nq, w->a_seeds, stream));
    std::vector<td::AdiaSeed> seeds((size_t)nq);
    HIPCHK(hipMemcpyAsync(seeds.data(), w->a_seeds, (size_t)nq * sizeof(td::AdiaSeed), hipMemcpyDeviceToHost,
                          stream));
    HIPCHK(hipStreamSynchronize(stream));
    enum { kAdia = 0, kZero = 1, kRcom = 2 };
    struct QueryRun {
        int mode = kRcom;
        std::map<std::vector<int>, int> Q;
        std::deque<std::vector<int>> N;
        int d0 = 0;
        std::vector<int> bestJ;
        uint64_t evals = 0;
    };
    std::vector<QueryRun> R((size_t)nq);
    uint64_t evaluations = 0;
    // Step 2(c): the seed subsets
    std::vector<td::AdiaJob> jobs;
    std::vector<int> jq;
    for (int q = 0; q < nq; ++q) {
        if (seeds[q].kneg == 0) { R[q].mode = kZero; continue; }
        if (!seeds[q].ok) continue;
        td::AdiaJob j;
        std::memset(&j, 0, sizeof(j));
        j.q = q;
        std::vector<int> I(seeds[q].idx, seeds[q].idx + ks);
        std::sort(I.begin(), I.end());
        for (int c = 0; c < ks; ++c) j.idx[c] = I[c];
        jobs.push_back(j);
        jq.push_back(q);
    }
    std::vector<td::AdiaRes> res;
    if ((st = adia_eval(w, pl, P, K, jobs, res, stream)) != TD_OK) return st;
    evaluations += jobs.size();
    for (size_t e = 0; e < jobs.size(); ++e) {
        QueryRun& qr = R[(size_t)jq[e]];
        std::vector<int> I(jobs[e].idx, jobs[e].idx + ks);
        // no seed, or more points next to a minimising state than an
        // evaluation lists: the query takes Algorithm 1
        if (res[e].term < 0 || res[e].tcount > td::kAdiaTMax) continue;
        int h = -1;
        for (int v : adia_points(res[e]))
            if (std::find(I.begin(), I.end(), v) == I.end()) { h = v; break; }
        if (h < 0) continue;
        std::vector<int> C0 = I;
        C0.push_back(h);
        std::sort(C0.begin(), C0.end());
        qr.mode = kAdia;
        qr.Q[C0] = res[e].term;
        qr.N.push_back(C0);
        qr.d0 = res[e].term;
        qr.bestJ = I;
    }
    // Steps 3-4
    while (true) {
        jobs.clear();
        std::vector<std::vector<std::vector<int>>> popped((size_t)nq);
        for (int q = 0; q < nq; ++q) {
            QueryRun& qr = R[(size_t)q];
            if (qr.mode != kAdia) continue;
            // a descent longer than the full enumeration gains nothing: that
            // query falls back to Algorithm 1
            if (qr.evals > 4 * binom_host(pr.n, ks) + 4096) {
                qr.mode = kRcom;
                continue;
            }
            while (!qr.N.empty() && popped[(size_t)q].size() < kAdiaBatch) {
                const std::vector<int> F = qr.N.front();
                qr.N.pop_front();
                for (int r = 0; r < ks + 1; ++r) {
                    td::AdiaJob j;
                    std::memset(&j, 0, sizeof(j));
                    j.q = q;
                    int c2 = 0;
                    for (int c = 0; c < ks + 1; ++c)
                        if (c != r) j.idx[c2++] = F[(size_t)c];
                    jobs.push_back(j);
                }
                popped[(size_t)q].push_back(F);
            }
        }
        if (jobs.empty()) break;
        if ((st = adia_eval(w, pl, P, K, jobs, res, stream)) != TD_OK) return st;
        evaluations += jobs.size();
        size_t e0 = 0;
        for (int q = 0; q < nq; ++q) {
            QueryRun& qr = R[(size_t)q];
            if (qr.mode != kAdia) {
                e0 += popped[(size_t)q].size() * ((size_t)ks + 1);
                continue;
            }
            for (const std::vector<int>& F : popped[(size_t)q]) {
                const size_t base = e0;
                e0 += (size_t)ks + 1;
                // deleted by an earlier node (not popped), or the query left
                // the descent
                if (qr.mode != kAdia || !qr.Q.count(F)) continue;
                qr.evals += (uint64_t)ks + 1;   // the descent's own work (not the speculation)
                bool listed = true;
                for (int r = 0; r < ks + 1; ++r) {
                    const td::AdiaRes& rr = res[base + (size_t)r];
                    if (rr.term < 0) continue;
                    // the set T of Step 4(a)(ii) is longer than an evaluation
                    // lists: the query takes Algorithm 1
                    if (rr.tcount > td::kAdiaTMax) {
                        listed = false;
                        break;
                    }
                    std::vector<int> J(jobs[base + (size_t)r].idx, jobs[base + (size_t)r].idx + ks);
                    for (int v : adia_points(rr)) {
                        if (std::find(F.begin(), F.end(), v) != F.end()) continue;
                        std::vector<int> Nn = J;
                        Nn.push_back(v);
                        std::sort(Nn.begin(), Nn.end());
                        if (!qr.Q.count(Nn)) {
                            qr.Q[Nn] = rr.term;
                            qr.N.push_back(Nn);
                        }
                    }
                    if (qr.d0 > rr.term) {
                        qr.d0 = rr.term;
                        qr.bestJ = J;
                        break;
                    }
                }
                if (!listed) {
                    qr.mode = kRcom;
                    continue;
                }
                for (auto it = qr.Q.begin(); it != qr.Q.end();) {
                    if (it->second > qr.d0) it = qr.Q.erase(it); else ++it;
                }
                std::deque<std::vector<int>> keep;
                for (auto& f : qr.N)
                    if (qr.Q.count(f)) keep.push_back(f);
                qr.N.swap(keep);
            }
        }
    }
    // Step 5(a): candidate points
    std::vector<td::AdiaNode> nodes;
    for (int q = 0; q < nq; ++q) {
        const QueryRun& qr = R[(size_t)q];
        if (qr.mode != kAdia) continue;
        for (const auto& e : qr.Q) {
            td::AdiaNode nd;
            std::memset(&nd, 0, sizeof(nd));
            nd.q = q;
            nd.count = ks + 1;
            for (int c = 0; c <= ks; ++c) nd.idx[c] = e.first[(size_t)c];
            nodes.push_back(nd);
        }
        td::AdiaNode nd;
        std::memset(&nd, 0, sizeof(nd));
        nd.q = q;
        nd.count = ks;
        for (int c = 0; c < ks; ++c) nd.idx[c] = qr.bestJ[(size_t)c];
        nodes.push_back(nd);
    }
    if ((st = grow(w, &w->a_nodes, &w->a_nodes_cap, std::max<size_t>(nodes.size(), 1))) != TD_OK) return st;
    if ((st = grow(w, &w->a_kmask, &w->a_kmask_cap, (size_t)nq * (td::kMaxN / 32))) != TD_OK) return st;
    if ((st = grow(w, &w->a_kmap, &w->a_kmap_cap, (size_t)nq * td::kMaxN)) != TD_OK) return st;
    if ((st = grow(w, &w->a_kcount, &w->a_kcount_cap, (size_t)nq)) != TD_OK) return st;
    if (!nodes.empty())
        HIPCHK(hipMemcpyAsync(w->a_nodes, nodes.data(), nodes.size() * sizeof(td::AdiaNode), hipMemcpyHostToDevice,
                              stream));
    HIPCHK(td_launch_adia_cand(&pl, nq, w->a_nodes, (int)nodes.size(), w->a_kmask, w->a_kmap, w->a_kcount, stream));
    std::vector<int32_t> kcount((size_t)nq);
    HIPCHK(hipMemcpyAsync(kcount.data(), w->a_kcount, (size_t)nq * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    // Step 5(b): the certified sweeps over the candidates' subsets
    std::vector<QueryPatch> patch((size_t)nq);
    uint64_t cands = 0;
    for (int q = 0; q < nq; ++q) {
        if (R[(size_t)q].mode == kAdia) {
            patch[(size_t)q].kmap = w->a_kmap + (size_t)q * td::kMaxN;
            patch[(size_t)q].kcount = kcount[(size_t)q];
            cands += (uint64_t)kcount[(size_t)q];
        } else if (R[(size_t)q].mode == kZero) {
            patch[(size_t)q].kmap = w->a_kmap;   // no subset: the minimum is 0
            patch[(size_t)q].kcount = 0;
            patch[(size_t)q].zero_term = 1;
        }
    }
    st = run(&pr, 1, po, stream, false, &patch);
    g_last.adia_evaluations = evaluations;
    g_last.adia_candidates = cands;
    for (int q = 0; q < nq; ++q) g_last.adia_rcom += R[(size_t)q].mode == kRcom ? 1 : 0;
    return st;
}

// ------------------------------------------------ vertex-form check
// Proposition 1 with r = p - 1: the count from the (p-1)-subsets (one
// hyperplane each), certified in float64; a query with an undecided side
// reports TD_DEV_NOT_GENERAL.  Work items are chunks of colex ranks of
// (p-1)-subsets; n <= 512 (8 points per lane), or n <= 1024 at p <= 4 (16);
// p = 1 is the closed form of the preparation kernel, as for Algorithm 1.
td_status run_vertex(const Problem& pr, const td_options& o, hipStream_t stream) {
    if (pr.p < 2) return run(&pr, 1, o, stream, false);
    if (pr.n > (pr.p <= 4 ? (int64_t)TD_MAX_N : kVertexMaxN)) return TD_ERR_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TD_ERR_NO_DEVICE;
    DeviceCtx* dc = nullptr;
    td_status st = ensure_device(dev, &dc);
    if (st != TD_OK) return st;
    Workspace* w = nullptr;
    if ((st = get_workspace(dc, dev, stream, &w)) != TD_OK) return st;
    // the vertex count is its own: no bound from the directions +-x_j
    td_options po = o;
    po.prune = 0;
    Plan plan;
    if ((st = make_plan(dc, &pr, 1, po, &plan)) != TD_OK) return st;
    if (plan.qd.empty() || plan.cls.empty()) return TD_OK;
    // items over the (p-1)-subsets (queries are grouped by class)
    for (ClassPlan& cp : plan.cls) cp.items = 0;
    uint64_t item = 0;
    for (QueryDesc& d : plan.qd) {
        d.item_begin = item;
        d.items = 0;
        if (d.cls < 0) continue;
        const uint64_t chunk = (uint64_t)plan.cls[d.cls].chunk;
        const uint64_t it = (binom_host(d.n, d.p - 1) + chunk - 1) / chunk;
        if (it > 0xffffffffull) return TD_ERR_UNSUPPORTED;
        d.items = (uint32_t)it;
        plan.cls[d.cls].items += it;
        item += it;
    }
    Pools pl;
    if ((st = setup_call(dc, w, plan, po, stream, &pl)) != TD_OK) return st;
    g_last.adia_evaluations = 0;
    g_last.adia_candidates = 0;
    g_last.adia_rcom = 0;
    g_last.ws = w;
    g_last.device = w->device;
    g_last.ctr = w->ctr;
    g_last.qs = w->qs;
    g_last.nq = (int)plan.qd.size();
    g_last.redo_cap = pl.redo_cap;
    g_last.timing = 0;
    HIPCHK(td_launch_init(&pl, stream));
    HIPCHK(td_launch_prep(&pl, plan.prep_blocks, stream));
    for (size_t c = 0; c < plan.cls.size(); ++c) {
        const ClassPlan& cp = plan.cls[c];
        if (cp.items == 0) continue;
        Pools pc = pl;
        pc.cls = (int)c;
        const int rb = std::max(1, td_resident_blocks_vertex(cp.p, cp.K));
        const int blocks = (int)std::min<uint64_t>(cp.items, (uint64_t)dc->num_cu * (uint64_t)rb);
        HIPCHK(td_launch_vertex(cp.p, cp.K, blocks, stream, &pc));
    }
    HIPCHK(td_launch_finalize(&pl, plan.fin_blocks, stream));
    return TD_OK;
}

// ------------------------------------------------ allocation-free call
constexpr int kNoAllocMaxDevices = 64;
constexpr uint64_t kNoAllocDeferCap = 1ull << 18;   // deferred subsets per call
constexpr uint64_t kNoAllocRedoCap = 1ull << 16;    // work items of the float64 pass

struct NoAllocDev {
    uint8_t* base = nullptr;    // device address of `scratch` on this device
    DeviceCtx* ctx = nullptr;   // launch-shape bookkeeping (host only; no binom)
};
NoAllocDev g_noalloc[kNoAllocMaxDevices];

// Byte offsets of one call's arrays inside `scratch` (256-byte aligned).
struct NoAllocLayout {
    uint64_t ctr, cp, binom, qd, qs, x64, x64lo, x32, xi, nrm, deferred, redo, ws, end;
};

uint64_t up256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

NoAllocLayout noalloc_layout(uint64_t m, uint64_t M, uint64_t p, uint64_t ws_bytes) {
    NoAllocLayout L;
    uint64_t o = 0;
    L.ctr = o;      o = up256(o + sizeof(Counters));
    L.cp = o;       o = up256(o + sizeof(CallParams));
    L.binom = o;    o = up256(o + (uint64_t)td::kBinomN * td::kBinomK * sizeof(uint64_t));
    L.qd = o;       o = up256(o + m * sizeof(QueryDesc));
    L.qs = o;       o = up256(o + m * sizeof(QueryState));
    const uint64_t vals = m * M * p, pts = m * M;
    L.x64 = o;      o = up256(o + vals * sizeof(double));
    L.x64lo = o;    o = up256(o + vals * sizeof(double));
    L.x32 = o;      o = up256(o + vals * sizeof(float));
    L.xi = o;       o = up256(o + vals * 2 * sizeof(uint64_t));
    L.nrm = o;      o = up256(o + pts * sizeof(float));
    L.deferred = o; o = up256(o + kNoAllocDeferCap * sizeof(Deferred));
    L.redo = o;     o = up256(o + kNoAllocRedoCap * sizeof(RedoItem));
    L.ws = o;       o = up256(o + ws_bytes);
    L.end = o;
    return L;
}

// Per-call descriptors written on the device (no host staging): the class
// ranges of CallParams and one QueryDesc per query of the single problem.
struct NoAllocArgs {
    CallParams* cp;
    QueryDesc* qd;
    const double* X;
    const double* Z;
    int32_t* counts;
    int32_t n, p, m, M, idx_bits, cls;
    uint32_t items_per_query, chunk;
    uint64_t scratch_off;   // class scratch offset (bytes, from pl.wscratch)
};

__global__ void noalloc_setup_kernel(NoAllocArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        CallParams c;
        memset(&c, 0, sizeof(c));
        c.num_queries = a.m;
        c.num_classes = a.cls >= 0 ? 1 : 0;
        c.cls_begin[0] = 0;
        c.cls_end[0] = a.cls >= 0 ? (uint64_t)a.items_per_query * (uint64_t)a.m : 0;
        c.cls_scratch[0] = a.scratch_off;
        c.cls_chunk[0] = a.chunk;
        *a.cp = c;
    }
    for (int q = t; q < a.m; q += gridDim.x * blockDim.x) {
        QueryDesc d;
        memset(&d, 0, sizeof(d));
        d.X = a.X;
        d.z = a.Z + (size_t)q * a.p;
        d.count = a.counts + q;
        d.n = a.n;
        d.p = a.p;
        d.M = a.M;
        d.idx_bits = a.idx_bits;
        d.v_off = (uint64_t)q * (uint64_t)a.M * (uint64_t)a.p;
        d.n_off = (uint64_t)q * (uint64_t)a.M;
        d.items = a.cls >= 0 ? a.items_per_query : 0;
        d.item_begin = (uint64_t)q * (uint64_t)d.items;
        d.cls = a.cls;
        a.qd[q] = d;
    }
}

// First call on a device: the device address of `scratch` (with that device
// current) and the binomial table copied into it once.
td_status noalloc_device(int dev, NoAllocDev** out) {
    if (dev < 0 || dev >= kNoAllocMaxDevices) return TD_ERR_UNSUPPORTED;
    NoAllocDev& d = g_noalloc[dev];
    if (!d.base) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TD_ERR_HIP;
        static uint64_t tab[(size_t)td::kBinomN * td::kBinomK];
        td::fill_binom_table(tab);
        const NoAllocLayout L = noalloc_layout(0, 0, 0, 0);
        if (hipMemcpy((uint8_t*)ptr + L.binom, tab, sizeof(tab), hipMemcpyHostToDevice) != hipSuccess)
            return TD_ERR_HIP;
        if (!d.ctx) {
            d.ctx = new DeviceCtx();
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess) d.ctx->num_cu = prop.multiProcessorCount;
        }
        d.base = (uint8_t*)ptr;
    }
    *out = &d;
    return TD_OK;
}

td_status run_noalloc(const Problem& pr, const td_options& o, hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TD_ERR_NO_DEVICE;
    NoAllocDev* nd = nullptr;
    td_status st = noalloc_device(dev, &nd);
    if (st != TD_OK) return st;
    DeviceCtx* dc = nd->ctx;
    // the plan of the single problem (one class; none at p = 1); the tuned
    // shapes of the allocating path are not consulted
    td_options po = o;
    po.autotune = 0;
    Plan plan;
    st = make_plan(dc, &pr, 1, po, &plan);
    if (st != TD_OK) return st;
    const uint64_t m = (uint64_t)pr.m;
    const uint64_t M = (uint64_t)std::max(64, next_pow2((int)pr.n));
    int blocks = 0, xblocks = 0;
    uint64_t per = 256;
    if (!plan.cls.empty()) {
        ClassPlan& cp = plan.cls[0];
        per = cp.scratch_per_block;
        blocks = cp.items > 0 ? cp.shape.blocks : 0;
        xblocks = std::min(cp.xblocks, dc->num_cu);
    }
    // shrink the grids to what `scratch` holds after the fixed arrays
    const NoAllocLayout L0 = noalloc_layout(m, M, (uint64_t)pr.p, 0);
    if (L0.end > kNoAllocBytes) return TD_ERR_TOO_LARGE;
    const uint64_t fit = (kNoAllocBytes - L0.end) / per;
    if (!plan.cls.empty() && plan.cls[0].items > 0) {
        if (fit < 1) return TD_ERR_TOO_LARGE;
        blocks = (int)std::min<uint64_t>((uint64_t)blocks, fit);
        xblocks = (int)std::min<uint64_t>((uint64_t)std::max(xblocks, 1), fit);
        plan.cls[0].shape.blocks = blocks;
        plan.cls[0].xblocks = xblocks;
        plan.cls[0].scratch_off = 0;
    }
    const uint64_t ws_bytes = per * (uint64_t)std::max(blocks, xblocks);
    const NoAllocLayout L = noalloc_layout(m, M, (uint64_t)pr.p, ws_bytes);
    if (L.end > kNoAllocBytes) return TD_ERR_TOO_LARGE;

    uint8_t* b = nd->base;
    Pools pl;
    std::memset(&pl, 0, sizeof(pl));
    pl.x64 = reinterpret_cast<double*>(b + L.x64);
    pl.x64lo = reinterpret_cast<double*>(b + L.x64lo);
    pl.x32 = reinterpret_cast<float*>(b + L.x32);
    pl.nrm = reinterpret_cast<float*>(b + L.nrm);
    pl.xi = reinterpret_cast<uint64_t*>(b + L.xi);
    pl.binom = reinterpret_cast<const uint64_t*>(b + L.binom);
    pl.qs = reinterpret_cast<QueryState*>(b + L.qs);
    pl.qd = reinterpret_cast<const QueryDesc*>(b + L.qd);
    pl.cp = reinterpret_cast<const CallParams*>(b + L.cp);
    pl.deferred = reinterpret_cast<Deferred*>(b + L.deferred);
    pl.ctr = reinterpret_cast<Counters*>(b + L.ctr);
    pl.defer_cap = std::min<uint64_t>(kNoAllocDeferCap, o.deferred_capacity > 0 ? (uint64_t)o.deferred_capacity
                                                                                : kNoAllocDeferCap);
    pl.redo = reinterpret_cast<RedoItem*>(b + L.redo);
    pl.redo_cap = kNoAllocRedoCap;
    pl.filter_scale = std::isinf(o.filter_scale) ? 3.0e38f : (float)o.filter_scale;
    pl.force_exact = (o.force_exact || o.precision == TD_PREC_EXACT) ? 1 : 0;
    pl.sweep_mode = o.sweep;
    pl.prune = (o.prune && subset_tier(o) != 0) ? 1 : 0;
    pl.wscratch = b + L.ws;

    NoAllocArgs a;
    a.cp = reinterpret_cast<CallParams*>(b + L.cp);
    a.qd = reinterpret_cast<QueryDesc*>(b + L.qd);
    a.X = pr.X;
    a.Z = pr.Z;
    a.counts = pr.counts;
    a.n = (int32_t)pr.n;
    a.p = pr.p;
    a.m = (int32_t)pr.m;
    a.M = (int32_t)M;
    a.idx_bits = plan.qd[0].idx_bits;
    a.cls = plan.qd[0].cls;
    a.items_per_query = plan.qd[0].items;
    a.chunk = plan.cls.empty() ? 64u : (uint32_t)plan.cls[0].chunk;
    a.scratch_off = 0;
    const int sblocks = (int)std::min<uint64_t>(1024, (m + 255) / 256);
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3(std::max(sblocks, 1)), dim3(256), 0, stream, a);
    HIPCHK(hipGetLastError());

    g_last.adia_evaluations = 0;
    g_last.adia_candidates = 0;
    g_last.adia_rcom = 0;
    g_last.ws = nullptr;
    g_last.device = dev;
    g_last.ctr = pl.ctr;
    g_last.redo_cap = pl.redo_cap;
    g_last.qs = pl.qs;
    g_last.nq = (int)m;
    g_last.timing = 0;
    return enqueue(plan, pl, o, stream, nullptr, false);
}

// Deterministic synthetic points for the autotuner: sums of four uniforms
// from a 64-bit LCG, centred and scaled (plumbing only, no depth arithmetic).
void synth(std::vector<double>& v, size_t count, uint64_t seed) {
    v.resize(count);
    uint64_t s = seed * 6364136223846793005ull + 1442695040888963407ull;
    for (size_t i = 0; i < count; ++i) {
        double acc = 0.0;
        for (int k = 0; k < 4; ++k) {
            s = s * 6364136223846793005ull + 1442695040888963407ull;
            acc += (double)(s >> 11) * (1.0 / 9007199254740992.0);
        }
        v[i] = (acc - 2.0) * 1.7320508075688772;
    }
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
    std::lock_guard<std::mutex> lk(g_mu);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TD_ERR_NO_DEVICE;
    if (o.method == TD_METHOD_ADIA) return run_adia(pr, o, (hipStream_t)stream);
    if (o.method == TD_METHOD_VERTEX) return run_vertex(pr, o, (hipStream_t)stream);
    return run(&pr, 1, o, (hipStream_t)stream, false);
}

td_status td_depth(const double* X, int64_t n, int32_t p, const double* Z, int64_t m, int32_t* counts,
                   void* stream) {
    return td_depth_ex(X, n, p, Z, m, counts, nullptr, stream);
}

td_status td_depth_batched(const td_problem* probs, int32_t num, const td_options* opt, void* stream) {
    if (num < 0 || (num > 0 && !probs)) return TD_ERR_INVALID_ARG;
    if (num == 0) return TD_OK;
    td_options o = opt ? *opt : defaults();
    td_status st = check_options(o);
    if (st != TD_OK) return st;
    if (o.method != TD_METHOD_RCOM) return TD_ERR_UNSUPPORTED;
    std::vector<Problem> pv(num);
    int64_t total = 0;
    for (int i = 0; i < num; ++i) {
        pv[i] = Problem{probs[i].X, probs[i].n, probs[i].p, probs[i].Z, probs[i].m, probs[i].counts};
        st = check_problem(pv[i]);
        if (st != TD_OK) return st;
        total += pv[i].m;
    }
    if (total == 0) return TD_OK;
    if (total > (int64_t)1 << 30) return TD_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TD_ERR_NO_DEVICE;
    return run(pv.data(), num, o, (hipStream_t)stream, true);
}

td_status td_depth_noalloc(const double* X, int64_t n, int32_t p, const double* Z, int64_t m, int32_t* counts,
                           const td_options* opt, void* stream) {
    td_options o = opt ? *opt : defaults();
    td_status st = check_options(o);
    if (st != TD_OK) return st;
    if (o.method != TD_METHOD_RCOM) return TD_ERR_UNSUPPORTED;
    Problem pr{X, n, p, Z, m, counts};
    st = check_problem(pr);
    if (st != TD_OK) return st;
    if (m == 0) return TD_OK;
    if (m > (int64_t)1 << 30) return TD_ERR_TOO_LARGE;
    std::lock_guard<std::mutex> lk(g_mu);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TD_ERR_NO_DEVICE;
    return run_noalloc(pr, o, (hipStream_t)stream);
}

td_status td_get_stats(td_stats* out) {
    if (!out) return TD_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    std::memset(out, 0, sizeof(*out));
    Workspace* w = g_last.ws;
    if (!g_last.ctr) return TD_OK;
    HIPCHK(hipSetDevice(g_last.device));
    HIPCHK(hipDeviceSynchronize());
    Counters c;
    HIPCHK(hipMemcpy(&c, g_last.ctr, sizeof(c), hipMemcpyDeviceToHost));
    out->subsets_swept = c.swept;
    out->fp64_rechecks = c.fp64_rechecks;
    out->deferred_subsets = c.deferred;
    out->exact_predicates = c.exact_preds;
    out->degenerate_subsets = c.degenerate;
    out->invalid_subsets = c.invalid;
    out->walked_sweeps = c.walked;
    out->pruned_subsets = c.pruned;
    out->exact_subsets = c.exact_done;
    out->adia_evaluations = g_last.adia_evaluations;
    out->adia_candidates = g_last.adia_candidates;
    out->adia_rcom_queries = g_last.adia_rcom;
    for (int k = 0; k < td::kMaxClasses; ++k) out->f64_items += std::min<uint64_t>(c.redo_count[k], g_last.redo_cap);
    std::vector<QueryState> qs(g_last.nq);
    if (g_last.nq > 0) HIPCHK(hipMemcpy(qs.data(), g_last.qs, qs.size() * sizeof(QueryState), hipMemcpyDeviceToHost));
    int dst = 0;
    for (auto& s : qs) dst |= (s.status & 0xff);
    out->device_status = dst;
    float a = 0;
    if (g_last.timing == 1 && w) {
        hipEventElapsedTime(&a, w->ev[0], w->ev[1]);
        out->prep_ms = a;
        hipEventElapsedTime(&a, w->ev[1], w->ev[2]);
        out->subset_ms = a;
        hipEventElapsedTime(&a, w->ev[2], w->ev[3]);
        out->exact_ms = a;
        hipEventElapsedTime(&a, w->ev[3], w->ev[4]);
        out->finalize_ms = a;
    }
    if (g_last.timing && w) {
        hipEventElapsedTime(&a, w->ev[0], w->ev[4]);
        out->total_ms = a;
    }
    return dst ? TD_ERR_DEVICE_STATUS : TD_OK;
}

td_status td_autotune(int32_t p, int64_t n, const td_options* base, void* stream) {
    td_options o = base ? *base : defaults();
    td_status st = check_options(o);
    if (st != TD_OK) return st;
    if (p < 2 || p > TD_MAX_P || n < 1 || n > TD_MAX_N) return TD_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TD_ERR_NO_DEVICE;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipStream_t s = (hipStream_t)stream;
    // synthetic problem of the requested shape (4 queries)
    const int m = 4;
    std::vector<double> hx, hz;
    synth(hx, (size_t)n * p, 1);
    synth(hz, (size_t)m * p, 2);
    double* dx = nullptr;
    double* dz = nullptr;
    int32_t* dcount = nullptr;
    if (hipMalloc(&dx, hx.size() * sizeof(double)) != hipSuccess) return TD_ERR_OUT_OF_MEMORY;
    if (hipMalloc(&dz, hz.size() * sizeof(double)) != hipSuccess) { hipFree(dx); return TD_ERR_OUT_OF_MEMORY; }
    if (hipMalloc(&dcount, m * sizeof(int32_t)) != hipSuccess) {
        hipFree(dx);
        hipFree(dz);
        return TD_ERR_OUT_OF_MEMORY;
    }
    td_status ret = TD_OK;
    if (hipMemcpy(dx, hx.data(), hx.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dz, hz.data(), hz.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        ret = TD_ERR_HIP;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    int num_cu = 256;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        DeviceCtx* dctx = nullptr;
        if (ensure_device(dev, &dctx) == TD_OK) num_cu = dctx->num_cu;
    }
    const int tier = class_tier(subset_tier(o), p);
    const int K = kernel_k(tier, p, n, std::max(64, next_pow2((int)n)) / 64);
    float best = 1e30f;
    Shape bs;
    const int chunks[] = {64, 128, 256, 512, 1024};
    const int grids[] = {4, 8, 12, 16};   // resident waves per CU: up to 3 per SIMD
    for (int ci = 0; ci < (int)(sizeof(chunks) / sizeof(chunks[0])) && ret == TD_OK; ++ci)
        for (int gi = 0; gi < 4 && ret == TD_OK; ++gi) {
            td_options t = o;
            t.autotune = 0;
            t.chunk = chunks[ci];
            t.grid_blocks = num_cu * grids[gi];
            t.timing = 0;
            float ms = 0.0f;
            for (int rep = 0; rep < 2; ++rep) {   // the first run warms up
                hipEventRecord(e0, s);
                const td_status r = td_depth_ex(dx, n, p, dz, m, dcount, &t, stream);
                hipEventRecord(e1, s);
                if (r != TD_OK) { ret = r; break; }
                hipEventSynchronize(e1);
                hipEventElapsedTime(&ms, e0, e1);
            }
            if (ret == TD_OK && ms < best) {
                best = ms;
                bs.chunk = t.chunk;
                bs.blocks = t.grid_blocks;
            }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(dx);
    hipFree(dz);
    hipFree(dcount);
    if (ret != TD_OK) return ret;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCtx* dctx = nullptr;
    st = ensure_device(dev, &dctx);
    if (st != TD_OK) return st;
    dctx->tuned[tune_key(tier, p, K)] = bs;
    return TD_OK;
}

td_status td_tuning_save(const char* path) {
    if (!path) return TD_ERR_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TD_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCtx* dc = nullptr;
    td_status st = ensure_device(dev, &dc);
    if (st != TD_OK) return st;
    FILE* f = std::fopen(path, "w");
    if (!f) return TD_ERR_INVALID_ARG;
    bool ok = std::fprintf(f, "td-tuning 1\nnum_cu %d\n", dc->num_cu) > 0;
    for (const auto& kv : dc->tuned) {
        int tier = 0, p = 0, K = 0;
        if (std::sscanf(kv.first.c_str(), "%d:%d:%d", &tier, &p, &K) != 3) continue;
        ok = ok && std::fprintf(f, "%d %d %d %d %d\n", tier, p, K, kv.second.chunk, kv.second.blocks) > 0;
    }
    ok = (std::fclose(f) == 0) && ok;
    return ok ? TD_OK : TD_ERR_INVALID_ARG;
}

td_status td_tuning_load(const char* path) {
    if (!path) return TD_ERR_INVALID_ARG;
    // the file is checked before any device is touched
    FILE* f = std::fopen(path, "r");
    if (!f) return TD_ERR_INVALID_ARG;
    int version = 0, ncu = 0;
    bool ok = std::fscanf(f, " td-tuning %d num_cu %d", &version, &ncu) == 2 && version == 1 && ncu > 0;
    std::vector<std::pair<std::string, Shape>> rows;
    while (ok) {
        int tier = 0, p = 0, K = 0, chunk = 0, blocks = 0;
        const int r = std::fscanf(f, "%d %d %d %d %d", &tier, &p, &K, &chunk, &blocks);
        if (r == EOF) break;
        const bool kok = K == 1 || K == 2 || K == 4 || K == 8 || K == 10 || K == 12 || K == 14 || K == 16;
        ok = r == 5 && (tier == td::kPlain || tier == td::kFilt || tier == td::kFiltBucket) && p >= 2 &&
             p <= TD_MAX_P && kok && chunk >= 64 && chunk <= (1 << 20) && chunk % 64 == 0 && blocks >= 1 &&
             blocks <= (1 << 20);
        if (ok) {
            Shape sh;
            sh.chunk = chunk;
            sh.blocks = blocks;
            rows.emplace_back(tune_key(tier, p, K), sh);
        }
    }
    std::fclose(f);
    if (!ok) return TD_ERR_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TD_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCtx* dc = nullptr;
    td_status st = ensure_device(dev, &dc);
    if (st != TD_OK) return st;
    if (ncu != dc->num_cu) return TD_ERR_UNSUPPORTED;
    for (const auto& r : rows) dc->tuned[r.first] = r.second;
    return TD_OK;
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
        case TD_ERR_TOO_LARGE: return "call needs more than the static workspace of td_depth_noalloc";
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

}  // extern "C"
