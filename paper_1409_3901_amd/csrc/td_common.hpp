// Internal layouts shared by the host launcher and the kernels.
#pragma once
#include <stdint.h>

namespace td {

constexpr int kMaxP = 8;
constexpr int kMaxN = 1024;
constexpr int kWave = 64;
constexpr int kBinomK = 8;             // binomial table columns k = 0..7
constexpr int kBinomN = kMaxN + 2;     // rows n = 0..kMaxN+1

// kFiltBucket: the float32-filtered tier with the bucketed sweep.
enum Tier : int { kPlain = 0, kFilt = 1, kExact = 2, kFiltBucket = 3 };

// Query status bits (match TD_DEV_* of td.h).
constexpr int kStNonfinite = 1;
constexpr int kStNoValid = 2;
constexpr int kStDeferOverflow = 4;
constexpr int kStExactRange = 8;
constexpr int kStDegenLimit = 16;
constexpr int kStNotGeneral = 32;       // vertex check: a side not certified
// internal: the exact integer copy of this query is unusable
constexpr int kStNoExactInts = 1 << 8;

// Per-query state written by the preparation kernel and the subset kernels.
struct QueryState {
    int32_t nnz;        // n' = number of observations different from the query
    int32_t n0;         // observations equal to the query
    int32_t status;     // kSt* bits
    int32_t min_term;   // running minimum of delta_I + b_I (atomicMin)
    int32_t ub_term;    // certified upper bound of the minimum from the
                        // directions +-x_j (0x7fffffff when not computed)
};

// Per-query description (one entry per query of every problem in a call).
struct QueryDesc {
    const double* X;    // n x p, device
    const double* z;    // p, device
    int32_t* count;     // output slot, device
    int32_t n, p;
    int32_t M;          // sort width: power of two >= n - (p-2), >= 64
    int32_t idx_bits;   // bits of the point index inside a 32-bit key
    uint64_t v_off;     // offset (values) of this query's x64 / x32 arrays
    uint64_t n_off;     // offset (points) of this query's nrm array
    uint64_t item_begin;// first global work item of this query
    uint32_t items;     // work items of this query
    int32_t cls;        // (p, K) class index for the batched dispatcher
    const int32_t* kmap;// if set, only the (p-2)-subsets of these kcount points
    int32_t kcount;     // (indices into the query's compacted points) are
                        // swept: the candidate points of Algorithm 3, Step 5
    int32_t zero_term;  // 1: the query's minimum is already known to be 0
                        // (Algorithm 3, Step 2(b))
};

// Deferred (uncertain) subset.
struct Deferred {
    uint32_t query;
    uint32_t pad;
    uint64_t rank;
};

// (p, K) classes of one call: p = 2..kMaxP with K = 1, 2, 4, 8, 16 points per
// lane, plus the bucketed sweep's 10, 12 and 14 points per lane at p <= 6.
constexpr int kNumPow2K = 5;
constexpr int kNarrowMaxP = 6;
constexpr int kNumNarrowK = 3;
constexpr int kMaxClasses = (kMaxP - 1) * kNumPow2K + (kNarrowMaxP - 1) * kNumNarrowK;
static_assert(kMaxClasses == 50, "class count");

// Device counters accumulated per call (cleared by the init kernel).
struct Counters {
    unsigned long long swept;
    unsigned long long fp64_rechecks;
    unsigned long long deferred;
    unsigned long long exact_preds;
    unsigned long long degenerate;
    unsigned long long invalid;
    unsigned long long walked;        // bucketed sweeps that needed the exact walk
    unsigned long long pruned;        // subsets of work items skipped once the
                                      // query's minimum had reached 0
    unsigned long long exact_done;    // deferred subsets the exact tier processed
    unsigned long long defer_next;    // deferred-queue write position
    unsigned long long prep_next;     // query counter of the preparation kernel
    unsigned long long work_next[kMaxClasses];   // work-item counter per class
    unsigned long long redo_count[kMaxClasses];  // work items handed to the
                                                 // float64 pass, per class
    unsigned long long redo_next[kMaxClasses];   // its work counter per class
};

// A work item of the bucketed subset kernel left to its float64 pass: the
// subsets of the batch of 64 at colex rank `base` whose bits are set in
// `mask`, and every subset of the item from base + 64 on.
struct RedoItem {
    uint64_t item;
    uint64_t base;
    uint64_t mask;
};

// Per-call parameters in device memory, so that the kernel arguments (and a
// captured graph) do not change from call to call.
struct CallParams {
    int32_t num_queries;
    int32_t num_classes;
    uint64_t cls_begin[kMaxClasses];  // global work items [begin, end) per class
    uint64_t cls_end[kMaxClasses];
    uint64_t cls_scratch[kMaxClasses];// byte offset of the class's block scratch
    uint32_t cls_chunk[kMaxClasses];  // subsets per work item of the class
                                      // (multiple of 64)
};

// Pools of per-query arrays (offsets QueryDesc::v_off in values for the AoS
// arrays, xi at 2 * v_off; QueryDesc::n_off in points for nrm).
struct Pools {
    double* x64;        // centred points, float64, AoS [M][p]
    double* x64lo;      // remainders: x64 + x64lo = X - z exactly (same layout)
    float* x32;         // centred points, float32, AoS [M][p]
    float* nrm;         // upper bound of ||x||_2 per point [M]
    uint64_t* xi;       // exact integers (x - z) * 2^-E, two's complement
                        // 128-bit (lo, hi) pairs, AoS [M][p][2]
    const uint64_t* binom;  // binomial table [kBinomN][kBinomK]
    QueryState* qs;
    const QueryDesc* qd;
    const CallParams* cp;
    Deferred* deferred;
    Counters* ctr;
    uint64_t defer_cap;
    RedoItem* redo;     // work items for the float64 pass (shared by the
    uint64_t redo_cap;  // classes, which run one after the other)
    float filter_scale;
    int32_t force_exact;
    int32_t cls;        // class slot of this launch (subset and exact kernels)
    int32_t sweep_mode; // 0: bucketed sweep kernels, 1: full-sort kernels
    int32_t prune;      // 1: upper bound from the directions +-x_j and skip of
                        // work items once the minimum is 0 (not in the plain tier)
    uint8_t* wscratch;       // per-block scratch in device memory
    uint64_t wscratch_bytes; // bytes per block
};

// Bytes of per-block scratch the subset kernels need for a sort width M.
inline constexpr uint64_t wave_scratch_bytes(int M) {
    // float64 basis slots: 64 x (2*kMaxP + 2) doubles; staging: M x (4+4+1+8+4)
    return (uint64_t)64 * (2 * kMaxP + 2) * 8 + (uint64_t)M * 21 + 256;
}

}  // namespace td
