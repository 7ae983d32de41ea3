// Records exchanged between the host's iteration of Algorithm 3 (ADIA,
// Section 4) and its kernels (td_adia.hip).
#pragma once
#include <stdint.h>

#include "td_common.hpp"

namespace td {

// Points next to a minimising state that an evaluation reports (more are
// counted in AdiaRes::tcount but not listed).
constexpr int kAdiaTMax = 32;

// Step 2 of one query: kneg = points strictly below u_min (0: the depth is
// n0), ok = a seed subset was found, idx = the seed subset; best = the
// smallest key count * 2n' + 2j + (sign < 0) of Step 2(a) over the directions
// +-x_j (device side only).
struct AdiaSeed {
    int32_t kneg;
    int32_t ok;
    int32_t idx[kMaxP - 2];
    unsigned long long best;
};

// One (p-2)-subset to evaluate: query and point indices (ascending).
struct AdiaJob {
    int32_t q;
    int32_t idx[kMaxP - 2];
};

// Its value (Algorithm 2, float64; -1: dependent points) and the points of
// the runs next to a minimising state.
struct AdiaRes {
    int32_t term;
    int32_t tcount;
    int32_t t[kAdiaTMax];
};

// A critical (p-1)-set of Step 5(a) (count = p - 1), or a subset whose
// points are simply marked as candidates (count = p - 2).
struct AdiaNode {
    int32_t q;
    int32_t count;
    int32_t idx[kMaxP - 1];
};

}  // namespace td
