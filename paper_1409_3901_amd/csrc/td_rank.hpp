// Subset ranks: the binomial table and the colexicographic unranking that
// the kernels use to walk the index set of (p-2)-subsets (Section 2; the loop
// of Algorithm 1, Step 1).  Host and device code share these functions: the
// host fills the table, the kernels unrank, and a host check can run the
// same unranking on every rank of small sets.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "td_common.hpp"

namespace td {

// C(n, k), saturated at UINT64_MAX (host).
inline uint64_t binom_host(int64_t n, int k) {
    if (k < 0 || n < k) return 0;
    unsigned __int128 r = 1;
    for (int i = 1; i <= k; ++i) r = r * (unsigned __int128)(n - k + i) / (unsigned __int128)i;
    if (r > (unsigned __int128)UINT64_MAX) return UINT64_MAX;
    return (uint64_t)r;
}

// tab[n * kBinomK + k] = C(n, k) for n < kBinomN, k < kBinomK.
inline void fill_binom_table(uint64_t* tab) {
    for (int n = 0; n < kBinomN; ++n)
        for (int k = 0; k < kBinomK; ++k) tab[(size_t)n * kBinomK + k] = binom_host(n, k);
}

__host__ __device__ __forceinline__ uint64_t binom_lookup(const uint64_t* tab, int n, int k) {
    if (k < 0 || n < k) return 0;
    return tab[n * kBinomK + k];
}

// Colexicographic unranking of k-subsets: rank = sum_i C(c_i, i+1) with
// c_0 < c_1 < ... < c_{k-1}.  The map does not depend on the ground-set size,
// so ranks below C(n', k) give subsets of {0..n'-1}.
template <int KS>
__host__ __device__ __forceinline__ void unrank_colex(const uint64_t* tab, uint64_t r, int nmax,
                                                      int (&c)[KS > 0 ? KS : 1]) {
    int hi = nmax;  // exclusive upper bound for the current element
#pragma unroll
    for (int i = KS; i >= 1; --i) {
        // largest x in [i-1, hi-1] with C(x, i) <= r
        int lo = i - 1, h = hi - 1;
        while (lo < h) {
            int mid = (lo + h + 1) >> 1;
            if (binom_lookup(tab, mid, i) <= r) lo = mid; else h = mid - 1;
        }
        c[i - 1] = lo;
        r -= binom_lookup(tab, lo, i);
        hi = lo;
    }
}

}  // namespace td
