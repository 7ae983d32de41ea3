// Instantiations of the subset kernel: float32-filtered tier, bucketed sweep.
#include "td_subset.hpp"

namespace {
using namespace td;
typedef void (*KernelFn)(Pools);

template <int P>
KernelFn pick_k(int K) {
    switch (K) {
        case 1: return subset_kernel<P, 1, kFiltBucket>;
        case 2: return subset_kernel<P, 2, kFiltBucket>;
        case 4: return subset_kernel<P, 4, kFiltBucket>;
        case 8: return subset_kernel<P, 8, kFiltBucket>;
        // samples of 512 < n <= 896 in steps of 128 (the sweep needs no
        // power-of-two width)
        case 10:
            if constexpr (P <= 6) return subset_kernel<P, 10, kFiltBucket>;
            return nullptr;
        case 12:
            if constexpr (P <= 6) return subset_kernel<P, 12, kFiltBucket>;
            return nullptr;
        case 14:
            if constexpr (P <= 6) return subset_kernel<P, 14, kFiltBucket>;
            return nullptr;
        case 16: return subset_kernel<P, 16, kFiltBucket>;
    }
    return nullptr;
}

// p >= 3: p = 2 runs the full-sort kernel
KernelFn pick(int P, int K) {
    switch (P) {
        case 3: return pick_k<3>(K);
        case 4: return pick_k<4>(K);
        case 5: return pick_k<5>(K);
        case 6: return pick_k<6>(K);
        case 7: return pick_k<7>(K);
        case 8: return pick_k<8>(K);
    }
    return nullptr;
}
}  // namespace

// Blocks of the (P, K) kernel that one compute unit holds at once (0 when
// the shape has no kernel or the query fails).
extern "C" int td_resident_blocks_bucket(int P, int K) {
    KernelFn f = pick(P, K);
    int n = 0;
    if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64, 0) != hipSuccess) return 0;
    return n;
}

extern "C" hipError_t td_launch_subset_bucket(int P, int K, int blocks, hipStream_t s, const td::Pools* pl) {
    KernelFn f = pick(P, K);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(blocks), dim3(64), 0, s, *pl);
    return hipGetLastError();
}
