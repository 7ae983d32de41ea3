// Instantiations of the subset kernel's float64 pass (bucketed sweep, p >= 3):
// the work items that the first pass handed over at a sweep that needed the
// float64 re-check or re-order.
#include "td_subset.hpp"

namespace {
using namespace td;
typedef void (*KernelFn)(Pools);

template <int P>
KernelFn pick_k(int K) {
    switch (K) {
        case 1: return subset_kernel<P, 1, kFiltBucket, true>;
        case 2: return subset_kernel<P, 2, kFiltBucket, true>;
        case 4: return subset_kernel<P, 4, kFiltBucket, true>;
        case 8: return subset_kernel<P, 8, kFiltBucket, true>;
        case 10:
            if constexpr (P <= 6) return subset_kernel<P, 10, kFiltBucket, true>;
            return nullptr;
        case 12:
            if constexpr (P <= 6) return subset_kernel<P, 12, kFiltBucket, true>;
            return nullptr;
        case 14:
            if constexpr (P <= 6) return subset_kernel<P, 14, kFiltBucket, true>;
            return nullptr;
        case 16: return subset_kernel<P, 16, kFiltBucket, true>;
    }
    return nullptr;
}

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

extern "C" hipError_t td_launch_subset_bucket64(int P, int K, int blocks, hipStream_t s, const td::Pools* pl) {
    KernelFn f = pick(P, K);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(blocks), dim3(64), 0, s, *pl);
    return hipGetLastError();
}
