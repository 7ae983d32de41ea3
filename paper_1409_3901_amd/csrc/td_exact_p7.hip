// Exact-tier instantiations for p = 7.
#include "td_exact.hpp"

extern "C" uint64_t td_exact_scratch_bytes_p7() { return sizeof(td::ExactScratch<7>); }

extern "C" hipError_t td_launch_exact_p7(int K, int blocks, hipStream_t s, const td::Pools* pl) {
    void (*f)(td::Pools) = nullptr;
    switch (K) {
        case 1: f = td::exact_kernel<7, 1>; break;
        case 2: f = td::exact_kernel<7, 2>; break;
        case 4: f = td::exact_kernel<7, 4>; break;
        case 8: f = td::exact_kernel<7, 8>; break;
        case 16: f = td::exact_kernel<7, 16>; break;
    }
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(blocks), dim3(64), 0, s, *pl);
    return hipGetLastError();
}
