// Exact-tier instantiations for p = 6.
#include "td_exact.hpp"

extern "C" uint64_t td_exact_scratch_bytes_p6() { return sizeof(td::ExactScratch<6>); }

extern "C" hipError_t td_launch_exact_p6(int K, int blocks, hipStream_t s, const td::Pools* pl) {
    void (*f)(td::Pools) = nullptr;
    switch (K) {
        case 1: f = td::exact_kernel<6, 1>; break;
        case 2: f = td::exact_kernel<6, 2>; break;
        case 4: f = td::exact_kernel<6, 4>; break;
        case 8: f = td::exact_kernel<6, 8>; break;
        case 16: f = td::exact_kernel<6, 16>; break;
    }
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(blocks), dim3(64), 0, s, *pl);
    return hipGetLastError();
}
