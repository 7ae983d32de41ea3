// Dispatch of the exact tier by dimension (instantiations in td_exact_p*.hip).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "td_common.hpp"

#define TD_DECL(P)                                                      \
    extern "C" uint64_t td_exact_scratch_bytes_p##P();                  \
    extern "C" hipError_t td_launch_exact_p##P(int K, int blocks, hipStream_t s, const td::Pools* pl);
TD_DECL(2)
TD_DECL(3)
TD_DECL(4)
TD_DECL(5)
TD_DECL(6)
TD_DECL(7)
TD_DECL(8)

// Bytes of per-block scratch the exact tier needs for dimension p.
extern "C" uint64_t td_exact_scratch_bytes(int P) {
    switch (P) {
        case 2: return td_exact_scratch_bytes_p2();
        case 3: return td_exact_scratch_bytes_p3();
        case 4: return td_exact_scratch_bytes_p4();
        case 5: return td_exact_scratch_bytes_p5();
        case 6: return td_exact_scratch_bytes_p6();
        case 7: return td_exact_scratch_bytes_p7();
        case 8: return td_exact_scratch_bytes_p8();
    }
    return 0;
}

extern "C" hipError_t td_launch_exact(int P, int K, int blocks, hipStream_t s, const td::Pools* pl, int all_items) {
    if (all_items) return hipErrorNotSupported;
    switch (P) {
        case 2: return td_launch_exact_p2(K, blocks, s, pl);
        case 3: return td_launch_exact_p3(K, blocks, s, pl);
        case 4: return td_launch_exact_p4(K, blocks, s, pl);
        case 5: return td_launch_exact_p5(K, blocks, s, pl);
        case 6: return td_launch_exact_p6(K, blocks, s, pl);
        case 7: return td_launch_exact_p7(K, blocks, s, pl);
        case 8: return td_launch_exact_p8(K, blocks, s, pl);
    }
    return hipErrorInvalidValue;
}
