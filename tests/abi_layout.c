/* Prints the size and every field offset of the structures of include/td.h,
 * compiled by tests/test_abi.py and compared with the ctypes binding. */
#include <stddef.h>
#include <stdio.h>

#include "../include/td.h"

#define F(T, f) printf("%s.%s %zu\n", #T, #f, offsetof(T, f))

int main(void) {
    printf("td_options %zu\n", sizeof(td_options));
    F(td_options, precision); F(td_options, autotune); F(td_options, chunk); F(td_options, grid_blocks);
    F(td_options, filter_scale); F(td_options, force_exact); F(td_options, timing);
    F(td_options, deferred_capacity); F(td_options, sweep); F(td_options, prune);
    F(td_options, method);
    printf("td_stats %zu\n", sizeof(td_stats));
    F(td_stats, subsets_swept); F(td_stats, fp64_rechecks); F(td_stats, deferred_subsets);
    F(td_stats, exact_predicates); F(td_stats, degenerate_subsets); F(td_stats, invalid_subsets);
    F(td_stats, device_status); F(td_stats, prep_ms); F(td_stats, subset_ms); F(td_stats, exact_ms);
    F(td_stats, finalize_ms); F(td_stats, total_ms); F(td_stats, walked_sweeps); F(td_stats, pruned_subsets);
    F(td_stats, exact_subsets); F(td_stats, adia_evaluations); F(td_stats, adia_candidates);
    F(td_stats, f64_items); F(td_stats, adia_rcom_queries);
    printf("td_problem %zu\n", sizeof(td_problem));
    F(td_problem, X); F(td_problem, n); F(td_problem, p); F(td_problem, Z); F(td_problem, m);
    F(td_problem, counts);
    return 0;
}
