// Host check of the kernels' subset enumerator (paper_1409_3901_amd/csrc/
// td_rank.hpp), built and run by tests/test_enumeration.py.  Every (p-2)-
// subset must be visited exactly once: for every rank r < C(n, k) the
// unranked indices are strictly increasing and below n, and their colex rank
// sum_i C(c_i, i+1), computed here from an independent Pascal triangle, is r
// again.  Exhaustive for n <= 30 and k <= 6; sampled ranks for n up to 1024.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_1409_3901_amd/csrc/td_rank.hpp"

static uint64_t pas[td::kBinomN][td::kBinomK + 1];

static uint64_t colex_rank(const int* c, int k) {
    uint64_t r = 0;
    for (int i = 0; i < k; ++i) r += pas[c[i]][i + 1];
    return r;
}

template <int KS>
static bool check_rank(const uint64_t* tab, int n, uint64_t r) {
    int c[KS > 0 ? KS : 1];
    td::unrank_colex<KS>(tab, r, n, c);
    for (int i = 0; i < KS; ++i) {
        if (c[i] < 0 || c[i] >= n || (i > 0 && c[i] <= c[i - 1])) {
            std::printf("FAIL n=%d k=%d r=%llu: invalid index %d at %d\n", n, KS, (unsigned long long)r, c[i], i);
            return false;
        }
    }
    if (colex_rank(c, KS) != r) {
        std::printf("FAIL n=%d k=%d r=%llu: rank back %llu\n", n, KS, (unsigned long long)r,
                    (unsigned long long)colex_rank(c, KS));
        return false;
    }
    return true;
}

template <int KS>
static bool check_k(const uint64_t* tab, uint64_t& visited) {
    for (int n = KS; n <= 30; ++n) {
        const uint64_t total = pas[n][KS];
        for (uint64_t r = 0; r < total; ++r) {
            if (!check_rank<KS>(tab, n, r)) return false;
            ++visited;
        }
    }
    std::mt19937_64 g(1234 + KS);
    for (int n : {31, 100, 257, 512, 640, 768, 896, 1023, 1024}) {
        if (n < KS) continue;
        const uint64_t total = pas[n][KS];
        for (uint64_t j = 0; j < 2000 && j < total; ++j) {
            if (!check_rank<KS>(tab, n, j) || !check_rank<KS>(tab, n, total - 1 - j)) return false;
            visited += 2;
        }
        for (int j = 0; j < 20000; ++j) {
            if (!check_rank<KS>(tab, n, g() % total)) return false;
            ++visited;
        }
    }
    return true;
}

int main() {
    for (int n = 0; n < td::kBinomN; ++n) {
        pas[n][0] = 1;
        for (int k = 1; k <= td::kBinomK; ++k) pas[n][k] = n == 0 ? 0 : pas[n - 1][k - 1] + pas[n - 1][k];
    }
    std::vector<uint64_t> tab((size_t)td::kBinomN * td::kBinomK);
    td::fill_binom_table(tab.data());
    for (int n = 0; n < td::kBinomN; ++n)
        for (int k = 0; k < td::kBinomK; ++k)
            if (tab[(size_t)n * td::kBinomK + k] != pas[n][k]) {
                std::printf("FAIL table C(%d,%d)\n", n, k);
                return 1;
            }
    uint64_t visited = 0;
    bool ok = check_k<1>(tab.data(), visited) && check_k<2>(tab.data(), visited) &&
              check_k<3>(tab.data(), visited) && check_k<4>(tab.data(), visited) &&
              check_k<5>(tab.data(), visited) && check_k<6>(tab.data(), visited);
    if (!ok) return 1;
    std::printf("ok %llu\n", (unsigned long long)visited);
    return 0;
}
