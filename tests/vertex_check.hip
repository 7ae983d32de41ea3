// Host check of the vertex-form arithmetic the kernel uses (td_vertex.hpp),
// run on the CPU by tests/test_vertex_host.py:
//   vertex_check self        exact checks; prints "ok <decisions>"
//   vertex_check count FILE  vertex counts of the problem in FILE ("n p m",
//                            then X and Z row by row); prints one count per
//                            query, -1 where a side is not certified
// Exact mode: integer matrices (and integers scaled by powers of two, which
// float64 holds exactly) against cofactors and determinants in 128-bit
// integers; the certified side must equal the exact sign, and points built
// on the hyperplane must come out undecided.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../paper_1409_3901_amd/csrc/td_vertex.hpp"

using i128 = __int128;

template <int P>
static void exact_cofactors(const long long (&A)[P][P > 1 ? P - 1 : 1], i128 (&u)[P]) {
    // Laplace expansion of each (P-1)x(P-1) minor, recursively, in 128 bits
    for (int k = 0; k < P; ++k) {
        int rows[P], nr = 0;
        for (int r = 0; r < P; ++r)
            if (r != k) rows[nr++] = r;
        // permutation expansion over the P-1 rows (P <= 8: at most 5040 terms)
        int perm[P];
        for (int i = 0; i < nr; ++i) perm[i] = i;
        i128 det = 0;
        // Heap-free: iterate permutations in lexicographic order
        while (true) {
            int inv = 0;
            for (int i = 0; i < nr; ++i)
                for (int j = i + 1; j < nr; ++j) inv += perm[i] > perm[j];
            i128 t = 1;
            for (int c = 0; c < nr; ++c) t *= (i128)A[rows[perm[c]]][c];
            det += (inv & 1) ? -t : t;
            int i = nr - 2;
            while (i >= 0 && perm[i] > perm[i + 1]) --i;
            if (i < 0) break;
            int j = nr - 1;
            while (perm[j] < perm[i]) --j;
            int tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
            for (int a = i + 1, b = nr - 1; a < b; ++a, --b) { tmp = perm[a]; perm[a] = perm[b]; perm[b] = tmp; }
        }
        u[k] = (k & 1) ? -det : det;
    }
}

static long long fails = 0, decisions = 0;

template <int P>
static void self_check(std::mt19937_64& rng, int trials, int range, int shift) {
    std::uniform_int_distribution<long long> U(-range, range);
    const double scale = std::ldexp(1.0, -shift);
    for (int t = 0; t < trials; ++t) {
        long long Ai[P][P > 1 ? P - 1 : 1];
        double A[P][P > 1 ? P - 1 : 1];
        for (int r = 0; r < P; ++r)
            for (int c = 0; c < P - 1; ++c) {
                Ai[r][c] = U(rng);
                A[r][c] = (double)Ai[r][c] * scale;
            }
        i128 ue[P];
        exact_cofactors<P>(Ai, ue);
        double u[P], b[P];
        td::vertex_cofactors<P>(A, u, b);
        // cofactor error within gamma_2P of the permanent (scaled by 2^-shift(P-1))
        const double cs = std::ldexp(1.0, -shift * (P - 1));
        for (int k = 0; k < P; ++k) {
            const double ex = (double)ue[k] * cs;   // exact up to one rounding
            const double tol = td::vertex_gamma(2 * P) * b[k] + std::fabs(ex) * 0x1p-52;
            if (std::fabs(u[k] - ex) > tol) {
                std::printf("cofactor P=%d k=%d got %.17g want %.17g tol %.3g\n", P, k, u[k], ex, tol);
                ++fails;
            }
        }
        // points: random, and on the hyperplane (integer combinations of A's columns)
        for (int j = 0; j < 16; ++j) {
            long long xi[P];
            if (j < 8) {
                for (int r = 0; r < P; ++r) xi[r] = U(rng);
            } else {
                long long w[P > 1 ? P - 1 : 1];
                for (int c = 0; c < P - 1; ++c) w[c] = U(rng) % 4;
                for (int r = 0; r < P; ++r) {
                    xi[r] = 0;
                    for (int c = 0; c < P - 1; ++c) xi[r] += w[c] * Ai[r][c];
                }
            }
            i128 s = 0;
            for (int r = 0; r < P; ++r) s += (i128)xi[r] * ue[r];
            const int es = s > 0 ? 1 : (s < 0 ? -1 : 0);
            double x[P];
            for (int r = 0; r < P; ++r) x[r] = (double)xi[r] * scale;
            const int side = td::vertex_side<P>(x, u, b);
            if (side != 0) {
                ++decisions;
                if (side != es) {
                    std::printf("side P=%d got %d exact %d\n", P, side, es);
                    ++fails;
                }
            } else if (es != 0 && j < 8 && range > 4) {
                // undecided although off the plane: allowed, but should be rare
            }
            if (es == 0 && side != 0) {
                std::printf("point on the plane decided P=%d\n", P);
                ++fails;
            }
        }
    }
}

template <int P>
static int vertex_count(const std::vector<double>& x, int nnz, bool& undecided) {
    // every (P-1)-subset of the nnz centred points, in lexicographic order
    int c[P > 1 ? P - 1 : 1];
    const int ks = P - 1;
    for (int i = 0; i < ks; ++i) c[i] = i;
    int best = 1 << 30;
    if (nnz < ks) return -1;
    while (true) {
        double A[P][P > 1 ? P - 1 : 1];
        for (int col = 0; col < ks; ++col)
            for (int r = 0; r < P; ++r) A[r][col] = x[(size_t)c[col] * P + r];
        double u[P], b[P];
        td::vertex_cofactors<P>(A, u, b);
        int np = 0, nn = 0;
        for (int i = 0; i < nnz; ++i) {
            bool mem = false;
            for (int col = 0; col < ks; ++col) mem = mem || c[col] == i;
            if (mem) continue;
            double xi[P];
            for (int r = 0; r < P; ++r) xi[r] = x[(size_t)i * P + r];
            const int s = td::vertex_side<P>(xi, u, b);
            np += s > 0;
            nn += s < 0;
            undecided = undecided || s == 0;
        }
        best = std::min(best, std::min(np, nn));
        int i = ks - 1;
        while (i >= 0 && c[i] == nnz - ks + i) --i;
        if (i < 0) break;
        ++c[i];
        for (int j = i + 1; j < ks; ++j) c[j] = c[j - 1] + 1;
    }
    return best;
}

template <int P>
static void count_file(FILE* f, int n, int m) {
    std::vector<double> X((size_t)n * P), Z((size_t)m * P);
    for (auto& v : X) if (std::fscanf(f, "%lf", &v) != 1) std::exit(2);
    for (auto& v : Z) if (std::fscanf(f, "%lf", &v) != 1) std::exit(2);
    for (int q = 0; q < m; ++q) {
        std::vector<double> x;
        int n0 = 0;
        for (int i = 0; i < n; ++i) {
            bool eq = true;
            double row[P];
            for (int r = 0; r < P; ++r) {
                row[r] = X[(size_t)i * P + r] - Z[(size_t)q * P + r];
                eq = eq && X[(size_t)i * P + r] == Z[(size_t)q * P + r];
            }
            if (eq) { ++n0; continue; }
            for (int r = 0; r < P; ++r) x.push_back(row[r]);
        }
        bool und = false;
        const int v = vertex_count<P>(x, (int)(x.size() / P), und);
        std::printf("%d\n", (und || v < 0) ? -1 : n0 + v);
    }
}

int main(int argc, char** argv) {
    if (argc >= 2 && std::strcmp(argv[1], "self") == 0) {
        std::mt19937_64 rng(20260);
        for (int shift : {0, 30}) {
            self_check<2>(rng, 400, 1 << 20, shift);
            self_check<3>(rng, 400, 1 << 16, shift);
            self_check<4>(rng, 300, 1 << 12, shift);
            self_check<5>(rng, 300, 1 << 9, shift);
            self_check<6>(rng, 200, 1 << 7, shift);
            self_check<7>(rng, 60, 1 << 6, shift);
            self_check<8>(rng, 20, 1 << 5, shift);
            // small ranges: many points on or near the planes
            self_check<3>(rng, 400, 3, shift);
            self_check<5>(rng, 200, 2, shift);
        }
        if (fails) { std::printf("FAILED %lld\n", fails); return 1; }
        std::printf("ok %lld\n", decisions);
        return 0;
    }
    if (argc >= 3 && std::strcmp(argv[1], "count") == 0) {
        FILE* f = std::fopen(argv[2], "r");
        if (!f) return 2;
        int n, p, m;
        if (std::fscanf(f, "%d %d %d", &n, &p, &m) != 3) return 2;
        switch (p) {
            case 2: count_file<2>(f, n, m); break;
            case 3: count_file<3>(f, n, m); break;
            case 4: count_file<4>(f, n, m); break;
            case 5: count_file<5>(f, n, m); break;
            case 6: count_file<6>(f, n, m); break;
            default: return 2;
        }
        std::fclose(f);
        return 0;
    }
    return 2;
}
