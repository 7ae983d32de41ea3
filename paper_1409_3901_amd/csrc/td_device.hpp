// Device building blocks of the subset kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "td_common.hpp"
#include "td_rank.hpp"

namespace td {

constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53
constexpr float kU32 = 5.9604645e-08f;            // 2^-24

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Values known to be equal on every lane, moved to scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ float unif(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Which query a global work item belongs to (binary search on item_begin).
__device__ __forceinline__ int item_query(const QueryDesc* qd, int nq, uint64_t item) {
    int lo = 0, hi = nq - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (qd[mid].item_begin <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------ wave helpers
template <typename T>
__device__ __forceinline__ T shfl_xor_t(T v, int mask) {
    return __shfl_xor(v, mask, 64);
}

// Wave-wide scans with DPP: row shifts 1, 2, 4, 8 inside each 16-lane row,
// then row broadcasts of lane 15 (to rows 1 and 3) and lane 31 (to rows 2
// and 3).  Lanes without a source read the identity.  Every helper below
// expects the whole wave to be active.
__device__ __forceinline__ int wave_incl_sum_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);
    return v;
}

__device__ __forceinline__ int wave_incl_min_dpp(int v) {
    constexpr int I = 0x7fffffff;
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x111, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x112, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x114, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x118, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x142, 0xA, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x143, 0xC, 0xF, false));
    return v;
}

__device__ __forceinline__ int wave_incl_max_dpp(int v) {
    constexpr int I = (int)0x80000000;
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x111, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x112, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x114, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x118, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x142, 0xA, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x143, 0xC, 0xF, false));
    return v;
}

// Totals (uniform: read from lane 63).
__device__ __forceinline__ int wave_sum(int v) { return __builtin_amdgcn_readlane(wave_incl_sum_dpp(v), 63); }
__device__ __forceinline__ int wave_min(int v) { return __builtin_amdgcn_readlane(wave_incl_min_dpp(v), 63); }
__device__ __forceinline__ int wave_max(int v) { return __builtin_amdgcn_readlane(wave_incl_max_dpp(v), 63); }
__device__ __forceinline__ int wave_min_dpp(int v) { return wave_min(v); }

// exclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_excl_sum(int v) { return wave_incl_sum_dpp(v) - v; }

// exclusive prefix max over the 64 lanes (identity `id` for lane 0): the
// inclusive scan moved up one lane (DPP wave_shr:1)
__device__ __forceinline__ int wave_excl_max(int v, int id) {
    return __builtin_amdgcn_update_dpp(id, wave_incl_max_dpp(v), 0x138, 0xF, 0xF, false);
}


// Value of the previous lane (DPP wave_shr:1; lane 0 reads `id`) and of the
// next lane (wave_shl:1; lane 63 reads `id`).
__device__ __forceinline__ int lane_prev(int v, int id) {
    return __builtin_amdgcn_update_dpp(id, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ int lane_next(int v, int id) {
    return __builtin_amdgcn_update_dpp(id, v, 0x130, 0xF, 0xF, false);
}

// ------------------------------------------------------------ bitonic sort
// Value of lane (lane ^ MASK) for the lane patterns of the bitonic network,
// using DPP lane moves and the gfx950 permlane swaps where they exist:
//   ^1, ^2, ^3      quad_perm
//   ^7, ^15         row_half_mirror, row_mirror
//   ^8              row_ror:8 (rotation by half a 16-lane row)
//   ^4              row_shl:4 / row_shr:4 and a select on lane bit 2
//   ^16, ^32        v_permlane16_swap / v_permlane32_swap
//   ^31, ^63        compositions of the above
template <int MASK>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
    if constexpr (MASK == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
    } else if constexpr (MASK == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
    } else if constexpr (MASK == 3) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x1B, 0xF, 0xF, false);
    } else if constexpr (MASK == 7) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);
    } else if constexpr (MASK == 15) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);
    } else if constexpr (MASK == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);
    } else if constexpr (MASK == 4) {
        const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x104, 0xF, 0xF, false);
        const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x114, 0xF, 0xF, false);
        return (lane_id() & 4) ? dn : up;
    } else if constexpr (MASK == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane_id() & 16) ? r[0] : r[1];
    } else if constexpr (MASK == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane_id() & 32) ? r[0] : r[1];
    } else if constexpr (MASK == 31) {
        return lane_xor<16>(lane_xor<15>(v));
    } else if constexpr (MASK == 63) {
        return lane_xor<32>(lane_xor<31>(v));
    } else {
        return (uint32_t)__shfl_xor((int)v, MASK, 64);
    }
}

template <int MASK>
__device__ __forceinline__ uint64_t lane_xor64(uint64_t v) {
    const uint32_t lo = lane_xor<MASK>((uint32_t)v);
    const uint32_t hi = lane_xor<MASK>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <int MASK, typename T>
__device__ __forceinline__ T lane_xor_t(T v) {
    if constexpr (sizeof(T) == 8) return (T)lane_xor64<MASK>((uint64_t)v);
    else return (T)lane_xor<MASK>((uint32_t)v);
}

// Ascending sort of M = 64*K keys held blocked: element e = lane*K + i lives
// in register i of lane `lane`.  The flip form of the bitonic network is used
// (first stage of every merge compares e with e ^ (size-1)), so every
// compare-exchange puts the minimum at the lower position.
template <typename T>
__device__ __forceinline__ void ce(T& a, T& b) {
    T lo = a < b ? a : b;
    T hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// Median of three unsigned words.  With c = 0 it is min(a, b), with c = ~0 it
// is max(a, b): one instruction for a cross-lane compare-exchange whose
// direction depends on the lane.
__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

template <typename T>
__device__ __forceinline__ T cx_pick(T a, T b, bool lower) {
    if constexpr (sizeof(T) == 4) {
        return (T)med3u((uint32_t)a, (uint32_t)b, lower ? 0u : 0xffffffffu);
    } else {
        T lo = a < b ? a : b, hi = a < b ? b : a;
        return lower ? lo : hi;
    }
}

template <int K, int SIZE, typename T>
__device__ __forceinline__ void flip_stage(T (&v)[K], int lane) {
    if constexpr (SIZE <= K) {
#pragma unroll
        for (int b = 0; b < K; b += SIZE)
#pragma unroll
            for (int i = 0; i < SIZE / 2; ++i) ce(v[b + i], v[b + SIZE - 1 - i]);
    } else {
        constexpr int LM = SIZE / K - 1;
        const bool lower = (lane & (SIZE / (2 * K))) == 0;
        T w[K];
#pragma unroll
        for (int i = 0; i < K; ++i) w[i] = lane_xor_t<LM>(v[K - 1 - i]);
#pragma unroll
        for (int i = 0; i < K; ++i) v[i] = cx_pick(v[i], w[i], lower);
    }
}

template <int K, int D, typename T>
__device__ __forceinline__ void half_stage(T (&v)[K], int lane) {
    if constexpr (D < K) {
#pragma unroll
        for (int i = 0; i < K; ++i)
            if ((i & D) == 0) ce(v[i], v[i | D]);
    } else {
        constexpr int LM = D / K;
        const bool lower = (lane & LM) == 0;
        if constexpr (sizeof(T) == 4 && (LM == 16 || LM == 32)) {
            // The swap hands every lane (own, partner) or (partner, own);
            // the median with 0 / ~0 picks min / max either way.
            const uint32_t sel = lower ? 0u : 0xffffffffu;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const uint32_t x = (uint32_t)v[i];
                if constexpr (LM == 16) {
                    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
                    v[i] = (T)med3u(r[0], r[1], sel);
                } else {
                    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
                    v[i] = (T)med3u(r[0], r[1], sel);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < K; ++i) v[i] = cx_pick(v[i], lane_xor_t<LM>(v[i]), lower);
        }
    }
}

template <int K, int D, typename T>
__device__ __forceinline__ void half_chain(T (&v)[K], int lane) {
    if constexpr (D >= 1) {
        half_stage<K, D>(v, lane);
        half_chain<K, D / 2>(v, lane);
    }
}

template <int K, int SIZE, typename T>
__device__ __forceinline__ void sort_phases(T (&v)[K], int lane) {
    if constexpr (SIZE <= 64 * K) {
        flip_stage<K, SIZE>(v, lane);
        half_chain<K, SIZE / 4>(v, lane);
        sort_phases<K, SIZE * 2>(v, lane);
    }
}

template <int K, typename T>
__device__ __forceinline__ void wave_sort(T (&v)[K]) {
    sort_phases<K, 2>(v, lane_id());
}

// Binomial table and colex unranking: td_rank.hpp.

// -------------------------------------------- minors of the p x (p-2) block
// Combination tables (rows of a p-row matrix) for the Laplace recursion that
// computes every c x c minor of the first c columns from the (c-1) x (c-1)
// minors.  Level c lists the c-subsets of rows in increasing mask order.
template <int P>
struct ComboTab {
    int cnt[P + 1];
    uint8_t mask[P + 1][70];
    uint8_t rows[P + 1][70][8];
    uint8_t child[P + 1][70][8];
};

constexpr int pc8(int m) {
    int c = 0;
    for (int b = 0; b < 8; ++b) c += (m >> b) & 1;
    return c;
}

template <int P>
constexpr ComboTab<P> make_combo_tab() {
    ComboTab<P> T{};
    for (int c = 0; c <= P; ++c) {
        int t = 0;
        for (int m = 0; m < (1 << P); ++m) {
            if (pc8(m) != c) continue;
            T.mask[c][t] = (uint8_t)m;
            int r = 0;
            for (int b = 0; b < P; ++b)
                if ((m >> b) & 1) T.rows[c][t][r++] = (uint8_t)b;
            ++t;
        }
        T.cnt[c] = t;
    }
    for (int c = 1; c <= P; ++c)
        for (int t = 0; t < T.cnt[c]; ++t)
            for (int pos = 0; pos < c; ++pos) {
                int m2 = T.mask[c][t] ^ (1 << T.rows[c][t][pos]);
                for (int u = 0; u < T.cnt[c - 1]; ++u)
                    if (T.mask[c - 1][u] == m2) T.child[c][t][pos] = (uint8_t)u;
            }
    return T;
}

// Index of the level-(P-2) combination that leaves out rows a and b.
template <int P>
constexpr int pair_combo(int a, int b) {
    constexpr ComboTab<P> T = make_combo_tab<P>();
    int m = ((1 << P) - 1) ^ (1 << a) ^ (1 << b);
    for (int u = 0; u < T.cnt[P - 2]; ++u)
        if (T.mask[P - 2][u] == m) return u;
    return -1;
}

template <int P>
struct MinorSet {
    // value of every (p-2)-minor, indexed by the combination of P-2 rows
    double v[70];
};

// All (p-2) x (p-2) minors of A (p rows, p-2 columns; A[r][c]) by the Laplace
// recursion along the last column.
template <int P>
__device__ __forceinline__ void all_minors(const double (&A)[P][P > 2 ? P - 2 : 1], MinorSet<P>& out) {
    constexpr int KC = P - 2;
    constexpr ComboTab<P> T = make_combo_tab<P>();
    double pv[70];
    if (KC == 0) {
        out.v[0] = 1.0;
        return;
    }
#pragma unroll
    for (int t = 0; t < T.cnt[1]; ++t) pv[t] = A[T.rows[1][t][0]][0];
#pragma unroll
    for (int c = 2; c <= KC; ++c) {
        double cv[70];
#pragma unroll
        for (int t = 0; t < T.cnt[c]; ++t) {
            double v = 0.0;
#pragma unroll
            for (int pos = 0; pos < c; ++pos) {
                const double x = A[T.rows[c][t][pos]][c - 1];
                v = fma(((pos + c - 1) & 1) ? -x : x, pv[T.child[c][t][pos]], v);
            }
            cv[t] = v;
        }
#pragma unroll
        for (int t = 0; t < T.cnt[c]; ++t) pv[t] = cv[t];
    }
#pragma unroll
    for (int t = 0; t < T.cnt[KC]; ++t) out.v[t] = pv[t];
}

// Rounding bound of every minor: the sum over the expansion of the absolute
// monomials is at most the product of the column 1-norms, and every monomial
// passes through at most k input roundings plus c roundings at level c.
template <int P>
constexpr double minor_gamma() {
    constexpr int k = P - 2;
    constexpr int N = k + k * (k + 1) / 2 + 3;
    return (double)N * kU64 * 1.0001;
}

// ------------------------------------------------------ complement basis
// Orthonormal basis (e1, e2) of the orthogonal complement of span(x_I), the
// first step of Algorithm 1.  Construction: for the row pair (j,k) with the
// largest certified minor omega = det[x_I | e_j | e_k], the vectors
//     g1_i = det[x_I | e_i | e_j],   g2_i = det[x_I | e_i | e_k]
// are exactly orthogonal to span(x_I) and span its complement; e1, e2 are
// their Gram-Schmidt orthonormalisation.  The exact linear maps
//     L1 = s1 g1,   L2 = s2 (g2 - c s1 g1)
// (s1, s2, c the float64 coefficients actually used) form the exact frame the
// float computations approximate: L = T phi with phi(x) = (g1.x, g2.x) and
// T lower triangular with positive diagonal, so orientations and the fold
// half-plane {L1 x > 0} U {L1 x = 0, L2 x > 0} are those of phi.
// `eta` bounds ||e_k - L_k||_1 for both k (input rounding included).
template <int P>
struct Basis {
    double e1[P], e2[P];
    double s1, s2, c;
    double eta;
    int j, k;
    int certified;   // 1: some minor is certified nonzero (the subset is valid)
    int anynz;       // 1: the largest float64 minor is nonzero
};

// Gram-Schmidt of the Pluecker rows g1, g2 (absolute errors E1, E2 against
// the exact rows) into e1, e2, with the frame coefficients and eta.
template <int P>
__device__ __forceinline__ void finish_basis(const double (&g1)[P], const double (&g2)[P], const double (&E1)[P],
                                             const double (&E2)[P], Basis<P>& B) {
    double n1 = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) n1 = fma(g1[i], g1[i], n1);
    const double s1 = (n1 > 0.0) ? 1.0 / sqrt(n1) : 0.0;
    double cc = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        B.e1[i] = g1[i] * s1;
        cc = fma(B.e1[i], g2[i], cc);
    }
    double n2 = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        B.e2[i] = fma(-cc, B.e1[i], g2[i]);
        n2 = fma(B.e2[i], B.e2[i], n2);
    }
    const double s2 = (n2 > 0.0) ? 1.0 / sqrt(n2) : 0.0;
    // eta >= ||e_k - L_k||_1: per component
    //   e1: s1*E1 + u|e1|,   e2: u|e2| + s2*(1.01u|v| + E2 + |c| eps1)
    double eta1 = 0.0, eta2 = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const double vi = B.e2[i];
        B.e2[i] = vi * s2;
        const double ep1 = s1 * E1[i] + kU64 * fabs(B.e1[i]);
        eta1 += ep1;
        eta2 += kU64 * fabs(B.e2[i]) + s2 * (1.01 * kU64 * fabs(vi) + E2[i] + fabs(cc) * ep1);
    }
    B.s1 = s1;
    B.s2 = s2;
    B.c = cc;
    B.eta = fmax(eta1, eta2) * 1.001;
}

template <int P>
__device__ __forceinline__ void build_basis(const double (&A)[P][P > 2 ? P - 2 : 1], Basis<P>& B) {
    MinorSet<P> ms;
    all_minors<P>(A, ms);
    // bound on the rounding error of every minor
    double colprod = 1.0;
#pragma unroll
    for (int c = 0; c < P - 2; ++c) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < P; ++r) s += fabs(A[r][c]);
        colprod *= s;
    }
    const double emin = minor_gamma<P>() * colprod * 1.0001;
    // pivot pair: largest |minor|; certified when it exceeds the bound
    double best = -1.0;
    int bj = 0, bk = 1;
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = a + 1; b < P; ++b) {
            const double v = fabs(ms.v[pair_combo<P>(a, b)]);
            if (v > best) { best = v; bj = a; bk = b; }
        }
    B.certified = best > emin;
    B.anynz = best > 0.0;
    B.j = bj;
    B.k = bk;
    double g1[P], g2[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        // det[A | e_i | e_j] = (-1)^(j + i' + 1) M_{ij},  i' = i - [i > j]
        double v1 = 0.0, v2 = 0.0;
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
            for (int b = a + 1; b < P; ++b) {
                const double mv = ms.v[pair_combo<P>(a, b)];
                if ((a == i && b == bj) || (b == i && a == bj)) v1 = mv;
                if ((a == i && b == bk) || (b == i && a == bk)) v2 = mv;
            }
        const int i1 = i - (i > bj ? 1 : 0);
        const int i2 = i - (i > bk ? 1 : 0);
        g1[i] = (i == bj) ? 0.0 : ((((bj + i1 + 1) & 1) ? -v1 : v1));
        g2[i] = (i == bk) ? 0.0 : ((((bk + i2 + 1) & 1) ? -v2 : v2));
    }
    double E1[P], E2[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        E1[i] = (i == bj) ? 0.0 : emin;
        E2[i] = (i == bk) ? 0.0 : emin;
    }
    finish_basis<P>(g1, g2, E1, E2, B);
}

// ------------------------------------ double-double refinement of the basis
// When the float64 minors cancel badly (strongly anisotropic data), the frame
// error eta is too large for the filters to decide anything.  The minors are
// then recomputed in double-double arithmetic from the exact centred values
// x = hi + lo (prep stores the remainder of the float64 subtraction), with an
// absolute error below gamma_dd * prod of the column 1-norms.
struct DD {
    double hi, lo;
};

// Error-free transformations need every operation rounded on its own:
// floating-point contraction (a*b + c fused into one FMA) is switched off in
// these helpers, where the compiler would otherwise fuse the product of
// dd_mul into the sum that follows it.
// Knuth's TwoSum (The Art of Computer Programming, vol. 2, 4.2.2): s + err =
// a + b exactly, in six operations and without a branch on the magnitudes.
__device__ __forceinline__ DD dd_two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double z = s - a;
    return DD{s, (a - (s - z)) + (b - z)};
}

// (ah + al) * (x.hi + x.lo): the leading product made exact by the FMA-based
// TwoProduct (p = fl(ah x.hi), e = fma(ah, x.hi, -p); Ogita, Rump and Oishi,
// 2005), cross terms rounded, al * x.lo dropped; absolute error
// <= 5 u^2 |a| |x|
__device__ __forceinline__ DD dd_mul(double ah, double al, DD x) {
#pragma clang fp contract(off)
    const double p = ah * x.hi;
    const double e = fma(ah, x.hi, -p);
    const double t = fma(ah, x.lo, fma(al, x.hi, e));
    return dd_two_sum(p, t);
}

// absolute error <= 6 u^2 (|x| + |y|)
__device__ __forceinline__ DD dd_add(DD x, DD y) {
#pragma clang fp contract(off)
    const DD s = dd_two_sum(x.hi, y.hi);
    return dd_two_sum(s.hi, s.lo + x.lo + y.lo);
}

// Bound factor of a k x k minor by the Laplace recursion in double-double:
// level c adds at most (5 + 6c) u^2 times the column-norm product.
template <int KS>
constexpr double dd_gamma() {
    double g = 0.0;
    for (int c = 2; c <= KS; ++c) g += 5.0 + 6.0 * c;
    return (g + 8.0) * kU64 * kU64 * 1.01;
}

// The (p-2)-minor of the subset matrix with rows ra and rb left out, in
// double-double: Laplace recursion along the columns, one column of entries
// (float64 value and remainder) loaded per level.
template <int P>
__device__ __forceinline__ DD dd_minor(const double* x64, const double* x64lo, const int* cc, int ra, int rb) {
    constexpr int KS = P - 2;
    constexpr ComboTab<KS> T = make_combo_tab<KS>();
    const int r0 = min(ra, rb), r1 = max(ra, rb);
    DD pv[10];
#pragma unroll
    for (int r = 0; r < KS; ++r) {
        const int row = r < r0 ? r : (r + 1 < r1 ? r + 1 : r + 2);
        pv[r] = DD{x64[(size_t)cc[0] * P + row], x64lo[(size_t)cc[0] * P + row]};
    }
#pragma unroll
    for (int c = 2; c <= KS; ++c) {
        double ch[KS], cl[KS];
#pragma unroll
        for (int r = 0; r < KS; ++r) {
            const int row = r < r0 ? r : (r + 1 < r1 ? r + 1 : r + 2);
            ch[r] = x64[(size_t)cc[c - 1] * P + row];
            cl[r] = x64lo[(size_t)cc[c - 1] * P + row];
        }
        DD cv[10];
#pragma unroll
        for (int t = 0; t < T.cnt[c]; ++t) {
            DD v = DD{0.0, 0.0};
#pragma unroll
            for (int pos = 0; pos < c; ++pos) {
                const int row = T.rows[c][t][pos];
                DD term = dd_mul(ch[row], cl[row], pv[T.child[c][t][pos]]);
                if ((pos + c - 1) & 1) term = DD{-term.hi, -term.lo};
                v = dd_add(v, term);
            }
            cv[t] = v;
        }
#pragma unroll
        for (int t = 0; t < T.cnt[c]; ++t) pv[t] = cv[t];
    }
    return pv[0];
}

// Recompute the Pluecker rows of the pivot pair (j, k) chosen by the float64
// pass in double-double and rebuild the basis; per-entry errors are the
// double-double bound plus the dropped low word.  Supported for p <= 6.
template <int P>
__device__ __noinline__ void refine_basis_dd(const double* x64, const double* x64lo, const int* cc, Basis<P>& B) {
    constexpr int KS = P - 2;
    if constexpr (KS < 1 || KS > 4) {
        return;
    } else {
        double colprod = 1.0;
#pragma unroll
        for (int c = 0; c < KS; ++c) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < P; ++r)
                s += fabs(x64[(size_t)cc[c] * P + r]) + fabs(x64lo[(size_t)cc[c] * P + r]);
            colprod *= s * (1.0 + 4.0 * P * kU64);
        }
        const double emin = dd_gamma<KS>() * colprod;
        const int bj = B.j, bk = B.k;
        double g1[P], g2[P], E1[P], E2[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            g1[i] = 0.0;
            E1[i] = 0.0;
            g2[i] = 0.0;
            E2[i] = 0.0;
        }
        double om = 0.0, om_err = 0.0;
        // one rolled loop over the 2p minors (the row index is uniform, so
        // the register arrays are indexed without memory)
#pragma unroll 1
        for (int u = 0; u < 2 * P; ++u) {
            const int i = u >> 1;
            const int piv = (u & 1) ? bk : bj;
            if (i == piv) continue;
            const DD m = dd_minor<P>(x64, x64lo, cc, i, piv);
            const int ii = i - (i > piv ? 1 : 0);
            const double g = ((piv + ii + 1) & 1) ? -m.hi : m.hi;
            const double e = emin + fabs(m.lo);
            if (u & 1) {
                g2[i] = g;
                E2[i] = e;
            } else {
                g1[i] = g;
                E1[i] = e;
                if (i == bk) {
                    om = fabs(m.hi);
                    om_err = e;
                }
            }
        }
        B.certified = om > om_err;
        B.anynz = om > 0.0;
        finish_basis<P>(g1, g2, E1, E2, B);
    }
}

// ------------------------------------------------------- exact 128-bit input
__device__ __forceinline__ int low_exp(double v) {
    // exponent of the lowest set bit of a finite nonzero double
    uint64_t b = (uint64_t)__double_as_longlong(v);
    int ex = (int)((b >> 52) & 0x7ff);
    uint64_t man = b & 0xfffffffffffffull;
    if (ex == 0) {  // subnormal
        return -1074 + __builtin_ctzll(man);
    }
    man |= (1ull << 52);
    return ex - 1075 + __builtin_ctzll(man);
}

__device__ __forceinline__ int high_exp(double v) {
    // exponent of the highest set bit of a finite nonzero double
    uint64_t b = (uint64_t)__double_as_longlong(v);
    int ex = (int)((b >> 52) & 0x7ff);
    uint64_t man = b & 0xfffffffffffffull;
    if (ex == 0) return -1074 + 63 - __builtin_clzll(man);
    return ex - 1023;
}

// v * 2^-E as a two's-complement 128-bit integer (lo, hi); requires v to be a
// multiple of 2^E and |v| * 2^-E < 2^126.
__device__ __forceinline__ void to_i128(double v, int E, uint64_t& lo, uint64_t& hi) {
    lo = 0;
    hi = 0;
    if (v == 0.0) return;
    uint64_t b = (uint64_t)__double_as_longlong(v);
    int ex = (int)((b >> 52) & 0x7ff);
    uint64_t man = b & 0xfffffffffffffull;
    int e2;
    if (ex == 0) { e2 = -1074; } else { man |= (1ull << 52); e2 = ex - 1075; }
    int sh = e2 - E;   // >= 0 by the choice of E... may be negative for low bits that are zero
    while (sh < 0) { man >>= 1; ++sh; }
    if (sh >= 128) { lo = 0; hi = 0; }
    else if (sh >= 64) { hi = man << (sh - 64); lo = 0; }
    else if (sh == 0) { lo = man; hi = 0; }
    else { lo = man << sh; hi = man >> (64 - sh); }
    if (b >> 63) {  // negate
        lo = ~lo;
        hi = ~hi;
        lo += 1;
        if (lo == 0) hi += 1;
    }
}

}  // namespace td
