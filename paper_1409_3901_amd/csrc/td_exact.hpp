// Exact tier: subsets whose float32/float64 decisions could not be certified.
//
// One wave per deferred subset.  The lanes project every point in float64
// with a rigorous error bound and sort 64-bit keys; points whose fold or
// angle float64 cannot settle get their exact Pluecker coordinates
//     phi(x) = (det[x_I | x | e_j], det[x_I | x | e_k])
// from the exact integer copy of the data (a point with phi(x) = 0 lies inside
// span(x_I)).  Lane 0 then walks the sorted sequence: runs of overlapping key
// intervals that hold both fold signs are re-ordered with the exact
// orientation sign(cross(phi_a, phi_b)) and exactly equal angles are grouped
// (Algorithm 2, Step 1(e)).  If extra points lie inside span(x_I), their depth
// delta_I inside that span is added: the fewest points to drop so that the
// rest lie in an open halfspace, found as a minimum hitting set of the
// positive circuits (minimal subsets with a positive linear dependency).
#pragma once
#include <hip/hip_runtime.h>

#include "td_bigint.hpp"
#include "td_subset.hpp"

namespace td {

template <int P>
struct XS {
    static constexpr int KS = P - 2;
    static constexpr int NG = (125 * (KS > 0 ? KS : 1) + 48) / 32 + 2;  // minors
    static constexpr int NF = (125 * (KS + 1) + 56) / 32 + 2;           // phi
    static constexpr int NC = 2 * NF;                                   // cross
};

constexpr int kExactClusterMax = 64;

// Lower end of a key interval [q - rq, q + rq], clamped at 0.  Keys are sorted
// by lower end, so that a lower end above every earlier upper end (lower end
// + 2 rq) is a strict gap of the exact order, whatever the radii.
__device__ __forceinline__ uint64_t lower_end64(uint64_t q, uint32_t rq) { return q > rq ? q - rq : 0ull; }
constexpr int kDeltaMax = 16;       // |K_I| handled by the hitting-set search
constexpr int kCircuitMax = 128;

// Exact determinant of an s x s matrix of 128-bit integers (row-major pairs
// lo, hi) by the permutation expansion (Heap's algorithm, sign tracked).
template <int NG>
__device__ void det_i128(const uint64_t* ent, int s, BigI<NG>& out) {
    big_zero(out);
    if (s == 0) { big_from_int(out, 1); return; }
    int perm[8], cnt[8];
    for (int i = 0; i < s; ++i) { perm[i] = i; cnt[i] = 0; }
    int sign = 1;
    auto add_term = [&]() {
        BigI<NG> t;
        big_from_i128(t, ent[(0 * s + perm[0]) * 2], ent[(0 * s + perm[0]) * 2 + 1]);
        for (int r = 1; r < s; ++r) {
            BigI<NG> u;
            BigI<4> x;
            const uint64_t lo = ent[(r * s + perm[r]) * 2], hi = ent[(r * s + perm[r]) * 2 + 1];
            x.w[0] = (uint32_t)lo;
            x.w[1] = (uint32_t)(lo >> 32);
            x.w[2] = (uint32_t)hi;
            x.w[3] = (uint32_t)(hi >> 32);
            big_mul<NG, NG, 4>(u, t, x);
            t = u;
        }
        if (sign < 0) big_neg(t);
        big_add(out, t);
    };
    add_term();
    int i = 1;
    while (i < s) {
        if (cnt[i] < i) {
            const int j = (i & 1) ? cnt[i] : 0;
            const int tmp = perm[j];
            perm[j] = perm[i];
            perm[i] = tmp;
            sign = -sign;
            add_term();
            ++cnt[i];
            i = 1;
        } else {
            cnt[i] = 0;
            ++i;
        }
    }
}

// int128 of point idx, coordinate c (query pool)
__device__ __forceinline__ void xi_at(const uint64_t* xi, int P, int idx, int c, uint64_t& lo, uint64_t& hi) {
    lo = xi[((size_t)idx * P + c) * 2];
    hi = xi[((size_t)idx * P + c) * 2 + 1];
}

// Complementary minor of the subset matrix (rows a, b deleted), exactly.
template <int P>
__device__ void minor_exact(const uint64_t* xi, const int* mem, int a, int b, BigI<XS<P>::NG>& out) {
    constexpr int KS = P - 2;
    uint64_t ent[(KS > 0 ? KS : 1) * (KS > 0 ? KS : 1) * 2];
    int r = 0;
    for (int row = 0; row < P; ++row) {
        if (row == a || row == b) continue;
        for (int c = 0; c < KS; ++c) {
            uint64_t lo, hi;
            xi_at(xi, P, mem[c], row, lo, hi);
            ent[(r * KS + c) * 2] = lo;
            ent[(r * KS + c) * 2 + 1] = hi;
        }
        ++r;
    }
    det_i128<XS<P>::NG>(ent, KS, out);
}

// Exact Pluecker rows: G1_i = det[A | e_i | e_j], G2_i = det[A | e_i | e_k].
template <int P>
__device__ void exact_rows(const uint64_t* xi, const int* mem, int j, int k, BigI<XS<P>::NG>* G1,
                           BigI<XS<P>::NG>* G2) {
    for (int i = 0; i < P; ++i) {
        if (i == j) {
            big_zero(G1[i]);
        } else {
            minor_exact<P>(xi, mem, i, j, G1[i]);
            const int i1 = i - (i > j ? 1 : 0);
            if ((j + i1 + 1) & 1) big_neg(G1[i]);
        }
        if (i == k) {
            big_zero(G2[i]);
        } else {
            minor_exact<P>(xi, mem, i, k, G2[i]);
            const int i2 = i - (i > k ? 1 : 0);
            if ((k + i2 + 1) & 1) big_neg(G2[i]);
        }
    }
}

// phi(x) = (G1 . x, G2 . x) exactly
template <int P>
__device__ void exact_phi(const uint64_t* xi, int idx, const BigI<XS<P>::NG>* G1, const BigI<XS<P>::NG>* G2,
                          BigI<XS<P>::NF>& f1, BigI<XS<P>::NF>& f2) {
    constexpr int NG = XS<P>::NG, NF = XS<P>::NF;
    big_zero(f1);
    big_zero(f2);
    for (int c = 0; c < P; ++c) {
        uint64_t lo, hi;
        xi_at(xi, P, idx, c, lo, hi);
        BigI<4> x;
        x.w[0] = (uint32_t)lo;
        x.w[1] = (uint32_t)(lo >> 32);
        x.w[2] = (uint32_t)hi;
        x.w[3] = (uint32_t)(hi >> 32);
        BigI<NF> g, t;
        // widen G to NF words (sign extension)
        const uint32_t e1 = ((int32_t)G1[c].w[NG - 1] < 0) ? 0xffffffffu : 0u;
        for (int w = 0; w < NF; ++w) g.w[w] = (w < NG) ? G1[c].w[w] : e1;
        big_mul<NF, NF, 4>(t, g, x);
        big_add(f1, t);
        const uint32_t e2 = ((int32_t)G2[c].w[NG - 1] < 0) ? 0xffffffffu : 0u;
        for (int w = 0; w < NF; ++w) g.w[w] = (w < NG) ? G2[c].w[w] : e2;
        big_mul<NF, NF, 4>(t, g, x);
        big_add(f2, t);
    }
}

// sign(a1 b2 - a2 b1) for folded exact coordinates
template <int P>
__device__ int exact_orient(const BigI<XS<P>::NF>& a1, const BigI<XS<P>::NF>& a2, const BigI<XS<P>::NF>& b1,
                            const BigI<XS<P>::NF>& b2) {
    constexpr int NF = XS<P>::NF, NC = XS<P>::NC;
    BigI<NC> u, v;
    big_mul<NC, NF, NF>(u, a1, b2);
    big_mul<NC, NF, NF>(v, a2, b1);
    big_sub(u, v);
    return big_sign(u);
}

// Is the column set T (bitmask over the points kidx[]) a positive circuit?
template <int P>
__device__ bool positive_circuit(const uint64_t* xi, const int* kidx, uint32_t T) {
    constexpr int NG = XS<P>::NG, NF = XS<P>::NF;
    int cols[kDeltaMax];
    int t = 0;
    for (int i = 0; i < kDeltaMax; ++i)
        if ((T >> i) & 1u) cols[t++] = kidx[i];
    if (t < 2 || t > P) return false;
    const int s = t - 1;
    int rows[8];
    for (int i = 0; i < s; ++i) rows[i] = i;
    while (true) {
        BigI<NG> lam[8];
        bool anynz = false;
        for (int i = 0; i < t; ++i) {
            uint64_t ent[7 * 7 * 2];
            for (int r = 0; r < s; ++r) {
                int cc = 0;
                for (int c = 0; c < t; ++c) {
                    if (c == i) continue;
                    uint64_t lo, hi;
                    xi_at(xi, P, cols[c], rows[r], lo, hi);
                    ent[(r * s + cc) * 2] = lo;
                    ent[(r * s + cc) * 2 + 1] = hi;
                    ++cc;
                }
            }
            det_i128<NG>(ent, s, lam[i]);
            if (i & 1) big_neg(lam[i]);
            if (!big_is_zero(lam[i])) anynz = true;
        }
        if (anynz) {
            // lam spans the kernel of the selected rows; a dependency of all
            // rows iff sum lam_i x_i = 0 everywhere
            for (int row = 0; row < P; ++row) {
                BigI<NF> acc;
                big_zero(acc);
                for (int i = 0; i < t; ++i) {
                    BigI<NF> g;
                    const uint32_t e = ((int32_t)lam[i].w[NG - 1] < 0) ? 0xffffffffu : 0u;
                    for (int w = 0; w < NF; ++w) g.w[w] = (w < NG) ? lam[i].w[w] : e;
                    uint64_t lo, hi;
                    xi_at(xi, P, cols[i], row, lo, hi);
                    big_fma_i128<NF>(acc, g, lo, hi, 1);
                }
                if (!big_is_zero(acc)) return false;   // independent columns
            }
            const int s0 = big_sign(lam[0]);
            if (s0 == 0) return false;
            for (int i = 1; i < t; ++i)
                if (big_sign(lam[i]) != s0) return false;
            return true;
        }
        // next row combination
        int i = s - 1;
        while (i >= 0 && rows[i] == P - s + i) --i;
        if (i < 0) return false;   // rank below t-1: not minimal
        ++rows[i];
        for (int j = i + 1; j < s; ++j) rows[j] = rows[j - 1] + 1;
    }
}

// delta_I: fewest points of K to remove so that the rest lies in an open
// halfspace (Gordan), i.e. a minimum hitting set of the positive circuits.
template <int P>
__device__ int delta_hitting(const uint64_t* xi, const int* kidx, int nk, int nfree, int& status,
                             unsigned long long& preds) {
    // kidx[0 .. nfree-1] are the subset's own points (independent), the rest
    // are the extra points inside its span; every circuit holds an extra point
    uint32_t circ[kCircuitMax];
    int nc = 0;
    const uint32_t all = (nk >= 32) ? 0xffffffffu : ((1u << nk) - 1u);
    const uint32_t extra = all & ~((1u << nfree) - 1u);
    for (uint32_t T = 1; T <= all && T != 0; ++T) {
        if (!(T & extra)) continue;
        const int pc = __popc(T);
        if (pc < 2 || pc > P - 1) continue;
        // only minimal sets matter: skip T containing a known circuit
        bool sup = false;
        for (int c = 0; c < nc; ++c)
            if ((circ[c] & T) == circ[c]) { sup = true; break; }
        if (sup) continue;
        ++preds;
        if (positive_circuit<P>(xi, kidx, T)) {
            if (nc == kCircuitMax) { status |= kStDegenLimit; return 0; }
            circ[nc++] = T;
        }
    }
    // smallest R hitting every circuit (nk <= 16, so `all` < 2^16)
    for (int r = 0; r <= nk; ++r)
        for (uint32_t R = 0; R <= all; ++R) {
            if (__popc(R) != r) continue;
            bool hit = true;
            for (int c = 0; c < nc; ++c)
                if (!(circ[c] & R)) { hit = false; break; }
            if (hit) return r;
        }
    return nk;
}

template <int P>
struct ExactScratch {
    BigI<XS<P>::NG> G1[P], G2[P];
    BigI<XS<P>::NF> H1[kExactClusterMax], H2[kExactClusterMax];
    int hidx[kExactClusterMax];
    int hsig[kExactClusterMax];
};

// Two waves per SIMD: the kernel is latency-bound (big-integer predicates,
// one lane's walks), and a second wave hides it (c5, 2.3 million deferred
// subsets: 347 -> 235 ms; four waves per SIMD gain little more and slow the
// single subsets of small calls).
template <int P, int K>
__global__ __launch_bounds__(64, 2) void exact_kernel(Pools pl) {
    constexpr int KS = P - 2;
    constexpr int M = 64 * K;
    constexpr int NF = XS<P>::NF;
    __shared__ uint64_t skey[M];
    __shared__ uint32_t sside[M];
    __shared__ int s_extra[kDeltaMax];
    __shared__ int s_nextra;
    __shared__ int s_flag;
    const int lane = lane_id();
    ExactScratch<P>* X = reinterpret_cast<ExactScratch<P>*>(pl.wscratch + pl.cp->cls_scratch[pl.cls] +
                                                            (uint64_t)blockIdx.x * pl.wscratch_bytes);
    unsigned long long taken = 0, preds = 0, degen = 0, ninvalid = 0;
    const unsigned long long nd = pl.ctr->defer_next;
    const unsigned long long total = nd < pl.defer_cap ? nd : pl.defer_cap;
    // Static striding over the deferred list: every class launch scans the
    // whole list and takes the entries of its own class (the class index:
    // classes of one sort width M differ in points per lane).
    unsigned long long it = blockIdx.x;
    constexpr double qscale = 4503599627370496.0;     // 2^52: t' in [0,2] -> 53 bits
    constexpr uint64_t qmax = (1ull << 54) - 2ull;
    constexpr uint32_t kWide = 0x3fffffffu;
    for (; it < total; it += gridDim.x) {
        const Deferred dfr = pl.deferred[it];
        const int q = uni((int)dfr.query);
        const QueryDesc d = pl.qd[q];
        const QueryState st = pl.qs[q];
        if (d.cls != pl.cls) continue;   // belongs to another class
        ++taken;
        const int nnz = uni(st.nnz);
        const double* x64 = pl.x64 + d.v_off;
        const float* nrm = pl.nrm + d.n_off;
        const uint64_t* xi = pl.xi + d.v_off * 2;
        int mem[KS > 0 ? KS : 1];
        mem[0] = 0;
        unrank_colex<KS>(pl.binom, dfr.rank, d.kmap ? d.kcount : nnz, mem);
        if (d.kmap) {
#pragma unroll
            for (int c = 0; c < KS; ++c) mem[c] = d.kmap[mem[c]];
        }
#pragma unroll
        for (int c = 0; c < KS; ++c) mem[c] = uni(mem[c]);
        double A[P][KS > 0 ? KS : 1];
#pragma unroll
        for (int col = 0; col < KS; ++col)
#pragma unroll
            for (int r = 0; r < P; ++r) A[r][col] = x64[(size_t)mem[col] * P + r];
        Basis<P> Bs;
        build_basis<P>(A, Bs);
        if (!Bs.certified || Bs.eta > 0x1p-30) refine_basis_dd<P>(x64, pl.x64lo + d.v_off, mem, Bs);
        const bool ints_ok = !(st.status & kStNoExactInts);
        bool have_rows = false;
        if (!Bs.certified) {
            // decide the rank of the subset exactly and rebuild the basis from
            // the exact Pluecker rows of the largest nonzero minor
            if (!ints_ok) {
                if (lane == 0) atomicOr(&pl.qs[q].status, kStExactRange);
                continue;
            }
            if (lane == 0) {
                double bestv = 0.0;
                int bj = -1, bk = -1;
                for (int a = 0; a < P; ++a)
                    for (int b = a + 1; b < P; ++b) {
                        BigI<XS<P>::NG> mnr;
                        minor_exact<P>(xi, mem, a, b, mnr);
                        ++preds;
                        const double v = fabs(big_to_double(mnr));
                        if (v > bestv) { bestv = v; bj = a; bk = b; }
                    }
                s_flag = (bj < 0) ? -1 : bj * 8 + bk;
                if (bj >= 0) exact_rows<P>(xi, mem, bj, bk, X->G1, X->G2);
            }
            __syncthreads();
            const int fl = uni(s_flag);
            if (fl < 0) { ++ninvalid; __syncthreads(); continue; }
            double g1[P], g2[P], E1[P], E2[P];
            for (int i = 0; i < P; ++i) {
                g1[i] = big_to_double(X->G1[i]);
                g2[i] = big_to_double(X->G2[i]);
                E1[i] = 4.0 * kU64 * fabs(g1[i]);
                E2[i] = 4.0 * kU64 * fabs(g2[i]);
            }
            finish_basis<P>(g1, g2, E1, E2, Bs);
            Bs.j = fl >> 3;
            Bs.k = fl & 7;
            have_rows = true;
            __syncthreads();
        }
        const double beta64 = (((double)P + 3.0) * kU64 + Bs.eta) * 1.01;
        const double s1 = Bs.s1, s2 = Bs.s2, cs1 = Bs.c * Bs.s1;
        // ---- float64 keys
        uint64_t key[K];
        uint32_t weak = 0;
        int nplus = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int idx = lane * K + i;
            bool valid = idx < nnz;
#pragma unroll
            for (int c = 0; c < KS; ++c) valid = valid && (idx != mem[c]);
            key[i] = ~0ull;
            if (!valid) continue;
            double y1, y2, t, r;
            bool pos;
            fp64_point<P>(x64, Bs.e1, Bs.e2, idx, y1, y2);
            const double eps = beta64 * (double)nrm[idx];
            if (key64(y1, y2, eps, pos, t, r) && r * qscale < (double)kWide) {
                const uint64_t qv = min((uint64_t)(t * qscale), qmax);
                const uint32_t rq = (uint32_t)(r * qscale) + 3u;
                key[i] = (lower_end64(qv, rq) << 10) | (uint64_t)idx;
                sside[idx] = rq | (pos ? 0u : 0x80000000u);
                nplus += pos ? 1 : 0;
            } else {
                weak |= 1u << i;
            }
        }
        // ---- lower bound from the points float64 places.  Every other point
        // only adds to the counts and delta_I >= 0, so when the smallest state
        // the certified points allow (runs of overlapping intervals in any
        // inner order) is not below a term the query already reached, the
        // subset cannot lower the minimum: no exact work is done for it.
        const int qbest = uni(__hip_atomic_load(&pl.qs[q].min_term, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (qbest < 0x7fffffff) {
            uint64_t kb[K];
#pragma unroll
            for (int i = 0; i < K; ++i) kb[i] = key[i];
            wave_sort<K>(kb);
#pragma unroll
            for (int i = 0; i < K; ++i) skey[lane * K + i] = kb[i];
            int mc = 0;
#pragma unroll
            for (int i = 0; i < K; ++i) mc += (key[i] != ~0ull) ? 1 : 0;
            const int mcert = wave_sum(mc);
            const int S0c = wave_sum(nplus);
            __syncthreads();
            int lb = 0;
            if (lane == 0) {
                int S = S0c;
                lb = fside(S0c, mcert);
                int i = 0;
#pragma unroll 1
                while (i < mcert) {
                    const uint64_t k0 = skey[i];
                    const uint32_t sd0 = sside[k0 & 1023u];
                    int64_t mhi = (int64_t)(k0 >> 10) + 2 * (int64_t)(sd0 & 0x7fffffffu);
                    int np = (sd0 >> 31) ? 0 : 1;
                    int j = i;
                    while (j + 1 < mcert) {
                        const uint64_t kk = skey[j + 1];
                        const uint32_t sd = sside[kk & 1023u];
                        if ((int64_t)(kk >> 10) > mhi) break;
                        mhi = max(mhi, (int64_t)(kk >> 10) + 2 * (int64_t)(sd & 0x7fffffffu));
                        np += (sd >> 31) ? 0 : 1;
                        ++j;
                    }
                    const int c = j - i + 1;
                    lb = min(lb, min(S - np, mcert - (S + (c - np))));
                    S += c - 2 * np;
                    lb = min(lb, fside(S, mcert));
                    i = j + 1;
                }
            }
            lb = __builtin_amdgcn_readfirstlane(lb);
            __syncthreads();
            if (lb >= qbest) continue;
        }
        if (lane == 0) { s_nextra = 0; s_flag = 0; }
        if (__any(weak != 0)) {
            if (!ints_ok) {
                if (lane == 0) atomicOr(&pl.qs[q].status, kStExactRange);
                __syncthreads();
                continue;
            }
            if (!have_rows) {
                if (lane == 0) exact_rows<P>(xi, mem, Bs.j, Bs.k, X->G1, X->G2);
                have_rows = true;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < K; ++i) {
                if (!((weak >> i) & 1u)) continue;
                const int idx = lane * K + i;
                BigI<NF> f1, f2;
                exact_phi<P>(xi, idx, X->G1, X->G2, f1, f2);
                ++preds;
                const int sg1 = big_sign(f1), sg2 = big_sign(f2);
                if (sg1 == 0 && sg2 == 0) {
                    // inside span(x_I)
                    const int slot = atomicAdd(&s_nextra, 1);
                    if (slot < kDeltaMax - KS) s_extra[slot] = idx;
                    continue;
                }
                const int sig = (sg1 != 0) ? sg1 : sg2;
                // key in the float64 frame L = T phi from the exact phi
                const double p1 = big_to_double(f1), p2 = big_to_double(f2);
                const double a1 = s1 * p1;
                const double a2 = s2 * fma(-cs1, p1, p2);
                const double e = (4.0 * kU64 + 1.0e-15) * (fabs(a1) + s2 * (fabs(p2) + fabs(cs1 * p1))) * 1.01;
                const double h1 = sig * a1, h2 = sig * a2;
                const double sabs = h1 + fabs(h2);
                uint64_t qv = 0;
                uint32_t rq = 0;
                const double t = h2 / sabs + 1.0;
                const double r = e / (sabs - 2.0 * e) * 1.001 + 4.0 * kU64;
                if (sabs > 4.0 * e && r * qscale < (double)kWide) {
                    qv = min((uint64_t)(t * qscale), qmax);
                    rq = (uint32_t)(r * qscale) + 3u;
                } else {
                    // the float64 frame cannot place it: refuse rather than guess
                    atomicOr(&s_flag, 1);
                }
                key[i] = (lower_end64(qv, rq) << 10) | (uint64_t)idx;
                sside[idx] = rq | (sig > 0 ? 0u : 0x80000000u);
                nplus += sig > 0 ? 1 : 0;
            }
        }
        __syncthreads();
        const int nextra = uni(s_nextra);
        if (uni(s_flag) != 0) {
            if (lane == 0) atomicOr(&pl.qs[q].status, kStDegenLimit);
            __syncthreads();
            continue;
        }
        // more points inside span(x_I) than the hitting-set search takes:
        // b_I is still computed; delta_I is needed only if b_I alone is below
        // the query's running minimum (otherwise the subset cannot lower it)
        const bool delta_over = nextra > kDeltaMax - KS;
        wave_sort<K>(key);
#pragma unroll
        for (int i = 0; i < K; ++i) skey[lane * K + i] = key[i];
        const int S0 = wave_sum(nplus);
        __syncthreads();
        // ---- serial walk on lane 0
        int term = 0;
        int status = 0;
        if (lane == 0) {
            const int m = nnz - KS - nextra;
            int S = S0;
            int best = fside(S0, m);
            int i = 0;
            while (i < m) {
                const uint64_t k0 = skey[i];
                const uint32_t sd0 = sside[k0 & 1023u];
                const int64_t q0 = (int64_t)(k0 >> 10);
                int64_t mhi = q0 + 2 * (int64_t)(sd0 & 0x7fffffffu);
                const int d0 = (sd0 >> 31) ? 1 : -1;
                bool mixed = false;
                int j = i;
                while (j + 1 < m) {
                    const uint64_t kk = skey[j + 1];
                    const uint32_t sd = sside[kk & 1023u];
                    const int64_t qq = (int64_t)(kk >> 10);   // lower end
                    const int64_t rr = (int64_t)(sd & 0x7fffffffu);
                    if (qq > mhi) break;
                    mhi = max(mhi, qq + 2 * rr);
                    if (((sd >> 31) ? 1 : -1) != d0) mixed = true;
                    ++j;
                }
                const int c = j - i + 1;
                if (!mixed) {
                    S += c * d0;
                    best = min(best, fside(S, m));
                } else if (c > kExactClusterMax || !ints_ok) {
                    status |= ints_ok ? kStDegenLimit : kStExactRange;
                    break;
                } else {
                    if (!have_rows) {
                        exact_rows<P>(xi, mem, Bs.j, Bs.k, X->G1, X->G2);
                        have_rows = true;
                    }
                    // exact folded coordinates, insertion-sorted by angle
                    for (int u = 0; u < c; ++u) {
                        const uint64_t kk = skey[i + u];
                        const int idx = (int)(kk & 1023u);
                        const int sig = (sside[idx] >> 31) ? -1 : 1;
                        BigI<NF> f1, f2;
                        exact_phi<P>(xi, idx, X->G1, X->G2, f1, f2);
                        if (sig < 0) { big_neg(f1); big_neg(f2); }
                        int w = u;
                        while (w > 0) {
                            ++preds;
                            if (exact_orient<P>(X->H1[w - 1], X->H2[w - 1], f1, f2) >= 0) break;
                            X->H1[w] = X->H1[w - 1];
                            X->H2[w] = X->H2[w - 1];
                            X->hsig[w] = X->hsig[w - 1];
                            --w;
                        }
                        X->H1[w] = f1;
                        X->H2[w] = f2;
                        X->hsig[w] = sig;
                    }
                    for (int u = 0; u < c; ++u) {
                        S += -X->hsig[u];
                        bool tie = false;
                        if (u + 1 < c) {
                            ++preds;
                            tie = exact_orient<P>(X->H1[u], X->H2[u], X->H1[u + 1], X->H2[u + 1]) == 0;
                        }
                        if (!tie) best = min(best, fside(S, m));
                    }
                }
                i = j + 1;
            }
            term = best;
            // delta_I >= 0: when b_I alone is not below the query's running
            // minimum the subset cannot lower it, and delta_I is not computed
            const int qb = __hip_atomic_load(&pl.qs[q].min_term, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (nextra > 0 && !status && term >= qb) {
                term = 0x7fffffff;
            } else if (delta_over && !status) {
                status |= kStDegenLimit;
            } else if (nextra > 0 && !status) {
                int kidx[kDeltaMax];
                for (int c2 = 0; c2 < KS; ++c2) kidx[c2] = mem[c2];
                for (int e2 = 0; e2 < nextra; ++e2) kidx[KS + e2] = s_extra[e2];
                term += delta_hitting<P>(xi, kidx, KS + nextra, KS, status, preds);
                ++degen;
            }
            if (status) atomicOr(&pl.qs[q].status, status);
            else atomicMin(&pl.qs[q].min_term, term);
        }
        __syncthreads();
    }
    if (lane == 0) {
        if (taken) atomicAdd(&pl.ctr->exact_done, taken);
        if (preds) atomicAdd(&pl.ctr->exact_preds, preds);
        if (degen) atomicAdd(&pl.ctr->degenerate, degen);
        if (ninvalid) atomicAdd(&pl.ctr->invalid, ninvalid);
    }
}

}  // namespace td

