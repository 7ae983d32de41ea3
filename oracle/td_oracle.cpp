/*
 * Exact CPU oracle for the sample Tukey depth count  n * D_n(z).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code with the HIP path.
 *
 * What it computes (Section 1, sample depth, equation (1)): for observations
 * X_1..X_n in R^p and a query z,
 *     d(z) = min over unit u of #{ i : u'(X_i - z) <= 0 },
 * the depth count (closed halfspaces).  The paper's first algorithm
 * (Section 3, Algorithm 1 with Algorithm 2 as its bivariate step, justified by
 * Proposition 1 with r = p-2, equation (8)) is followed step by step:
 *
 *   shift to z = 0 (Section 2), drop the observations equal to z (they lie on
 *   every hyperplane and count n0 for every u);
 *   for every (p-2)-subset I of the rest (Algorithm 1, Step 1):
 *     (a) a basis of the 2-D complement of span(x_I),
 *     (b) the bivariate depth of the projected points by one angular sort and
 *         one circular sweep (Algorithm 2),
 *     (c) keep the minimum;
 *   return n0 + minimum (the count form of Algorithm 1, Step 2).
 *
 * Readings taken where the paper assumes general position (it suggests a
 * perturbation instead; here the exact count of the given doubles is the
 * target, so no perturbation is applied):
 *   - the complement coordinates are the exact Pluecker coordinates
 *       phi(x) = (det[x_I | x | e_j], det[x_I | x | e_k])
 *     for a row pair (j,k) with det[x_I | e_j | e_k] != 0; they are an
 *     invertible linear image of the orthonormal coordinates of Algorithm 1
 *     Step 1(a)-(b), so the sweep result is the same;
 *   - points with phi(x) = 0 are the points inside span(x_I) (Algorithm 2,
 *     Step 1(a) drops them); instead of the literal correction (p-2), the
 *     depth delta_I of 0 among those points inside span(x_I) is added, which
 *     equals 0 whenever span(x_I) holds only the subset itself;
 *   - points are folded into the half-plane {h1 > 0} U {h1 = 0, h2 > 0}
 *     instead of using theta = -y1/y2, which is undefined for y2 = 0
 *     (Algorithm 2, Step 1(b)-(c));
 *   - the running count is compared only at the end of each run of exactly
 *     equal angles (Algorithm 2, Step 1(e));
 *   - subsets whose points are linearly dependent have no 2-D complement and
 *     are skipped; if the centred data span fewer than p dimensions they are
 *     first mapped injectively into their span.
 *
 * Arithmetic: each predicate (a sign of an integer determinant) is first
 * evaluated in float64 together with a rigorous bound on its rounding error
 * (the sum of absolute values of the same expression times gamma_N, N the
 * number of roundings on any path, input rounding included); when the bound
 * does not settle the sign, it is recomputed exactly with arbitrary-precision
 * integers from the exactly integerised inputs (every finite double is an
 * integer multiple of 2^E for the smallest exponent E present).
 * With ORACLE_EXACT_ONLY every predicate is computed exactly.
 */
#include <algorithm>
#include <cmath>
#include <deque>
#include <map>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ------------------------------------------------------------ big integers
struct Big {
    int sgn = 0;                 // -1, 0, +1
    std::vector<uint32_t> mag;   // little-endian magnitude, no leading zeros

    static Big from_u64(uint64_t v, int s = 1) {
        Big b;
        if (v == 0) return b;
        b.sgn = s;
        b.mag.push_back((uint32_t)v);
        if (v >> 32) b.mag.push_back((uint32_t)(v >> 32));
        return b;
    }
    static Big from_i64(int64_t v) {
        if (v < 0) return from_u64((uint64_t)(-(v + 1)) + 1u, -1);
        return from_u64((uint64_t)v, 1);
    }
    bool zero() const { return sgn == 0; }
};

void trim(std::vector<uint32_t>& m) {
    while (!m.empty() && m.back() == 0) m.pop_back();
}

int cmp_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;) {
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    }
    return 0;
}

std::vector<uint32_t> add_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    std::vector<uint32_t> r(std::max(a.size(), b.size()) + 1, 0);
    uint64_t c = 0;
    for (size_t i = 0; i < r.size(); ++i) {
        uint64_t s = c;
        if (i < a.size()) s += a[i];
        if (i < b.size()) s += b[i];
        r[i] = (uint32_t)s;
        c = s >> 32;
    }
    trim(r);
    return r;
}

// a - b with |a| >= |b|
std::vector<uint32_t> sub_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    std::vector<uint32_t> r(a.size(), 0);
    int64_t br = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        int64_t s = (int64_t)a[i] - br - (i < b.size() ? (int64_t)b[i] : 0);
        if (s < 0) { s += ((int64_t)1 << 32); br = 1; } else br = 0;
        r[i] = (uint32_t)s;
    }
    trim(r);
    return r;
}

Big add(const Big& a, const Big& b) {
    if (a.zero()) return b;
    if (b.zero()) return a;
    Big r;
    if (a.sgn == b.sgn) {
        r.mag = add_mag(a.mag, b.mag);
        r.sgn = a.sgn;
        return r;
    }
    int c = cmp_mag(a.mag, b.mag);
    if (c == 0) return r;
    if (c > 0) { r.mag = sub_mag(a.mag, b.mag); r.sgn = a.sgn; }
    else       { r.mag = sub_mag(b.mag, a.mag); r.sgn = b.sgn; }
    return r;
}

Big neg(Big a) { a.sgn = -a.sgn; return a; }
Big sub(const Big& a, const Big& b) { return add(a, neg(b)); }

Big mul(const Big& a, const Big& b) {
    Big r;
    if (a.zero() || b.zero()) return r;
    std::vector<uint64_t> acc(a.mag.size() + b.mag.size() + 1, 0);
    for (size_t i = 0; i < a.mag.size(); ++i) {
        uint64_t carry = 0;
        for (size_t j = 0; j < b.mag.size(); ++j) {
            uint64_t t = (uint64_t)a.mag[i] * b.mag[j] + (acc[i + j] & 0xffffffffu) + carry;
            acc[i + j] = t & 0xffffffffu;
            carry = t >> 32;
        }
        size_t k = i + b.mag.size();
        while (carry) {
            uint64_t t = acc[k] + carry;
            acc[k] = t & 0xffffffffu;
            carry = t >> 32;
            ++k;
        }
    }
    r.mag.resize(acc.size());
    for (size_t i = 0; i < acc.size(); ++i) r.mag[i] = (uint32_t)acc[i];
    trim(r.mag);
    r.sgn = r.mag.empty() ? 0 : a.sgn * b.sgn;
    return r;
}

Big shl(const Big& a, int s) {
    if (a.zero() || s == 0) return a;
    Big r;
    r.sgn = a.sgn;
    int w = s / 32, bits = s % 32;
    r.mag.assign(a.mag.size() + w + 1, 0);
    for (size_t i = 0; i < a.mag.size(); ++i) {
        uint64_t v = (uint64_t)a.mag[i] << bits;
        r.mag[i + w] |= (uint32_t)v;
        r.mag[i + w + 1] |= (uint32_t)(v >> 32);
    }
    trim(r.mag);
    return r;
}

// ----------------------------------------------------- exact integerisation
// Exponent of the lowest set bit of a finite nonzero double.
int low_exponent(double v) {
    int e;
    double f = std::frexp(std::fabs(v), &e);           // v = f * 2^e, f in [0.5,1)
    uint64_t M = (uint64_t)std::ldexp(f, 53);           // exact 53-bit integer
    int tz = __builtin_ctzll(M);
    return e - 53 + tz;
}

// v * 2^-E as an exact integer (v must be a multiple of 2^E).
Big scaled(double v, int E) {
    if (v == 0.0) return Big();
    int e;
    double f = std::frexp(std::fabs(v), &e);
    uint64_t M = (uint64_t)std::ldexp(f, 53);
    int sh = e - 53 - E;
    while (sh < 0) { M >>= 1; ++sh; }                   // drops only zero bits
    Big b = Big::from_u64(M, v < 0 ? -1 : 1);
    return shl(b, sh);
}

// ------------------------------------------------------------- determinants
const double U64 = std::ldexp(1.0, -53);

// Laplace expansion along the last column (zero entries skipped).
// Returns the value; *abs_out receives the same expression over |entries|.
double det_fp(const std::vector<double>& M, int s, double* abs_out) {
    if (s == 0) { *abs_out = 1.0; return 1.0; }
    if (s == 1) { *abs_out = std::fabs(M[0]); return M[0]; }
    double val = 0.0, ab = 0.0;
    std::vector<double> sub((s - 1) * (s - 1));
    for (int i = 0; i < s; ++i) {
        double a = M[i * s + (s - 1)];
        if (a == 0.0) continue;
        int r = 0;
        for (int ii = 0; ii < s; ++ii) {
            if (ii == i) continue;
            for (int jj = 0; jj < s - 1; ++jj) sub[r * (s - 1) + jj] = M[ii * s + jj];
            ++r;
        }
        double sa;
        double sv = det_fp(sub, s - 1, &sa);
        double sign = ((i + s - 1) % 2 == 0) ? 1.0 : -1.0;
        val += sign * a * sv;
        ab += std::fabs(a) * sa;
    }
    *abs_out = ab;
    return val;
}

// Error bound for det_fp on an s x s matrix whose entries carry at most one
// relative rounding each.  Every monomial passes through at most s input
// roundings, s-1 products and, per level, at most s additions.
double det_bound(double absval, int s) {
    double N = (double)(s * s + 3 * s + 4);
    return absval * (N * U64) / (1.0 - N * U64) * 1.0001;
}

Big det_big(const std::vector<Big>& M, int s) {
    if (s == 0) return Big::from_i64(1);
    if (s == 1) return M[0];
    Big val;
    std::vector<Big> sub((s - 1) * (s - 1));
    for (int i = 0; i < s; ++i) {
        const Big& a = M[i * s + (s - 1)];
        if (a.zero()) continue;
        int r = 0;
        for (int ii = 0; ii < s; ++ii) {
            if (ii == i) continue;
            for (int jj = 0; jj < s - 1; ++jj) sub[r * (s - 1) + jj] = M[ii * s + jj];
            ++r;
        }
        Big t = mul(a, det_big(sub, s - 1));
        if ((i + s - 1) % 2 != 0) t = neg(t);
        val = add(val, t);
    }
    return val;
}

Big dot_big(const std::vector<Big>& g, const Big* x, int p) {
    Big s;
    for (int i = 0; i < p; ++i) s = add(s, mul(g[i], x[i]));
    return s;
}

// ------------------------------------------------------------ point sets
struct PointSet {
    int p = 0;
    int n = 0;
    std::vector<Big> xi;     // n*p exact integers
    std::vector<double> xd;  // n*p rounded values (relative error <= u)
    const Big* ex(int i) const { return &xi[(size_t)i * p]; }
    const double* fd(int i) const { return &xd[(size_t)i * p]; }
};

// Is the s-minor of the (p x cols) column set on the given rows nonzero?
// cols: indices into P.  Exact unless the float64 filter settles it.
int minor_sign(const PointSet& P, const std::vector<int>& cols, const std::vector<int>& rows,
               bool exact_only) {
    int s = (int)cols.size();
    if (!exact_only) {
        std::vector<double> M(s * s);
        for (int r = 0; r < s; ++r)
            for (int c = 0; c < s; ++c) M[r * s + c] = P.fd(cols[c])[rows[r]];
        double ab;
        double v = det_fp(M, s, &ab);
        if (std::fabs(v) > det_bound(ab, s)) return v > 0 ? 1 : -1;
    }
    std::vector<Big> M(s * s);
    for (int r = 0; r < s; ++r)
        for (int c = 0; c < s; ++c) M[r * s + c] = P.ex(cols[c])[rows[r]];
    return det_big(M, s).sgn;
}

bool next_comb(std::vector<int>& c, int n) {
    int k = (int)c.size();
    for (int i = k - 1; i >= 0; --i) {
        if (c[i] < n - k + i) {
            ++c[i];
            for (int j = i + 1; j < k; ++j) c[j] = c[j - 1] + 1;
            return true;
        }
    }
    return false;
}

// Rank of the columns `idx` of P, and rows giving a nonzero maximal minor.
int rank_of(const PointSet& P, const std::vector<int>& idx, std::vector<int>* basis_rows,
            bool exact_only) {
    std::vector<int> basis;
    for (int v : idx) {
        if ((int)basis.size() == P.p) break;
        std::vector<int> cols = basis;
        cols.push_back(v);
        int s = (int)cols.size();
        std::vector<int> rows(s);
        for (int i = 0; i < s; ++i) rows[i] = i;
        bool indep = false;
        do {
            if (minor_sign(P, cols, rows, exact_only) != 0) { indep = true; break; }
        } while (next_comb(rows, P.p));
        if (indep) basis.push_back(v);
    }
    if (basis_rows) {
        int s = (int)basis.size();
        std::vector<int> rows(s);
        for (int i = 0; i < s; ++i) rows[i] = i;
        basis_rows->clear();
        if (s == 0) return 0;
        do {
            if (minor_sign(P, basis, rows, exact_only) != 0) { *basis_rows = rows; break; }
        } while (next_comb(rows, P.p));
    }
    return (int)basis.size();
}

PointSet restrict_rows(const PointSet& P, const std::vector<int>& idx, const std::vector<int>& rows) {
    PointSet Q;
    Q.p = (int)rows.size();
    Q.n = (int)idx.size();
    Q.xi.resize((size_t)Q.n * Q.p);
    Q.xd.resize((size_t)Q.n * Q.p);
    for (int i = 0; i < Q.n; ++i)
        for (int r = 0; r < Q.p; ++r) {
            Q.xi[(size_t)i * Q.p + r] = P.ex(idx[i])[rows[r]];
            Q.xd[(size_t)i * Q.p + r] = P.fd(idx[i])[rows[r]];
        }
    return Q;
}

// ---------------------------------------------------- small exact depth
// min over generic u of #{ v : u'v < 0 } for nonzero integer vectors, by the
// critical-direction route (equation (4)): every optimal open cone has an
// extreme ray normal to d-1 independent points; near that ray the count is
// the strict count plus the depth of the points on the hyperplane.
int small_depth(const PointSet& V) {
    if (V.n == 0) return 0;
    std::vector<int> all(V.n);
    for (int i = 0; i < V.n; ++i) all[i] = i;
    std::vector<int> rows;
    int rho = rank_of(V, all, &rows, true);
    if (rho < V.p) return small_depth(restrict_rows(V, all, rows));
    int d = V.p;
    if (d == 1) {
        int pos = 0, neg = 0;
        for (int i = 0; i < V.n; ++i) (V.ex(i)[0].sgn > 0 ? pos : neg)++;
        return std::min(pos, neg);
    }
    int best = V.n;
    std::vector<int> J(d - 1);
    for (int i = 0; i < d - 1; ++i) J[i] = i;
    if (V.n < d - 1) return 0;
    do {
        // generalised cross product u_i = det[v_J | e_i]
        std::vector<Big> u(d);
        bool nz = false;
        for (int i = 0; i < d; ++i) {
            std::vector<Big> M(d * d);
            for (int r = 0; r < d; ++r) {
                for (int c = 0; c < d - 1; ++c) M[r * d + c] = V.ex(J[c])[r];
                M[r * d + (d - 1)] = Big::from_i64(r == i ? 1 : 0);
            }
            u[i] = det_big(M, d);
            if (!u[i].zero()) nz = true;
        }
        if (!nz) continue;
        int pos = 0, neg = 0, drop = -1;
        for (int i = 0; i < d; ++i) if (!u[i].zero()) { drop = i; break; }
        std::vector<int> on;
        for (int l = 0; l < V.n; ++l) {
            int s = dot_big(u, V.ex(l), d).sgn;
            if (s > 0) ++pos; else if (s < 0) ++neg; else on.push_back(l);
        }
        std::vector<int> keep;
        for (int r = 0; r < d; ++r) if (r != drop) keep.push_back(r);
        int rec = small_depth(restrict_rows(V, on, keep));
        best = std::min(best, std::min(pos, neg) + rec);
    } while (next_comb(J, V.n));
    return best;
}

// ------------------------------------------------- per-subset computation
struct Ctx {
    const PointSet* P;
    bool exact_only;
};

// Returns delta_I + b_I for the subset `I`, or -1 if the subset is invalid.
// If `argmin` is given, it receives the points (indices, ascending) of the
// runs of equal angle next to a state of the sweep where min(S, m - S) = b_I:
// the points that, with I, span a critical hyperplane attaining b_I
// (Algorithm 3, Steps 2(c) and 4(a)(ii)).
int subset_term(const Ctx& C, const std::vector<int>& I, std::vector<int>* argmin = nullptr) {
    const PointSet& P = *C.P;
    const int p = P.p, k = p - 2;
    const bool xo = C.exact_only;

    // ---- row pair (j,kk) with omega = det[x_I | e_j | e_kk] != 0
    auto build_unit = [&](int a, int b, std::vector<double>* Md, std::vector<Big>* Mb) {
        // p x p matrix [x_I | e_a | e_b]
        if (Md) {
            Md->assign(p * p, 0.0);
            for (int r = 0; r < p; ++r) {
                for (int c = 0; c < k; ++c) (*Md)[r * p + c] = P.fd(I[c])[r];
                (*Md)[r * p + k] = (r == a) ? 1.0 : 0.0;
                (*Md)[r * p + k + 1] = (r == b) ? 1.0 : 0.0;
            }
        }
        if (Mb) {
            Mb->assign(p * p, Big());
            for (int r = 0; r < p; ++r) {
                for (int c = 0; c < k; ++c) (*Mb)[r * p + c] = P.ex(I[c])[r];
                (*Mb)[r * p + k] = Big::from_i64(r == a ? 1 : 0);
                (*Mb)[r * p + k + 1] = Big::from_i64(r == b ? 1 : 0);
            }
        }
    };
    int J = -1, K = -1;
    {
        double bestv = -1.0;
        std::vector<double> Md;
        std::vector<std::pair<double, std::pair<int, int>>> cand;
        for (int a = 0; a < p; ++a)
            for (int b = a + 1; b < p; ++b) {
                build_unit(a, b, &Md, nullptr);
                double ab;
                double v = det_fp(Md, p, &ab);
                cand.push_back({std::fabs(v), {a, b}});
                if (!xo && std::fabs(v) > det_bound(ab, p) && std::fabs(v) > bestv) {
                    bestv = std::fabs(v);
                    J = a; K = b;
                }
            }
        if (J < 0) {
            std::sort(cand.begin(), cand.end(), [](auto& x, auto& y) { return x.first > y.first; });
            std::vector<Big> Mb;
            for (auto& c : cand) {
                build_unit(c.second.first, c.second.second, nullptr, &Mb);
                if (!det_big(Mb, p).zero()) { J = c.second.first; K = c.second.second; break; }
            }
        }
        if (J < 0) return -1;   // x_I linearly dependent: no 2-D complement
    }

    // ---- Pluecker rows g1_i = det[x_I | e_i | e_J], g2_i = det[x_I | e_i | e_K]
    std::vector<double> g1(p), g2(p), E1(p), E2(p);
    {
        std::vector<double> Md;
        for (int i = 0; i < p; ++i) {
            double ab;
            build_unit(i, J, &Md, nullptr);
            g1[i] = det_fp(Md, p, &ab);
            E1[i] = det_bound(ab, p);
            build_unit(i, K, &Md, nullptr);
            g2[i] = det_fp(Md, p, &ab);
            E2[i] = det_bound(ab, p);
        }
    }
    std::vector<Big> G1, G2;     // exact rows, computed on first need
    auto need_exact_rows = [&]() {
        if (!G1.empty()) return;
        G1.resize(p); G2.resize(p);
        std::vector<Big> Mb;
        for (int i = 0; i < p; ++i) {
            build_unit(i, J, nullptr, &Mb);
            G1[i] = det_big(Mb, p);
            build_unit(i, K, nullptr, &Mb);
            G2[i] = det_big(Mb, p);
        }
    };

    std::vector<char> inI(P.n, 0);
    for (int v : I) inI[v] = 1;

    struct Pt {
        int idx;
        int sig;          // fold sign
        double h1, h2;    // folded float64 coordinates
        double e;         // absolute error bound on h1 and h2
        bool have_exact;
        Big H1, H2;       // folded exact coordinates (if computed)
    };
    std::vector<Pt> pts;
    pts.reserve(P.n);
    std::vector<int> inspan;   // K_I \ I
    const double gam = (double)(p + 3) * U64 * 1.0001;
    for (int l = 0; l < P.n; ++l) {
        if (inI[l]) continue;
        const double* x = P.fd(l);
        double y1 = 0, y2 = 0, a1 = 0, a2 = 0, b1 = 0, b2 = 0;
        for (int i = 0; i < p; ++i) {
            y1 += g1[i] * x[i];
            y2 += g2[i] * x[i];
            a1 += std::fabs(g1[i] * x[i]);
            a2 += std::fabs(g2[i] * x[i]);
            b1 += E1[i] * std::fabs(x[i]);
            b2 += E2[i] * std::fabs(x[i]);
        }
        double e1 = (b1 * (1 + 2 * U64) + gam * a1) * 1.0001;
        double e2 = (b2 * (1 + 2 * U64) + gam * a2) * 1.0001;
        double e = std::max(e1, e2);
        Pt q;
        q.idx = l;
        q.e = e;
        q.have_exact = false;
        int s1 = (!xo && std::fabs(y1) > e1) ? (y1 > 0 ? 1 : -1) : 2;   // 2 = unknown
        if (s1 == 2) {
            need_exact_rows();
            Big Y1 = dot_big(G1, P.ex(l), p);
            Big Y2 = dot_big(G2, P.ex(l), p);
            if (Y1.zero() && Y2.zero()) { inspan.push_back(l); continue; }
            q.sig = Y1.zero() ? Y2.sgn : Y1.sgn;
            q.have_exact = true;
            q.H1 = q.sig > 0 ? Y1 : neg(Y1);
            q.H2 = q.sig > 0 ? Y2 : neg(Y2);
        } else {
            q.sig = s1;
        }
        q.h1 = q.sig * y1;
        q.h2 = q.sig * y2;
        pts.push_back(std::move(q));
    }

    auto exact_of = [&](Pt& q) {
        if (q.have_exact) return;
        need_exact_rows();
        Big Y1 = dot_big(G1, P.ex(q.idx), p);
        Big Y2 = dot_big(G2, P.ex(q.idx), p);
        q.H1 = q.sig > 0 ? Y1 : neg(Y1);
        q.H2 = q.sig > 0 ? Y2 : neg(Y2);
        q.have_exact = true;
    };
    // orientation of the folded pair: sign of cross(h_a, h_b)
    auto orient = [&](Pt& a, Pt& b) -> int {
        if (!xo) {
            double c = a.h1 * b.h2 - a.h2 * b.h1;
            double bound = a.e * (std::fabs(b.h1) + std::fabs(b.h2)) + b.e * (std::fabs(a.h1) + std::fabs(a.h2))
                         + 2.0 * a.e * b.e + 3.0 * U64 * (std::fabs(a.h1 * b.h2) + std::fabs(a.h2 * b.h1));
            bound *= 1.0001;
            if (std::fabs(c) > bound) return c > 0 ? 1 : -1;
        }
        exact_of(a);
        exact_of(b);
        return sub(mul(a.H1, b.H2), mul(a.H2, b.H1)).sgn;
    };

    // Angular order of the folded points (Algorithm 2, Step 1(e)).  A float64
    // angle gives a candidate order; it is accepted only if every adjacent
    // pair is confirmed non-decreasing by the exact orientation predicate,
    // which for a total preorder proves the whole order.  Otherwise the points
    // are sorted again with the exact predicate as comparator.
    std::vector<int> order(pts.size());
    for (size_t i = 0; i < pts.size(); ++i) order[i] = (int)i;
    std::vector<double> ang(pts.size());
    for (size_t i = 0; i < pts.size(); ++i) ang[i] = std::atan2(pts[i].h2, pts[i].h1);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return ang[a] < ang[b]; });
    std::vector<int> adj(order.empty() ? 0 : order.size() - 1);
    bool ok = true;
    for (size_t i = 0; i + 1 < order.size(); ++i) {
        adj[i] = orient(pts[order[i]], pts[order[i + 1]]);
        if (adj[i] < 0) { ok = false; break; }
    }
    if (!ok) {
        std::sort(order.begin(), order.end(), [&](int a, int b) { return orient(pts[a], pts[b]) > 0; });
        for (size_t i = 0; i + 1 < order.size(); ++i) adj[i] = orient(pts[order[i]], pts[order[i + 1]]);
    }

    // ---- circular sweep with grouped ties (Algorithm 2, Step 1(c)-(e))
    const int m = (int)pts.size();
    int S = 0;
    for (auto& q : pts) if (q.sig > 0) ++S;
    int best = std::min(S, m - S);
    const int S_start = S;
    for (size_t i = 0; i < order.size(); ++i) {
        S += -pts[order[i]].sig;
        bool run_end = (i + 1 == order.size()) || adj[i] != 0;
        if (run_end) best = std::min(best, std::min(S, m - S));
    }
    if (argmin) {
        // runs of exactly equal angle; state r is the one after run r - 1
        // (state 0 before the first run, state R after the last: both lie
        // next to the last and the first run, the sweep being circular)
        argmin->clear();
        std::vector<int> run_of(order.size());
        int R = 0;
        for (size_t i = 0; i < order.size(); ++i) {
            run_of[i] = R;
            if ((i + 1 == order.size()) || adj[i] != 0) ++R;
        }
        std::vector<int> st((size_t)R + 1);
        int Sr = S_start;
        st[0] = Sr;
        for (size_t i = 0; i < order.size(); ++i) {
            Sr += -pts[order[i]].sig;
            if ((i + 1 == order.size()) || adj[i] != 0) st[(size_t)run_of[i] + 1] = Sr;
        }
        std::vector<char> hot((size_t)R, 0);
        for (int r = 0; r <= R && R > 0; ++r) {
            if (std::min(st[(size_t)r], m - st[(size_t)r]) != best) continue;
            if (r == 0 || r == R) { hot[(size_t)R - 1] = 1; hot[0] = 1; }
            else { hot[(size_t)r - 1] = 1; hot[(size_t)r] = 1; }
        }
        for (size_t i = 0; i < order.size(); ++i)
            if (hot[(size_t)run_of[i]]) argmin->push_back(pts[order[i]].idx);
        std::sort(argmin->begin(), argmin->end());
    }

    // ---- depth of 0 inside span(x_I) among the points lying there
    int delta = 0;
    if (!inspan.empty()) {
        std::vector<int> Kset = I;
        for (int v : inspan) Kset.push_back(v);
        std::vector<int> rows(p);
        for (int r = 0; r < p; ++r) rows[r] = r;
        delta = small_depth(restrict_rows(P, Kset, rows));
    }
    return delta + best;
}

uint64_t binom(int n, int k) {
    if (k < 0 || n < k) return 0;
    uint64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
    return r;
}

// lexicographic unranking of k-subsets of {0..n-1}
void unrank_lex(uint64_t r, int n, int k, std::vector<int>& c) {
    c.resize(k);
    int x = 0;
    for (int i = 0; i < k; ++i) {
        while (true) {
            uint64_t b = binom(n - x - 1, k - i - 1);
            if (r < b) break;
            r -= b;
            ++x;
        }
        c[i] = x++;
    }
}

// Visits the subsets of lexicographic rank [r0, r1) in rank order, in
// chunks of `chunk` consecutive ranks: each chunk starts from an unranked
// subset and steps with next_comb (the loop of Algorithm 1, Step 1, over
// the index set of (p-2)-subsets, split for the threads).  fn(chunk, rank,
// subset) is called once per rank; the chunks run in parallel.
template <typename Fn>
void visit_range(uint64_t r0, uint64_t r1, int n, int k, uint64_t chunk, Fn&& fn) {
    if (r1 <= r0) return;
    const int64_t nchunks = (int64_t)((r1 - r0 + chunk - 1) / chunk);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        uint64_t a = r0 + (uint64_t)ch * chunk, b = std::min(r1, a + chunk);
        std::vector<int> I;
        unrank_lex(a, n, k, I);
        for (uint64_t r = a; r < b; ++r) {
            fn(ch, r, I);
            if (r + 1 < b) next_comb(I, n);
        }
    }
}

// Minimum of the valid subsets' terms over the ranks [r0, r1) (INT_MAX if
// none is valid), and the number of subsets visited.
int thread_slot() {
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

int thread_slots() {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int min_over_range(const Ctx& C, uint64_t r0, uint64_t r1, uint64_t* visited) {
    const int n = C.P->n, k = C.P->p - 2;
    // per-thread minimum and count, combined after the loop
    std::vector<int> best((size_t)thread_slots(), std::numeric_limits<int>::max());
    std::vector<uint64_t> cnt((size_t)thread_slots(), 0);
    visit_range(r0, r1, n, k, 256, [&](int64_t, uint64_t, const std::vector<int>& I) {
        const int t = subset_term(C, I);
        const size_t w = (size_t)thread_slot();
        if (t >= 0 && t < best[w]) best[w] = t;
        ++cnt[w];
    });
    int b = std::numeric_limits<int>::max();
    uint64_t v = 0;
    for (size_t w = 0; w < best.size(); ++w) {
        b = std::min(b, best[w]);
        v += cnt[w];
    }
    if (visited) *visited = v;
    return b;
}

struct Prepared {
    int n0 = 0;
    int kind = 0;   // 0: use subsets, 1: closed form value in `value`
    int value = 0;
    PointSet P;     // centred nonzero points, mapped into their span
};

Prepared prepare(const double* X, int64_t n, int p, const double* z, bool exact_only) {
    Prepared R;
    int E = std::numeric_limits<int>::max();
    for (int64_t i = 0; i < n * p; ++i) if (X[i] != 0.0) E = std::min(E, low_exponent(X[i]));
    for (int c = 0; c < p; ++c) if (z[c] != 0.0) E = std::min(E, low_exponent(z[c]));
    if (E == std::numeric_limits<int>::max()) E = 0;
    PointSet W;
    W.p = p;
    std::vector<Big> zi(p);
    for (int c = 0; c < p; ++c) zi[c] = scaled(z[c], E);
    for (int64_t i = 0; i < n; ++i) {
        bool same = true;
        for (int c = 0; c < p; ++c) if (X[i * p + c] != z[c]) { same = false; break; }
        if (same) { ++R.n0; continue; }
        for (int c = 0; c < p; ++c) {
            W.xi.push_back(sub(scaled(X[i * p + c], E), zi[c]));
            W.xd.push_back(X[i * p + c] - z[c]);
        }
        ++W.n;
    }
    if (W.n == 0) { R.kind = 1; R.value = 0; return R; }
    std::vector<int> all(W.n);
    for (int i = 0; i < W.n; ++i) all[i] = i;
    std::vector<int> rows;
    int rho = rank_of(W, all, &rows, exact_only);
    PointSet Q = (rho < p) ? restrict_rows(W, all, rows) : W;
    if (Q.p == 1) {
        int pos = 0, neg = 0;
        for (int i = 0; i < Q.n; ++i) (Q.ex(i)[0].sgn > 0 ? pos : neg)++;
        R.kind = 1;
        R.value = std::min(pos, neg);
        return R;
    }
    R.P = std::move(Q);
    return R;
}

// ------------------------------------------------ Algorithm 3 (ADIA)
// Exact sign of the inner product x_a . x_b of two centred points.
int dot_sign(const PointSet& P, int a, int b, bool exact_only) {
    const int p = P.p;
    if (!exact_only) {
        double v = 0.0, ab = 0.0;
        for (int c = 0; c < p; ++c) {
            v += P.fd(a)[c] * P.fd(b)[c];
            ab += std::fabs(P.fd(a)[c] * P.fd(b)[c]);
        }
        const double N = (double)(2 * p + 4);
        if (std::fabs(v) > ab * N * U64 / (1.0 - N * U64) * 1.0001) return v > 0 ? 1 : -1;
    }
    return dot_big(std::vector<Big>(P.ex(a), P.ex(a) + p), P.ex(b), p).sgn;
}

bool contains(const std::vector<int>& v, int x) { return std::find(v.begin(), v.end(), x) != v.end(); }

std::vector<int> with(std::vector<int> v, int x) {
    v.push_back(x);
    std::sort(v.begin(), v.end());
    return v;
}

std::vector<int> without(const std::vector<int>& v, size_t r) {
    std::vector<int> w;
    for (size_t i = 0; i < v.size(); ++i)
        if (i != r) w.push_back(v[i]);
    return w;
}

// Algorithm 3 (Section 4) on the centred nonzero points of one query, with
// the counts of Algorithm 1 (a subset's value is delta_I + b_I, so that the
// value of a critical (p-1)-set is that of the subset it came from).
// Returns the ADIA value (without n0), or -1 where the algorithm does not
// apply (p < 3, n' <= 2p, or no seed subset; the caller then uses
// Algorithm 1, as the paper recommends for n <= 2p).  *ksize receives the
// number of candidate points of Step 5.
//
// Readings: the popped node's (p-2)-subsets are taken in the order of the
// element left out (first element first); new nodes are appended in
// ascending order of the added point; the seed point x_{i_{p-1}} of Step 2(c)
// is the smallest index next to a minimising state of the seed subset; the
// side X_F of Step 5(a) is the closed side of F's hyperplane holding fewer
// points (the side with det[x_F | x] <= 0 on a tie); Step 5's candidates
// also hold the points of the subset that attained d0 in Step 4, so that its
// value is one of those of Step 5(b).
int adia_term(const PointSet& P, bool xo, int64_t* ksize) {
    const int p = P.p, k = p - 2, n = P.n;
    *ksize = -1;
    if (p < 3 || n <= 2 * p) return -1;
    Ctx C{&P, xo};
    // Step 2(a): the direction among +-x_j with the fewest points on its
    // closed negative side
    int bestc = std::numeric_limits<int>::max(), bj = -1, bs = 0;
    for (int j = 0; j < n; ++j) {
        int cp = 0, cn = 0;   // #{x_j . x_i <= 0}, #{x_j . x_i >= 0}
        for (int i = 0; i < n; ++i) {
            const int d = dot_sign(P, j, i, xo);
            if (d <= 0) ++cp;
            if (d >= 0) ++cn;
        }
        if (cp < bestc) { bestc = cp; bj = j; bs = 1; }
        if (cn < bestc) { bestc = cn; bj = j; bs = -1; }
    }
    // Step 2(b): order by u_min . x; the seed subset is the p - 2 points with
    // the smallest nonnegative projections
    std::vector<Big> pr((size_t)n);
    int kneg = 0;
    for (int i = 0; i < n; ++i) {
        Big d = dot_big(std::vector<Big>(P.ex(bj), P.ex(bj) + p), P.ex(i), p);
        pr[(size_t)i] = bs > 0 ? d : neg(d);
        if (pr[(size_t)i].sgn < 0) ++kneg;
    }
    if (kneg == 0) { *ksize = 0; return 0; }   // no point strictly below: depth 0 (Step 6)
    std::vector<int> nonneg;
    for (int i = 0; i < n; ++i)
        if (pr[(size_t)i].sgn >= 0) nonneg.push_back(i);
    std::sort(nonneg.begin(), nonneg.end(), [&](int a, int b) {
        const int c = sub(pr[(size_t)a], pr[(size_t)b]).sgn;
        return c < 0 || (c == 0 && a < b);
    });
    if ((int)nonneg.size() < k) return -1;
    std::vector<int> I0(nonneg.begin(), nonneg.begin() + k);
    std::sort(I0.begin(), I0.end());
    // Step 2(c): the seed critical set
    std::vector<int> T;
    const int t0 = subset_term(C, I0, &T);
    if (t0 < 0) return -1;
    int h = -1;
    for (int v : T)
        if (!contains(I0, v)) { h = v; break; }
    if (h < 0) return -1;
    // Step 3
    std::map<std::vector<int>, int> Q;
    std::deque<std::vector<int>> N;
    const std::vector<int> C0 = with(I0, h);
    Q[C0] = t0;
    N.push_back(C0);
    int d0 = t0;
    std::vector<int> bestJ = I0;
    // Step 4
    while (!N.empty()) {
        const std::vector<int> F = N.front();
        N.pop_front();
        for (size_t r = 0; r < F.size(); ++r) {
            const std::vector<int> J = without(F, r);
            std::vector<int> TJ;
            const int dt = subset_term(C, J, &TJ);
            if (dt < 0) continue;
            for (int v : TJ) {
                if (contains(F, v)) continue;
                const std::vector<int> Nn = with(J, v);
                if (!Q.count(Nn)) {
                    Q[Nn] = dt;
                    N.push_back(Nn);
                }
            }
            if (d0 > dt) {
                d0 = dt;
                bestJ = J;
                break;
            }
        }
        for (auto it = Q.begin(); it != Q.end();) {
            if (it->second > d0) it = Q.erase(it); else ++it;
        }
        std::deque<std::vector<int>> keep;
        for (auto& e : N)
            if (Q.count(e)) keep.push_back(e);
        N.swap(keep);
    }
    // Step 5(a): candidate points, the closed smaller side of every remaining
    // critical hyperplane
    std::vector<char> inK((size_t)n, 0);
    std::vector<int> rows((size_t)p);
    for (int r = 0; r < p; ++r) rows[(size_t)r] = r;
    for (const auto& e : Q) {
        std::vector<int> sg((size_t)n);
        int cneg = 0, cpos = 0;
        for (int l = 0; l < n; ++l) {
            std::vector<int> cols = e.first;
            cols.push_back(l);
            sg[(size_t)l] = contains(e.first, l) ? 0 : minor_sign(P, cols, rows, xo);
            if (sg[(size_t)l] < 0) ++cneg;
            if (sg[(size_t)l] > 0) ++cpos;
        }
        const int side = (cneg <= cpos) ? -1 : 1;
        for (int l = 0; l < n; ++l)
            if (sg[(size_t)l] == 0 || sg[(size_t)l] == side) inK[(size_t)l] = 1;
    }
    for (int v : bestJ) inK[(size_t)v] = 1;
    std::vector<int> K;
    for (int l = 0; l < n; ++l)
        if (inK[(size_t)l]) K.push_back(l);
    *ksize = (int64_t)K.size();
    // Step 5(b): Algorithm 1 over the (p-2)-subsets of the candidates
    const uint64_t total = binom((int)K.size(), k);
    std::vector<int> best5((size_t)thread_slots(), std::numeric_limits<int>::max());
    visit_range(0, total, (int)K.size(), k, 256, [&](int64_t, uint64_t, const std::vector<int>& pos) {
        std::vector<int> I((size_t)k);
        for (int c = 0; c < k; ++c) I[(size_t)c] = K[(size_t)pos[(size_t)c]];
        const int t = subset_term(C, I);
        const size_t w = (size_t)thread_slot();
        if (t >= 0 && t < best5[w]) best5[w] = t;
    });
    for (int b : best5) d0 = std::min(d0, b);
    return d0;
}

}  // namespace

extern "C" {

enum { ORACLE_EXACT_ONLY = 1 };

// Depth counts of the m queries Z (m x p, row-major) w.r.t. X (n x p).
// out[q] = n * D_n(Z_q).  threads <= 0: OpenMP default.  Returns 0 on success.
int oracle_depth(const double* X, int64_t n, int32_t p, const double* Z, int64_t m,
                 int64_t* out, int32_t threads, int32_t flags) {
    if (!X || !Z || !out || n < 1 || p < 1 || m < 0) return 1;
    for (int64_t i = 0; i < n * p; ++i) if (!std::isfinite(X[i])) return 2;
    for (int64_t i = 0; i < m * p; ++i) if (!std::isfinite(Z[i])) return 2;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
    const bool xo = (flags & ORACLE_EXACT_ONLY) != 0;
    for (int64_t q = 0; q < m; ++q) {
        Prepared R = prepare(X, n, p, Z + q * p, xo);
        if (R.kind == 1) { out[q] = R.n0 + R.value; continue; }
        const int k = R.P.p - 2;
        const uint64_t total = binom(R.P.n, k);
        Ctx C{&R.P, xo};
        const int best = min_over_range(C, 0, total, nullptr);
        out[q] = R.n0 + best;   // at least one valid subset exists after the span map
    }
    return 0;
}

// Minimum of delta_I + b_I over the subsets of lexicographic rank [r0, r1)
// for one query (a bounded sample of the full loop), plus n0 (-1 if no
// subset in the range is valid).  Only defined when the centred points span
// R^p.  *swept receives the number of subsets visited (counted).
int oracle_depth_range(const double* X, int64_t n, int32_t p, const double* z, uint64_t r0,
                       uint64_t r1, int64_t* out_min, uint64_t* swept, int32_t threads,
                       int32_t flags) {
    if (!X || !z || !out_min || !swept || n < 1 || p < 3) return 1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
    const bool xo = (flags & ORACLE_EXACT_ONLY) != 0;
    Prepared R = prepare(X, n, p, z, xo);
    if (R.kind == 1 || R.P.p != p) return 3;
    const int k = p - 2;
    const uint64_t total = binom(R.P.n, k);
    r1 = std::min(r1, total);
    if (r0 > r1) r0 = r1;
    Ctx C{&R.P, xo};
    const int best = min_over_range(C, r0, r1, swept);
    *out_min = (best == std::numeric_limits<int>::max()) ? -1 : (int64_t)(R.n0 + best);
    return 0;
}

// Depth count by the critical-direction route alone (equation (4) with the
// exact recursion for points on the critical hyperplane).  O(n^p): tiny inputs.
int oracle_depth_vertex(const double* X, int64_t n, int32_t p, const double* z, int64_t* out) {
    if (!X || !z || !out || n < 1 || p < 1) return 1;
    int E = std::numeric_limits<int>::max();
    for (int64_t i = 0; i < n * p; ++i) if (X[i] != 0.0) E = std::min(E, low_exponent(X[i]));
    for (int c = 0; c < p; ++c) if (z[c] != 0.0) E = std::min(E, low_exponent(z[c]));
    if (E == std::numeric_limits<int>::max()) E = 0;
    PointSet W;
    W.p = p;
    int n0 = 0;
    for (int64_t i = 0; i < n; ++i) {
        bool same = true;
        for (int c = 0; c < p; ++c) if (X[i * p + c] != z[c]) { same = false; break; }
        if (same) { ++n0; continue; }
        for (int c = 0; c < p; ++c) {
            W.xi.push_back(sub(scaled(X[i * p + c], E), scaled(z[c], E)));
            W.xd.push_back(X[i * p + c] - z[c]);
        }
        ++W.n;
    }
    *out = n0 + small_depth(W);
    return 0;
}

uint64_t oracle_binom(int32_t n, int32_t k) { return binom(n, k); }

// Depth counts by Algorithm 3 (ADIA, Section 4): out[q] = n0 + the ADIA
// value, ksize[q] = the number of candidate points of its Step 5, or -1
// where ADIA does not apply and Algorithm 1 gave the count.  The paper
// assumes general position; the value is then the depth in the paper's
// experiments, and in every case a value attained by some subset, hence
// never below the depth.
int oracle_depth_adia(const double* X, int64_t n, int32_t p, const double* Z, int64_t m, int64_t* out,
                      int64_t* ksize, int32_t threads, int32_t flags) {
    if (!X || !Z || !out || !ksize || n < 1 || p < 1 || m < 0) return 1;
    for (int64_t i = 0; i < n * p; ++i) if (!std::isfinite(X[i])) return 2;
    for (int64_t i = 0; i < m * p; ++i) if (!std::isfinite(Z[i])) return 2;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
    const bool xo = (flags & ORACLE_EXACT_ONLY) != 0;
    for (int64_t q = 0; q < m; ++q) {
        Prepared R = prepare(X, n, p, Z + q * p, xo);
        ksize[q] = -1;
        if (R.kind == 1) { out[q] = R.n0 + R.value; continue; }
        int v = -1;
        if (R.P.p == p) v = adia_term(R.P, xo, &ksize[q]);
        if (v < 0) {
            Ctx C{&R.P, xo};
            v = min_over_range(C, 0, binom(R.P.n, R.P.p - 2), nullptr);
            ksize[q] = -1;
        }
        out[q] = R.n0 + v;
    }
    return 0;
}

// The k-subsets of {0..n-1} of lexicographic rank [r0, r1), written in rank
// order to out (k ints each), visited as the depth loop visits them: chunks
// of `chunk` ranks, each unranked at its start and stepped with next_comb.
// Returns the number of subsets written.
int64_t oracle_enumerate(int32_t n, int32_t k, uint64_t r0, uint64_t r1, uint64_t chunk,
                         int32_t* out) {
    if (n < 0 || k < 0 || k > n || !out || chunk == 0) return -1;
    r1 = std::min(r1, binom(n, k));
    if (r0 > r1) r0 = r1;
    visit_range(r0, r1, n, k, chunk, [&](int64_t, uint64_t r, const std::vector<int>& I) {
        for (int i = 0; i < k; ++i) out[(r - r0) * (uint64_t)k + (uint64_t)i] = I[(size_t)i];
    });
    return (int64_t)(r1 - r0);
}

}  // extern "C"
