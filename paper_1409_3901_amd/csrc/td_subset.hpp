// The subset kernel: Algorithm 1's loop over (p-2)-subsets with Algorithm 2
// (projection, angular sort, circular sweep) as the per-subset step.
//
// Layout: one wave64 per workgroup.  A work item is a range of `chunk` (per
// class) consecutive colex ranks of one query; waves pull items from a device
// counter until none is left (persistent grid).  The points of the current
// query stay in registers: lane L holds points L*K .. L*K+K-1 (blocked), so
// the sort starts with element e = point e.  Bases are built 64 at a time,
// one subset per lane, and staged in LDS; the wave then sweeps the 64 subsets
// one after the other, every lane taking part in each sweep.
#pragma once
#include <hip/hip_runtime.h>

#include "td_common.hpp"
#include "td_device.hpp"

namespace td {

constexpr int kDefer = -2;
constexpr int kSkip = -3;
constexpr int kFallback = -4;   // bucketed sweep gave up: the exact tier takes the subset
constexpr int kNeed64 = -5;     // bucketed sweep needs the float64 basis
constexpr uint64_t kRedoUnit = 1024;   // subsets per unit of the float64 pass
constexpr int kBig = 0x7fffffff;

template <int P>
struct SlotPlain {
    double e1[P], e2[P];
    int16_t mem[P > 2 ? P - 2 : 1];
    int32_t state;   // 0 ok, 1 skip
};

template <int P>
struct SlotFilt {        // LDS: what every sweep reads
    float f1[P], f2[P];
    float beta32;    // float32 projection error of a unit-length point
    int32_t state;   // 0 ok, 1 skip (out of range / invalid), 3 defer
    int16_t mem[P > 2 ? P - 2 : 1];
};

template <int P>
struct SlotF64 {         // device scratch: read only by float64 re-checks
    double e1[P], e2[P];
    double beta64;   // float64 projection error <= beta64 * ||x||_2
    double pad;
};

// Per-block staging for the rare re-ordering of uncertain runs.
struct Staging {
    uint32_t* pkey;
    int* pS;
    uint8_t* pflag;
    double* rt;
    float* rr;
};

// f(S) = min(S, m - S): the smaller side of the line through the origin.
__device__ __forceinline__ int fside(int s, int m) { return min(s, m - s); }

// ---------------------------------------------------------------- plain
template <int P, int K>
__device__ int sweep_plain(const double (&xr)[K][P], const SlotPlain<P>& S, int nnz) {
    constexpr int KS = P - 2;
    const int lane = lane_id();
    double e1[P], e2[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
        e1[c] = S.e1[c];
        e2[c] = S.e2[c];
    }
    int mem[KS > 0 ? KS : 1];
#pragma unroll
    for (int c = 0; c < KS; ++c) mem[c] = uni(S.mem[c]);
    uint64_t key[K];
    int zc = 0, nplus = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int idx = lane * K + i;
        bool valid = idx < nnz;
#pragma unroll
        for (int c = 0; c < KS; ++c) valid = valid && (idx != mem[c]);
        double y1 = 0.0, y2 = 0.0;
#pragma unroll
        for (int c = 0; c < P; ++c) {
            y1 = fma(e1[c], xr[i][c], y1);
            y2 = fma(e2[c], xr[i][c], y2);
        }
        uint64_t kk = ~0ull;
        if (valid) {
            if (y1 == 0.0 && y2 == 0.0) {
                ++zc;   // projects to the origin (Algorithm 2, Step 1(a))
            } else {
                const bool pos = (y1 > 0.0) || (y1 == 0.0 && y2 > 0.0);
                const double h1 = pos ? y1 : -y1;
                const double h2 = pos ? y2 : -y2;
                const double t = h2 / (h1 + fabs(h2)) + 1.0;   // pseudo-angle in (0, 2]
                kk = ((uint64_t)__double_as_longlong(t) & ~1ull) | (pos ? 0ull : 1ull);
                nplus += pos ? 1 : 0;
            }
        }
        key[i] = kk;
    }
    wave_sort<K>(key);
    const int ztot = wave_sum(zc);
    const int m = nnz - KS - ztot;
    const int S0 = wave_sum(nplus);
    int dl[K];
    int loc = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        dl[i] = (key[i] == ~0ull) ? 0 : ((key[i] & 1ull) ? 1 : -1);
        loc += dl[i];
    }
    int s = S0 + wave_excl_sum(loc);
    const uint64_t nxt = ((uint64_t)(uint32_t)lane_next((int)(key[0] >> 32), 0) << 32) |
                         (uint32_t)lane_next((int)(uint32_t)key[0], 0);
    int best = (lane == 0) ? fside(S0, m) : kBig;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        s += dl[i];
        const uint64_t nk = (i + 1 < K) ? key[i + 1] : ((lane == 63) ? ~0ull : nxt);
        const bool real = key[i] != ~0ull;
        const bool run_end = real && (nk == ~0ull || ((key[i] >> 1) != (nk >> 1)));
        if (run_end) best = min(best, fside(s, m));
    }
    return wave_min(best) + ztot;
}

// ---------------------------------------------------------------- filtered
// Side table entry of a point (LDS, indexed by point): interval half-width in
// key quanta (15 bits) and the sign bit set when the point was folded
// (delta = +1).
constexpr uint32_t kSideNeg = 0x8000u;
constexpr int kRqMax = 4096;    // larger radius: re-check in float64
constexpr int kClusterMax = 64; // larger uncertain run: defer to the exact tier

struct FiltCtx {
    const double* x64;  // this query's float64 points (AoS)
    const float* nrm;
    float fscale;       // filter scale
    int idx_bits;
};

template <int P>
__device__ __forceinline__ void fp64_point(const double* x64, const double (&e1)[P], const double (&e2)[P],
                                           int idx, double& y1, double& y2) {
    y1 = 0.0;
    y2 = 0.0;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        const double v = x64[(size_t)idx * P + c];
        y1 = fma(e1[c], v, y1);
        y2 = fma(e2[c], v, y2);
    }
}

// Float64 key and radius of a point (in the pseudo-angle t' = t + 1 in [0,2]);
// returns false if the fold or the magnitude is not certified.
__device__ __forceinline__ bool key64(double y1, double y2, double eps, bool& pos, double& t, double& r) {
    if (!(fabs(y1) > eps)) return false;
    pos = y1 > 0.0;
    const double h1 = fabs(y1);
    const double h2 = pos ? y2 : -y2;
    const double s = h1 + fabs(h2);
    if (!(s > 4.0 * eps)) return false;
    t = h2 / s + 1.0;
    r = eps / (s - 2.0 * eps) * 1.001 + 4.0 * kU64;
    return true;
}

// Lower end of a key interval [q - rq, q + rq] in quanta, clamped at 0 (a
// lower end taken lower only widens the interval).
__device__ __forceinline__ uint32_t lower_end(uint32_t q, uint32_t rq) { return q > rq ? q - rq : 0u; }

// Float64 interval [lo, lo + w] holding [t - r, t + r], for the re-ordering of
// uncertain runs: with r' = r + 8 u64 and t in [0, 2], lo = fl(t - r') errs
// by at most 2 u64 and stays below t - r; w = 2 r' rounded up to float32, and
// fl(lo + w) stays above t + r.
__device__ __forceinline__ void interval64(double t, double r, double& lo, float& w) {
    const double rr = r + 8.0 * kU64;
    lo = t - rr;
    w = (float)(2.0 * rr * 1.0000001) + 1e-30f;
}

template <int P, int K>
__device__ int sweep_filt(const float (&xr)[K][P], const SlotFilt<P>& S,
                          const SlotF64<P>& S64, int nnz, const FiltCtx& fc, uint16_t* side, const Staging& sg,
                          unsigned long long& rechecks) {
    uint32_t* pkey = sg.pkey;
    int* pS = sg.pS;
    uint8_t* pflag = sg.pflag;
    double* rt = sg.rt;
    float* rr = sg.rr;
    constexpr int KS = P - 2;
    const int lane = lane_id();
    const int ib = fc.idx_bits;
    const uint32_t imask = (1u << ib) - 1u;
    const int B = 32 - ib;
    const double qscale = (double)(1u << (B - 1));
    const float qscalef = (float)qscale;
    const uint32_t qmax = (1u << B) - 2u;   // keeps every real key below the pad value
    // float32 basis and error coefficient in registers; the float64 basis is
    // read from LDS only by the rare re-checks
    float f1[P], f2[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
        f1[c] = unif(S.f1[c]);
        f2[c] = unif(S.f2[c]);
    }
    int mem[KS > 0 ? KS : 1];
#pragma unroll
    for (int c = 0; c < KS; ++c) mem[c] = uni(S.mem[c]);
    const float beta = unif(S.beta32 * fc.fscale);
    // rounding of t' (8 u32) and truncation (4 quanta), scaled with the
    // filter: none at a filter scale of 0 (negative control)
    const float r8 = unif(8.0f * kU32 * fc.fscale);
    const uint32_t rpad = fc.fscale > 0.0f ? 4u : 0u;
    uint32_t key[K];
    int nplus = 0;
    uint32_t weak = 0;   // points whose float32 key is not certified
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int idx = lane * K + i;
        bool valid = idx < nnz;
#pragma unroll
        for (int c = 0; c < KS; ++c) valid = valid && (idx != mem[c]);
        float y1 = 0.0f, y2 = 0.0f;
#pragma unroll
        for (int c = 0; c < P; ++c) {
            y1 = fmaf(f1[c], xr[i][c], y1);
            y2 = fmaf(f2[c], xr[i][c], y2);
        }
        // Fold into {h1 > 0} U {h1 = 0, h2 > 0} by the sign of the first
        // coordinate; pseudo-angle t' = h2 / (h1 + |h2|) + 1 in (0, 2], which
        // is strictly increasing with the angle on that half-plane.  With the
        // float32 error eps of each coordinate the key error is at most
        // eps / (s - 2 eps) plus the rounding of t' (Algorithm 2, Step 1(b)).
        // Branch-free: invalid and uncertain points are masked afterwards.
        const float eps = beta;
        const bool pos = y1 > 0.0f;
        const float h1 = fabsf(y1);
        const float h2 = pos ? y2 : -y2;
        const float s = h1 + fabsf(h2);
        // hardware reciprocals are within 1 ulp: covered by the 8 u32 term
        // and the factor 1.001
        const float t = h2 * __builtin_amdgcn_rcpf(s) + 1.0f;
        const float r = eps * __builtin_amdgcn_rcpf(s - 2.0f * eps) * 1.001f + r8;
        const float rqf = r * qscalef;
        const bool ok = (h1 > eps) && (s > 4.0f * eps) && (rqf < (float)kRqMax);
        const uint32_t q = min((uint32_t)(t * qscalef), qmax);
        const uint32_t rq = ok ? (uint32_t)rqf + rpad : 0u;
        // idx < M always: the side entry of a point that is not swept is
        // written but never read
        side[idx] = (uint16_t)(rq | (pos ? 0u : kSideNeg));
        // the sort key is the interval's lower end (clamped at 0, which only
        // widens the interval), so that a lower end above every earlier upper
        // end is a strict gap of the exact order
        key[i] = (valid && ok) ? ((lower_end(q, rq) << ib) | (uint32_t)idx) : 0xffffffffu;
        weak |= (valid && !ok) ? (1u << i) : 0u;
        nplus += (valid && ok && pos) ? 1 : 0;
    }
    int defer = 0;
    if (__any(weak != 0)) {
        // float32 cannot settle the fold or the angle: float64 re-check.  The
        // loop is kept rolled (rare path); new keys go through the staging
        // array so that no register array is indexed dynamically.
        uint32_t* wk = sg.pkey + lane * K;
#pragma unroll 1
        for (int i = 0; i < K; ++i) {
            if (!((weak >> i) & 1u)) continue;
            const int idx = lane * K + i;
            ++rechecks;
            double d1, d2, t, r;
            bool pos;
            fp64_point<P>(fc.x64, S64.e1, S64.e2, idx, d1, d2);
            const double eps64 = S64.beta64 * (double)fc.nrm[idx];
            if (key64(d1, d2, eps64, pos, t, r) && r * qscale < (double)kRqMax) {
                const uint32_t q = min((uint32_t)(t * qscale), qmax);
                const uint32_t rq = (uint32_t)(r * qscale) + 4u;
                wk[i] = (lower_end(q, rq) << ib) | (uint32_t)idx;
                side[idx] = (uint16_t)(rq | (pos ? 0u : kSideNeg));
                nplus += pos ? 1 : 0;
            } else {
                defer = 1;
            }
        }
        if (__any(defer)) return kDefer;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if ((weak >> i) & 1u) key[i] = wk[i];
    }
    __syncthreads();   // side table visible to every lane
    wave_sort<K>(key);
    const int m = nnz - KS;
    const int S0 = wave_sum(nplus);
    // Pass 1: per-lane sum of delta and max of the interval ends (upper end
    // = lower end + 2 rq).
    int loc = 0, lmax = -kBig;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const bool real = key[i] != 0xffffffffu;
        const uint32_t sd = side[key[i] & imask];   // in bounds for pads too
        loc += real ? ((sd & kSideNeg) ? 1 : -1) : 0;
        lmax = real ? max(lmax, (int)(key[i] >> ib) + 2 * (int)(sd & 0x7fffu)) : lmax;
    }
    const int pm0 = wave_excl_max(lmax, -kBig);
    const int s0 = S0 + wave_excl_sum(loc);
    // Pass 2: cluster starts, states after each element, and runs holding
    // both fold signs.  The keys are sorted by lower end, so an element whose
    // lower end exceeds every earlier upper end starts a cluster: every later
    // interval starts above it too, and the boundary is a strict gap of the
    // exact order.  The state after element e is legitimate when e ends a
    // cluster, i.e. when the next element starts one (checked one element
    // late).
    int pm = pm0, s = s0;
    uint32_t startm = 0, mixm = 0;
    int best = (lane == 0) ? fside(S0, m) : kBig;
    int prev_s = 0;
    bool prev_real = false;
    // delta of the element before this lane's first one
    int dl_before;
    {
        const uint32_t sdl = side[key[K - 1] & imask];
        const int dl_last_lane = (key[K - 1] != 0xffffffffu) ? ((sdl & kSideNeg) ? 1 : -1) : 0;
        dl_before = lane_prev(dl_last_lane, 0);
    }
    int dp = dl_before;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const bool real = key[i] != 0xffffffffu;
        const uint32_t sd = side[key[i] & imask];
        const int rq = (int)(sd & 0x7fffu);
        const int qv = (int)(key[i] >> ib);
        const int dl = real ? ((sd & kSideNeg) ? 1 : -1) : 0;
        const int lo = real ? qv : kBig;
        const int hi = real ? qv + 2 * rq : -kBig;
        const bool st = real && lo > pm;
        pm = max(pm, hi);
        if (st) startm |= 1u << i;
        if (real && !st && dl != dp) mixm |= 1u << i;
        // the previous element ends a cluster if this one starts one or is a pad
        if (i > 0 && prev_real && (st || !real)) best = min(best, fside(prev_s, m));
        s += dl;
        prev_s = s;
        prev_real = real;
        dp = dl;
    }
    {
        // last element of the lane: look at the next lane's first element
        const int nstart = lane_next((int)(startm & 1u), 0);
        const int nreal = lane_next((int)(key[0] != 0xffffffffu), 0);
        const bool ends = (lane == 63) || nstart || !nreal;
        if (prev_real && ends) best = min(best, fside(prev_s, m));
    }
    if (__any(mixm != 0)) {
        // Runs of overlapping key intervals that hold both fold signs: their
        // inner order matters.  Stage the sorted sequence in LDS; the lane
        // holding the first mixed position of a run re-orders the run with
        // float64 keys and evaluates the states between certified gaps.
        int ss = s0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int e = lane * K + i;
            int dl = 0;
            if (key[i] != 0xffffffffu) dl = (side[key[i] & imask] & kSideNeg) ? 1 : -1;
            ss += dl;
            pkey[e] = key[i];
            pS[e] = ss;
            pflag[e] = (uint8_t)(((startm >> i) & 1u) | (((mixm >> i) & 1u) << 1));
        }
        __syncthreads();
#pragma unroll 1
        for (int i = 0; i < K; ++i) {
            if (!((mixm >> i) & 1u)) continue;
            const int e = lane * K + i;
            int a = e - 1;
            bool first = true;
            while (!(pflag[a] & 1)) {
                if (pflag[a] & 2) { first = false; break; }
                --a;
            }
            if (!first) continue;
            int b = e;
            while (b + 1 < m && !(pflag[b + 1] & 1)) ++b;
            const int c = b - a + 1;
            if (c > kClusterMax) { defer = 1; continue; }
            // float64 intervals of the run, insertion-sorted by lower end in
            // place at the run's own positions of the LDS staging arrays (runs
            // are disjoint)
            bool ok = true;
            for (int u = 0; u < c; ++u) {
                const uint32_t kv = pkey[a + u];
                const int idx = (int)(kv & imask);
                double d1, d2, t, r;
                bool pos;
                fp64_point<P>(fc.x64, S64.e1, S64.e2, idx, d1, d2);
                const double eps64 = S64.beta64 * (double)fc.nrm[idx];
                if (!key64(d1, d2, eps64, pos, t, r)) { ok = false; break; }
                double lo;
                float wd;
                interval64(t, r, lo, wd);
                int w = u;
                while (w > 0 && rt[a + w - 1] > lo) {
                    rt[a + w] = rt[a + w - 1];
                    rr[a + w] = rr[a + w - 1];
                    --w;
                }
                rt[a + w] = lo;
                rr[a + w] = pos ? wd : -wd;   // width; the sign carries the fold
            }
            rechecks += (unsigned long long)c;
            if (!ok) { defer = 1; continue; }
            int sc = (a == 0) ? S0 : pS[a - 1];
            double mhi = rt[a] + (double)fabsf(rr[a]);
            int hasp = rr[a] < 0.0f, hasn = rr[a] > 0.0f;
            sc += (rr[a] < 0.0f) ? 1 : -1;
            for (int u = 1; u < c; ++u) {
                const double tu = rt[a + u];
                const float ru = rr[a + u];
                if (tu > mhi) {
                    // certified gap between u-1 and u: a legitimate state
                    if (hasp && hasn) { ok = false; break; }
                    best = min(best, fside(sc, m));
                    hasp = hasn = 0;
                }
                hasp |= ru < 0.0f;
                hasn |= ru > 0.0f;
                mhi = fmax(mhi, tu + (double)fabsf(ru));   // upper end
                sc += (ru < 0.0f) ? 1 : -1;
            }
            if (!ok || (hasp && hasn)) defer = 1;
        }
        __syncthreads();
        if (__any(defer)) return kDefer;
    }
    return wave_min(best);
}

// ---------------------------------------------------------------- bucketed
// The sweep only needs the states where min(S, m - S) can be smallest, so the
// angular order is taken at bucket granularity first (a counting sort by
// pseudo-angle) and refined exactly only where the minimum may lie.
//
// Keys: t' in [0, 2] maps to q = t' QS + W in quanta, q in [W, (NB - 1) W],
// with NB buckets (M/8, 64 or 128) of W = 2^16 quanta.  The float32 path
// forms q as the float 2^23 + q, whose bit pattern is the integer
// 0x4B000000 + q (one binade, unit spacing): the interval ends need no
// float-to-integer conversion, and a bucket index is byte 2 of those bits
// (one byte-select).  Every point carries a certified interval [lo, hi]
// (hi - lo < W / 2) that contains the key of the exact frame, so a bucket
// boundary that no interval crosses is a strict gap of the angular order, and
// the state there is a state of the sweep.  Bucket word (LDS): bits 0-10 points folded with delta = -1, bits
// 11-21 points with delta = +1 (counted by the bucket of the interval's lower
// end), bits 22-31 points whose interval crosses into the next bucket.
//
// With S_j the state at the left boundary of bucket j (by counts), the states
// reachable inside the bucket lie in [S_j - pos_j - c_j, S_j + neg_j + c_j],
// c_j the points crossing in from bucket j-1.  U = min of min(S, m - S) over
// boundaries that no interval crosses (real states), L = min over buckets of
// the range bound; L <= b_I <= U.  When L = U the sweep is done; otherwise the
// runs of buckets (between uncrossed boundaries) whose range dips below U are
// gathered and walked in exact order from the state at their left boundary.
constexpr uint32_t kHistPos = 1u;
constexpr uint32_t kHistNeg = 1u << 11;
constexpr uint32_t kHistStr = 1u << 22;
constexpr uint32_t kAuxNeg = 1u << 31;
constexpr int kListMax = 128;   // gathered points of the runs walked exactly
// Key of a point that is not swept (padding, a member of I, or a point float64
// cannot place): byte 2 of its lower end is 255, a histogram word past the NB
// buckets (the histogram holds 256 words, and the scan reads only the first
// NB).
constexpr uint32_t kKeyOut = 0xffffffffu;
// Bits of the float 2^23: key bits = kKeyBias + q for q in [0, 2^23).
constexpr uint32_t kKeyBias = 0x4B000000u;
// Histogram word of a key's lower-end bits.
__device__ __forceinline__ uint32_t key_bucket(uint32_t bits) { return (bits >> 16) & 0xffu; }

// Buckets per lane: an eighth of the points per lane (about eight points per
// bucket).  The bounds L and U only decide when a sweep must be walked in
// exact order, and with the running-minimum bound that is rare, so fewer,
// wider buckets cost little there and shorten the scan (measured on p = 5,
// n = 500: M/8 buckets walk twice as often as M/4 and are 2% faster; M/2
// is 5% slower than M/4).
// Twelve points per lane round up to two buckets: one bucket of twelve made
// the walks gather more than the list holds, which sent those sweeps to the
// exact tier.
template <int K>
constexpr int buckets_per_lane() { return K >= 8 ? (K + 7) / 8 : 1; }

template <int K>
struct BucketGeom {
    static constexpr int NBL = buckets_per_lane<K>();
    static constexpr int NB = 64 * NBL;
    static constexpr int SH = 16;
    static constexpr int HW = 256;              // histogram words (byte 2 of a key)
    static constexpr uint32_t W = 1u << SH;
    static constexpr double QS = (double)(NB - 2) * (double)W / 2.0;   // quanta per unit of t'
    static constexpr double QB = QS + (double)W;                        // q at t' = 1
    static constexpr uint32_t RQMAX = W / 4;
    // b = 4 eps / s below which a key radius passes the RQMAX check
    static constexpr double BCAP = 4.0 * (double)RQMAX / QS;
    static_assert((uint64_t)NB * W <= (1ull << 23), "keys stay in the binade [2^23, 2^24)");
    static_assert(NB <= 128 && HW >= NB + 64, "words of the lanes' uncertified keys past the buckets");
};

// float64 key of a point in bucket quanta: the bits of its interval's lower
// end (kKeyBias + q - rq) and the interval's width 2 rq with the fold bit;
// false if not certified
template <int K>
__device__ __forceinline__ bool bucket_key64(double d1, double d2, double eps64, uint32_t& lo, uint32_t& aux) {
    using G = BucketGeom<K>;
    double t, r;
    bool pos;
    if (!key64(d1, d2, eps64, pos, t, r)) return false;
    const double rqd = r * G::QS;
    if (!(rqd < (double)(G::RQMAX - 4))) return false;
    // t' = t in [0, 2]: q = (t - 1) QS + QS + W
    const uint32_t q = (uint32_t)(t * G::QS + (double)G::W);
    const uint32_t rq = (uint32_t)rqd + 2u;
    lo = kKeyBias + q - rq;
    aux = (2u * rq) | (pos ? 0u : kAuxNeg);
    return true;
}

// Float32 key of one point for the bucketed sweep: projection on (e1, e2),
// fold by the sign of the first coordinate, pseudo-angle
// t' = h2 / (h1 + |h2|) + 1 in bucket quanta, and its interval: the bits lo,
// hi of the floats 2^23 + q -+ r.  With eps the
// float32 error of each coordinate and a = eps / s <= 1/4 (from h1 > 4 eps),
// the key moves by at most eps / (s - 2 eps) = a / (1 - 2a) <= a + 4a^2 =
// (b + b^2) / 4 with b = 4a.  A radius that passes the check has b < BCAP, so
// b^2 < BCAP b and the linear bound b (1 + BCAP) / 4 covers it; 8 u32 covers
// the rounding of t' (hardware reciprocal within 1 ulp) and of the scaling to
// quanta, 2 quanta the roundings of 2^23 + q and of its sum and difference
// with the radius (half a quantum each: unit spacing in that binade)
// (Algorithm 2, Step 1(b)).  Returns whether the fold and the key are
// certified.  Contraction is off, so every evaluation of a point gives the
// same bits.
template <int P, int K>
__device__ __forceinline__ bool key32(const float (&x)[P], const float (&f1)[P], const float (&f2)[P], float eps4,
                                      float eR, float eC, uint32_t& lo, uint32_t& hi, bool& pos) {
#pragma clang fp contract(off)
    using G = BucketGeom<K>;
    const float QSf = (float)G::QS;
    const float QBf = (float)(G::QB + 8388608.0);   // 2^23 + q at t' = 1, exact
    float y1 = 0.0f, y2 = 0.0f;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        y1 = fmaf(f1[c], x[c], y1);
        y2 = fmaf(f2[c], x[c], y2);
    }
    pos = y1 > 0.0f;
    const float ay1 = fabsf(y1);
    const float h2 = pos ? y2 : -y2;
    const float s = ay1 + fabsf(h2);
    const float rs = __builtin_amdgcn_rcpf(s);
    const float u = h2 * rs;
    // b RQS with b = eps4 / s, as rs (eps4 RQS), plus eC = 8 u32 QS + 2
    // quanta for the roundings
    const float rqf = fmaf(rs, eR, eC);
    const float Q = fmaf(u, QSf, QBf);
    // meaningful only when the key is certified: then both ends stay in the
    // binade [2^23, 2^24), where the bits grow with the value
    lo = __float_as_uint(Q - rqf);
    hi = __float_as_uint(Q + rqf);
    return (ay1 > eps4) && (rqf < (float)(G::RQMAX - 4));
}

// Histogram add of a key interval [lo, hi] (bits) that may be uncertified
// (ok false): such a point takes the lane's own word past the buckets, and a
// point that float64 cannot place either (lo = kKeyOut) the word 255 (the
// words past NB are never read).  The crossing count field is 1 when the
// interval ends in the next bucket.
__device__ __forceinline__ void hist_add32(uint32_t* hist, uint32_t lo, uint32_t hi, bool pos, bool ok, uint32_t out_lo) {
    const uint32_t blo = key_bucket(ok ? lo : out_lo);
    const uint32_t inc = (pos ? kHistPos : kHistNeg) | ((key_bucket(hi) - blo) << 22);
    atomicAdd(&hist[blo], inc);
}

// A zero made in a vector register where it is used (a volatile move the
// compiler cannot hoist): the histogram clears otherwise read a zero pair
// that the register allocator keeps in scratch memory at 14 points per lane,
// one scratch load and a full memory wait per sweep.
__device__ __forceinline__ uint32_t vzero() {
    uint32_t z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return z;
}

// Inclusive sum over the lanes of the same segment (segments are contiguous
// runs of lanes with equal `seg`): the rare walk's scans.
__device__ __forceinline__ int seg_incl_sum(int v, int seg) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int vv = __shfl_up(v, d, 64);
        const int gg = __shfl_up(seg, d, 64);
        if (lane >= d && gg == seg) v += vv;
    }
    return v;
}

// Exclusive prefix maximum over the lanes (lane 0 reads `id`).
__device__ __forceinline__ int excl_max_shfl(int v, int id) {
    const int lane = lane_id();
    int m = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int vv = __shfl_up(m, d, 64);
        if (lane >= d) m = max(m, vv);
    }
    const int prev = __shfl_up(m, 1, 64);
    return lane == 0 ? id : prev;
}

// The walk of the first pass (no float64 code), over the gathered points
// sorted by the lower ends of their key intervals (at most 128: entry e in
// lane e % 64 of half e / 64).  The same clusters as the one-lane walk of
// the float64 pass, decided in parallel: an entry starts a cluster when it
// starts a run or its lower end lies above every upper end before it in its
// run; the state after an entry is its run's left-boundary state plus the
// +1 / -1 of the entries of the run up to it.  The states after the clusters
// hold for any order inside the clusters, and their minimum `best` bounds
// every cluster's inner states from above, so a cluster with both fold
// signs needs an exact inner order only if its states could go below
// min(U, ubound, best).  Returns min(U, best), or kNeed64 (kDefer for a
// cluster above kClusterMax) when some cluster needs its inner order.
__device__ __forceinline__ int walk_lean(const uint4* list, int gtot, int m, int U, int ubound) {
    const int lane = lane_id();
    constexpr int kNoRun = 0x7fff;
    int run[2], srun[2], comb[2], delta[2], pos[2];
    uint32_t lo[2];
    bool in[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = lane + 64 * h;
        in[h] = e < gtot;
        const uint4 v = in[h] ? list[e] : make_uint4(0u, 0u, 0u, 0u);
        run[h] = in[h] ? (int)(v.z >> 11) : kNoRun;
        srun[h] = (int)(v.z & 0x7ffu);
        lo[h] = v.x;
        const uint32_t hi = v.x + (v.y & 0x7fffffffu);
        pos[h] = (in[h] && !(v.y & kAuxNeg)) ? 1 : 0;
        delta[h] = in[h] ? (pos[h] ? -1 : 1) : 0;
        // run and upper end in one key that grows along the sorted list
        // (runs in increasing order; upper ends below 2^24 in the binade)
        comb[h] = in[h] ? (run[h] << 23) | (int)(hi - kKeyBias) : -1;
    }
    // cluster starts
    bool start[2];
    {
        const int m0 = __builtin_amdgcn_readlane(wave_incl_max_dpp(comb[0]), 63);
        const int ex0 = excl_max_shfl(comb[0], -1);
        const int ex1 = max(excl_max_shfl(comb[1], -1), m0);
        const int ex[2] = {ex0, ex1};
#pragma unroll
        for (int h = 0; h < 2; ++h)
            start[h] = in[h] && (ex[h] < 0 || (ex[h] >> 23) != run[h] ||
                                 lo[h] > (uint32_t)(ex[h] & 0x7fffff) + kKeyBias);
    }
    // cluster ids (global count of starts up to the entry)
    int cid[2];
    cid[0] = wave_incl_sum_dpp(start[0] ? 1 : 0);
    cid[1] = __builtin_amdgcn_readlane(cid[0], 63) + wave_incl_sum_dpp(start[1] ? 1 : 0);
    if (!in[0]) cid[0] = -1 - lane;
    if (!in[1]) cid[1] = -1000 - lane;
    // states after the entries (sums over the run), and counts and positive
    // points of the cluster up to the entry; the second half continues the
    // segment of the first half's last entry
    int send[2], cnt[2], np[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        send[h] = seg_incl_sum(delta[h], run[h]);
        cnt[h] = seg_incl_sum(in[h] ? 1 : 0, cid[h]);
        np[h] = seg_incl_sum(pos[h], cid[h]);
    }
    {
        const int r63 = __builtin_amdgcn_readlane(run[0], 63);
        const int s63 = __builtin_amdgcn_readlane(send[0], 63);
        const int c63 = __builtin_amdgcn_readlane(cid[0], 63);
        const int n63 = __builtin_amdgcn_readlane(cnt[0], 63);
        const int p63 = __builtin_amdgcn_readlane(np[0], 63);
        if (in[1] && run[1] == r63) send[1] += s63;
        if (in[1] && cid[1] == c63) {
            cnt[1] += n63;
            np[1] += p63;
        }
    }
    // cluster ends: the last entry, or one followed by a start
    bool end[2];
    {
        const int sb0 = __builtin_amdgcn_readlane(start[1] ? 1 : 0, 0);
        const int nx0 = __shfl_down(start[0] ? 1 : 0, 1, 64);
        const int nx1 = __shfl_down(start[1] ? 1 : 0, 1, 64);
        end[0] = in[0] && (lane + 1 == gtot || (lane < 63 ? nx0 != 0 : sb0 != 0));
        end[1] = in[1] && (lane + 65 == gtot || (lane < 63 && nx1 != 0));
    }
    int best = kBig;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        send[h] += srun[h];
        if (end[h]) best = min(best, fside(send[h], m));
    }
    best = wave_min(best);
    const int bound = min(min(U, ubound), best);
    bool need = false, big = false;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (!end[h]) continue;
        const int c = cnt[h], npc = np[h];
        if (npc == 0 || npc == c) continue;   // one fold sign: any order
        const int s0 = send[h] - (c - 2 * npc);   // state before the cluster
        const int dip = min(s0 - npc, m - (s0 + (c - npc)));
        if (dip < bound) {
            need = true;
            big = big || c > kClusterMax;
        }
    }
    if (__any(big)) return kDefer;
    if (__any(need)) return kNeed64;
    return min(U, best);
}

// F64 = false: the sweep without any float64 code (its registers cost the
// kernel's loop about 12% at p = 5 even where it never runs): where float64
// is needed it returns kNeed64.  F64 = true: the same sweep with the float64
// re-check of uncertified points and the float64 re-order of mixed clusters
// (the float64 pass of the subset kernel).
template <int P, int K, bool F64>
__device__ __forceinline__ int sweep_bucket(const float (&xr)[K][P], const SlotFilt<P>& S, const SlotF64<P>& S64,
                                            int nnz, const FiltCtx& fc, uint32_t* hist, uint4* list,
                                            const Staging& sg, int ubound, unsigned long long& rechecks,
                                            unsigned long long& walked) {
    using G = BucketGeom<K>;
    constexpr int KS = P - 2;
    constexpr int NB = G::NB;
    constexpr int NBL = G::NBL;
    const int lane = lane_id();
    // basis rows as read from LDS (every lane reads the same words), kept in
    // vector registers: no lane-to-scalar moves per sweep
    float f1[P], f2[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
        f1[c] = S.f1[c];
        f2[c] = S.f2[c];
    }
    // 4 eps, eps the float32 error of each coordinate of a unit-length point
    const float eps4 = unif(4.0f * S.beta32 * fc.fscale);
    // eps4 times the quanta per unit of b = 4 eps / s in the linear radius bound
    const float eR = eps4 * (float)(G::QS * (1.001 / 4.0) * (1.0 + G::BCAP));
    // quanta for the roundings of t' and of the scaling (8 u32 QS) and the
    // truncations (2); scaled with the filter like the error term, so that a
    // filter scale of 0 leaves no margin at all (negative control)
    const float eC = unif((8.0f * kU32 * (float)G::QS + 2.0f) * fc.fscale);
    // Keys and histogram in one pass; the keys are not kept: the rare walk
    // evaluates them again.  Points float32 cannot certify are re-checked in
    // float64 below and keep their keys in the staging arrays.
    // The members of I lie in span(x_I): their float32 coordinates are within
    // the error bound of 0, so they never pass the key check and are left out
    // like every other point that fails it.
    // Padding rows past nnz are zero and fail the key check too.  A point
    // that fails it adds to the word 128 + lane, past the buckets.
    const uint32_t out_lo = (128u + (uint32_t)lane) << 16;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        uint32_t lo, hi;
        bool pos;
        const bool ok = key32<P, K>(xr[i], f1, f2, eps4, eR, eC, lo, hi, pos);
        hist_add32(hist, lo, hi, pos, ok, out_lo);
    }
    __syncthreads();
    // totals of the lane's NBL buckets [lane NBL, lane NBL + NBL) and of the
    // sweep: m points placed, S0 of them with delta = -1
    uint32_t w[NBL];
    uint32_t tl;
    int incl, tot;
    auto totals = [&]() {
#pragma unroll
        for (int j = 0; j < NBL; ++j) w[j] = hist[lane * NBL + j];
        tl = 0;
#pragma unroll
        for (int j = 0; j < NBL; ++j) tl += w[j];
        tl &= 0x3fffffu;   // per-field sums stay below 2^11: no carry between fields
        incl = wave_incl_sum_dpp((int)tl);
        tot = __builtin_amdgcn_readlane(incl, 63);
    };
    totals();
    // Every point outside I and below nnz that float32 placed is counted; if
    // fewer than nnz - |I| are, some need the float64 re-check (F64 only:
    // otherwise the missing points are left out, as below).  Points that
    // float64 cannot place either (near the fold line, or inside span(x_I))
    // are left out of the sweep; `partial` records it.  Leaving points out
    // lowers every count, and delta_I >= 0, so the bounds of the remaining
    // points still bound delta_I + b_I from below.
    bool partial = false;
    uint32_t* wq = sg.pkey + lane * K;
    int* wa = sg.pS + lane * K;
    uint32_t weak = 0;
    const bool short32 = (tot & 0x7ff) + ((tot >> 11) & 0x7ff) < nnz - KS;
    if (!F64) {
        partial = short32;
    } else if (short32) {
        // which points: the same evaluation again (from an opaque copy of
        // eps4, so that the compiler does not keep the first evaluation's
        // values live instead); then a float64 re-check with the keys kept in
        // the staging arrays (rolled loop, rare path)
        float eps4r = eps4;
        int mem[KS > 0 ? KS : 1];
#pragma unroll
        for (int c = 0; c < KS; ++c) mem[c] = uni(S.mem[c]);
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int idx = lane * K + i;
            bool valid = idx < nnz;
#pragma unroll
            for (int c = 0; c < KS; ++c) valid = valid && (idx != mem[c]);
            uint32_t lo, hi;
            bool pos;
            const bool ok = key32<P, K>(xr[i], f1, f2, eps4r, eR, eC, lo, hi, pos);
            weak |= (valid && !ok) ? (1u << i) : 0u;
        }
        uint32_t lost = 0;
#pragma unroll 1
        for (int i = 0; i < K; ++i) {
            if (!((weak >> i) & 1u)) continue;
            const int idx = lane * K + i;
            ++rechecks;
            double d1, d2;
            fp64_point<P>(fc.x64, S64.e1, S64.e2, idx, d1, d2);
            uint32_t lo2, a2;
            if (!bucket_key64<K>(d1, d2, S64.beta64 * (double)fc.nrm[idx], lo2, a2)) {
                lo2 = kKeyOut;
                a2 = 0u;
                lost |= 1u << i;
            }
            wq[i] = lo2;
            wa[i] = (int)a2;
            hist_add32(hist, lo2, lo2 + (a2 & 0x7fffffffu), !(a2 & kAuxNeg), true, 0u);
        }
        partial = __any(lost != 0);
        __syncthreads();
        totals();
    }
#pragma unroll
    for (int j = 0; j < NBL; ++j) hist[lane * NBL + j] = vzero();
    const int pre = incl - (int)tl;
    const int S0 = tot & 0x7ff;
    const int m = S0 + ((tot >> 11) & 0x7ff);
    const int Sst = S0 - (pre & 0x7ff) + ((pre >> 11) & 0x7ff);
    // crossings into this lane's first bucket: the previous lane's last
    // bucket (DPP wave_shr:1; lane 0 reads 0)
    const int cin = lane_prev((int)(w[NBL - 1] >> 22), 0);
    int U = kBig, L = kBig;
    {
        int s = Sst;
#pragma unroll
        for (int j = 0; j < NBL; ++j) {
            const int np = (int)(w[j] & 0x7ffu);
            const int nn = (int)((w[j] >> 11) & 0x7ffu);
            const int c = (j == 0) ? cin : (int)(w[j - 1] >> 22);
            if (c == 0) U = min(U, fside(s, m));
            L = min(L, min(s - np - c, m - (s + nn + c)));
            s += nn - np;
        }
    }
    // When L is not below `ubound` (a term the query already reached, or the
    // bound from the directions +-x_j), no state of this sweep can lower the
    // minimum over subsets: the subset is not needed (the caller records the
    // bound for it).  This holds with points left out too, since leaving
    // points out only lowers the states; otherwise such a sweep goes to the
    // exact tier.  Every lane's bound reaching `ubound` is a wave vote; the
    // minimum itself is reduced only when it is needed.
    if (__all(L >= ubound)) return kSkip;
    if (partial) return F64 ? kDefer : kNeed64;
    L = wave_min_dpp(L);
    // Done when L = U.
    U = wave_min_dpp(U);
    if (L >= U) return U;
    ++walked;

    // ---- rare: walk the runs whose range dips below U in exact order.
    // Run info per bucket: (first bucket of its run << 11) | state at the
    // run's left boundary; bit 31 of a run's first entry marks it for the walk.
    int loc[NBL];
    uint32_t hot = 0;
    int last = -1;
    {
        int s = Sst;
#pragma unroll
        for (int j = 0; j < NBL; ++j) {
            const int np = (int)(w[j] & 0x7ffu);
            const int nn = (int)((w[j] >> 11) & 0x7ffu);
            const int c = (j == 0) ? cin : (int)(w[j - 1] >> 22);
            if (c == 0) last = ((lane * NBL + j) << 11) | s;
            loc[j] = last;
            if (min(s - np - c, m - (s + nn + c)) < U) hot |= 1u << j;
            s += nn - np;
        }
    }
    {
        const int carry = wave_excl_max(last, -1);   // bucket 0 starts a run: carry >= 0 where needed
#pragma unroll
        for (int j = 0; j < NBL; ++j)
            if (loc[j] < 0) loc[j] = carry;
    }
#pragma unroll
    for (int j = 0; j < NBL; ++j) hist[lane * NBL + j] = (uint32_t)loc[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NBL; ++j)
        if ((hot >> j) & 1u) atomicOr(&hist[(loc[j] >> 11) & (NB - 1)], 0x80000000u);
    __syncthreads();
    uint32_t gm = 0;
    int cnt = 0;
    uint32_t qk[K], aux[K], rinf[K];
    int mem[KS > 0 ? KS : 1];
#pragma unroll
    for (int c = 0; c < KS; ++c) mem[c] = uni(S.mem[c]);
    float eps4w = eps4;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        // the same keys as the histogram's: float32 again, or the float64
        // re-check's from the staging arrays; qk: bits of the interval's
        // lower end, aux: its width and the fold
        if ((weak >> i) & 1u) {
            qk[i] = wq[i];
            aux[i] = (uint32_t)wa[i];
        } else {
            const int idx = lane * K + i;
            bool valid = idx < nnz;
#pragma unroll
            for (int c = 0; c < KS; ++c) valid = valid && (idx != mem[c]);
            uint32_t lo, hi;
            bool pos;
            const bool ok = key32<P, K>(xr[i], f1, f2, eps4w, eR, eC, lo, hi, pos);
            qk[i] = (valid && ok) ? lo : kKeyOut;
            aux[i] = ((hi - lo) & 0x7fffffffu) | (pos ? 0u : kAuxNeg);
        }
        const uint32_t blo = key_bucket(qk[i]) & (NB - 1);
        const uint32_t ri = hist[blo] & 0x7fffffffu;
        rinf[i] = ri;
        const bool g = (qk[i] != kKeyOut) && (hist[(ri >> 11) & (NB - 1)] >> 31);
        gm |= g ? (1u << i) : 0u;
        cnt += g ? 1 : 0;
    }
    const int gincl = wave_incl_sum_dpp(cnt);
    const int gbase = gincl - cnt;
    const int gtot = __builtin_amdgcn_readlane(gincl, 63);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NBL; ++j) hist[lane * NBL + j] = vzero();
    if (gtot > kListMax) {
        __syncthreads();
        return kFallback;   // too many points to walk: the caller defers the subset
    }
    {
        int k = gbase;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if ((gm >> i) & 1u) {
                list[k] = make_uint4(qk[i], aux[i], rinf[i], (uint32_t)(lane * K + i));
                ++k;
            }
    }
    __syncthreads();
    // Order the gathered points by the lower ends of their intervals (runs are
    // separated by strict gaps, so this order keeps every run contiguous and
    // in order; inside a run, a lower end above every earlier upper end is a
    // strict gap): every lane ranks its two entries against the whole list,
    // equal keys by gathering position, and writes them to their ranks.
    {
        static_assert(kListMax <= 128, "two list entries per lane");
        const int j0 = lane, j1 = lane + 64;
        uint4 v0 = make_uint4(0u, 0u, 0u, 0u), v1 = v0;
        if (j0 < gtot) v0 = list[j0];
        if (j1 < gtot) v1 = list[j1];
        int r0 = 0, r1 = 0;
#pragma unroll 4
        for (int u = 0; u < gtot; ++u) {
            const uint32_t ku = list[u].x;
            r0 += (ku < v0.x || (ku == v0.x && u < j0)) ? 1 : 0;
            r1 += (ku < v1.x || (ku == v1.x && u < j1)) ? 1 : 0;
        }
        __syncthreads();
        if (j0 < gtot) list[r0] = v0;
        if (j1 < gtot) list[r1] = v1;
        __syncthreads();
    }
    if constexpr (!F64) {
        const int term = walk_lean(list, gtot, m, U, ubound);
        __syncthreads();
        return term;
    }
    int best = kBig, defer = 0;
    if (lane == 0) {
        // every entry is read from LDS once, as one 16-byte load: `nx` holds
        // the entry after the current cluster (zero past the end)
        const uint4 kNone = make_uint4(0u, 0u, 0u, 0u);
        uint4 nx = gtot > 0 ? list[0] : kNone;
        int k = 0;
#pragma unroll 1
        while (k < gtot && !defer) {
            const uint32_t run = nx.z >> 11;
            int s = (int)(nx.z & 0x7ffu);
            int a = k;
#pragma unroll 1
            while (a < gtot && (nx.z >> 11) == run && !defer) {
                // cluster: maximal run of overlapping intervals, with the
                // count of its positive-fold points
                const uint4 va = nx;
                uint32_t mhi = va.x + (va.y & 0x7fffffffu);   // upper end
                int npos_c = (va.y & kAuxNeg) ? 0 : 1;
                int b = a;
                nx = (b + 1 < gtot) ? list[b + 1] : kNone;
#pragma unroll 1
                while (b + 1 < gtot && (nx.z >> 11) == run && nx.x <= mhi) {
                    ++b;
                    mhi = max(mhi, nx.x + (nx.y & 0x7fffffffu));
                    npos_c += (nx.y & kAuxNeg) ? 0 : 1;
                    nx = (b + 1 < gtot) ? list[b + 1] : kNone;
                }
                const int c = b - a + 1;
                const int hp = npos_c > 0 ? 1 : 0, hn = npos_c < c ? 1 : 0;
                // states inside the run lie in [s - (pos in run), s + (neg in
                // run)]: if min(S, m - S) cannot go below the bound there, the
                // inner order does not matter
                const int dip = min(s - npos_c, m - (s + (c - npos_c)));
                const bool needed = dip < min(min(U, ubound), best);
                if (hp && hn && !needed) {
                    s += c - 2 * npos_c;
                } else if (hp && hn) {
                    // both fold signs inside uncertain order: float64 keys,
                    // insertion-sorted in the block's staging arrays (with the
                    // float64 basis only; otherwise the exact tier orders them)
                    if (c > kClusterMax) { defer = 1; break; }
                    if (!F64) { defer = 2; break; }
                    double* rt = sg.rt;
                    float* rr = sg.rr;
                    bool ok = true;
#pragma unroll 1
                    for (int u = 0; u < c; ++u) {
                        const int idx = (int)list[a + u].w;
                        double d1, d2, t, r;
                        bool pos;
                        fp64_point<P>(fc.x64, S64.e1, S64.e2, idx, d1, d2);
                        const double eps64 = S64.beta64 * (double)fc.nrm[idx];
                        if (!key64(d1, d2, eps64, pos, t, r)) { ok = false; break; }
                        double lo;
                        float wd;
                        interval64(t, r, lo, wd);
                        int v = u;
                        while (v > 0 && rt[v - 1] > lo) {
                            rt[v] = rt[v - 1];
                            rr[v] = rr[v - 1];
                            --v;
                        }
                        rt[v] = lo;
                        rr[v] = pos ? wd : -wd;
                    }
                    rechecks += (unsigned long long)c;
                    if (!ok) { defer = 1; break; }
                    // float64 sub-runs of overlapping intervals (sorted by lower
                    // end: a lower end above every earlier upper end is a
                    // strict gap); one that holds both signs is settled only
                    // if its states could go below the bound (then the subset
                    // goes to the exact tier)
                    double thi = rt[0] + (double)fabsf(rr[0]);
                    int s_sub = s, np_sub = 0, nn_sub = 0;
                    if (rr[0] < 0.0f) ++nn_sub; else ++np_sub;
                    s += (rr[0] < 0.0f) ? 1 : -1;
#pragma unroll 1
                    for (int u = 1; u < c; ++u) {
                        const double tu = rt[u];
                        const float ru = rr[u];
                        if (tu > thi) {
                            if (np_sub && nn_sub &&
                                min(s_sub - np_sub, m - (s_sub + nn_sub)) < min(min(U, ubound), best)) {
                                ok = false;
                                break;
                            }
                            best = min(best, fside(s, m));
                            s_sub = s;
                            np_sub = nn_sub = 0;
                        }
                        if (ru < 0.0f) ++nn_sub; else ++np_sub;
                        thi = fmax(thi, tu + (double)fabsf(ru));
                        s += (ru < 0.0f) ? 1 : -1;
                    }
                    if (ok && np_sub && nn_sub &&
                        min(s_sub - np_sub, m - (s_sub + nn_sub)) < min(min(U, ubound), best))
                        ok = false;
                    if (!ok) { defer = 1; break; }
                } else {
                    s += hn ? c : -c;
                }
                best = min(best, fside(s, m));
                a = b + 1;
            }
            k = a;
        }
    }
    __syncthreads();
    const int dv = __builtin_amdgcn_readfirstlane(defer);
    if (dv) return dv == 2 ? kNeed64 : kDefer;
    return min(U, __builtin_amdgcn_readfirstlane(best));
}

// ------------------------------------------------------------------ kernel
template <int P, int TIER>
struct SlotOf { using type = SlotFilt<P>; };
template <int P>
struct SlotOf<P, kPlain> { using type = SlotPlain<P>; };

template <int P>
__device__ __forceinline__ void push_deferred(const Pools& pl, int q, uint64_t rank) {
    const unsigned long long pos = atomicAdd(&pl.ctr->defer_next, 1ull);
    if (pos < pl.defer_cap) {
        Deferred d;
        d.query = (uint32_t)q;
        d.pad = 0;
        d.rank = rank;
        pl.deferred[pos] = d;
    } else {
        atomicOr(&pl.qs[q].status, kStDeferOverflow);
    }
}

// Waves per SIMD the register allocator is asked to fit for the bucketed
// sweep (more resident waves hide the LDS and DPP latencies of the sweep);
// chosen per instantiation so that no register spills land in the common
// path of the sweep (spills in the per-batch set-up and on the rare paths
// are accepted: at p <= 5, K = 8, four waves measured 7% faster than three
// and five 30% slower; at p <= 5, K = 16, three waves measured 11% faster than
// two on the batched workload although spills reach the sweep, and four
// twice as slow).
template <int P, int K, int TIER>
constexpr int min_waves() {
    if (TIER != kFiltBucket) return 1;
    if (K <= 8) {
        if (P <= 5) return 4;
        if (P == 6 && K <= 4) return 3;
        return P <= 7 ? 2 : 1;
    }
    if (P <= 5) return 3;
    return P <= 6 ? 2 : 1;
}

// REDO = false: the work items of the class in turn.  REDO = true (bucketed
// sweep, p >= 3): the float64 pass, which finishes the work items that the
// first pass handed over at a sweep that needed float64 (the float64 basis of
// every subset kept, sweeps with the float64 code).
template <int P, int K, int TIER, bool REDO = false>
__global__ __launch_bounds__(64, (min_waves<P, K, TIER>())) void subset_kernel(Pools pl) {
    constexpr int KS = P - 2;
    constexpr int M = 64 * K;
    using Slot = typename SlotOf<P, TIER>::type;
    __shared__ Slot slots[64];
    constexpr bool BUCKET = TIER == kFiltBucket;
    // p = 2 (one sweep per query) always takes the full sort
    static_assert(!(BUCKET && P == 2), "no bucketed sweep at p = 2");
    // side table of the full-sort sweep
    constexpr bool FULLSORT = TIER == kFilt;
    __shared__ uint16_t side[FULLSORT ? M : 1];
    __shared__ uint32_t hist[BUCKET ? BucketGeom<K>::HW : 1];
    __shared__ uint4 glist[BUCKET ? kListMax : 1];
    // per-block device scratch: float64 basis slots, then the staging arrays
    uint8_t* wsc = pl.wscratch + pl.cp->cls_scratch[pl.cls] + (uint64_t)blockIdx.x * pl.wscratch_bytes;
    SlotF64<P>* slots64 = reinterpret_cast<SlotF64<P>*>(wsc);
    Staging sg;
    {
        uint8_t* p0 = wsc + (uint64_t)64 * (2 * kMaxP + 2) * 8;
        sg.rt = reinterpret_cast<double*>(p0);
        sg.pkey = reinterpret_cast<uint32_t*>(p0 + (size_t)M * 8);
        sg.pS = reinterpret_cast<int*>(p0 + (size_t)M * 12);
        sg.rr = reinterpret_cast<float*>(p0 + (size_t)M * 16);
        sg.pflag = p0 + (size_t)M * 20;
    }
    const int lane = lane_id();
    if constexpr (BUCKET) {
#pragma unroll
        for (int j = 0; j < BucketGeom<K>::NBL; ++j) hist[lane * BucketGeom<K>::NBL + j] = 0u;
        __syncthreads();
    }
    double xd[TIER == kPlain ? K : 1][P];
    float xf[TIER == kPlain ? 1 : K][P];
    unsigned long long swept = 0, rechecks = 0, ndefer = 0, ninvalid = 0, nwalked = 0;
    FiltCtx fc;
    fc.fscale = pl.filter_scale;
    const uint64_t cbeg = pl.cp->cls_begin[pl.cls];
    const uint64_t cend = pl.cp->cls_end[pl.cls];
    const uint32_t chunk = pl.cp->cls_chunk[pl.cls];
    const int nq = pl.cp->num_queries;
    // float64 pass: the handed-over items, counted by the first pass (which
    // has completed: the launches are stream-ordered); none, as a rule, and
    // then no block touches the shared work counter (4096 atomics on one
    // address cost about 0.5 ms), nor when the grid covers every unit
    const uint64_t nredo = REDO ? uni64(min((uint64_t)pl.ctr->redo_count[pl.cls], pl.redo_cap)) : 0;
    if (REDO && nredo == 0) return;
    // block b takes item (float64 pass: unit) b first, then the shared
    // counter hands out the ones past the grid (no atomic at all when the
    // grid covers them)
    bool first = true;
    while (true) {
        unsigned long long item = 0;
        uint64_t rstart = 0;
        uint64_t rstop = ~0ull;
        uint64_t rmask = ~0ull;   // subsets of the first batch to sweep
        if constexpr (REDO) {
            // each handed-over item cut into units that the waves take in
            // turn: unit 0 the marked subsets of the batch at `base`, then
            // kRedoUnit subsets each from base + 64 on, so that no item's
            // rest is left to a single wave
            const uint64_t upe = 1 + (chunk + kRedoUnit - 1) / kRedoUnit;
            unsigned long long u = 0;
            if (first) {
                u = blockIdx.x;
                first = false;
            } else {
                if ((uint64_t)gridDim.x >= nredo * upe) break;
                if (lane == 0) u = gridDim.x + atomicAdd(&pl.ctr->redo_next[pl.cls], 1ull);
                u = uni64(__shfl(u, 0, 64));
            }
            const uint64_t e = u / upe;
            if (e >= nredo) break;
            const uint64_t k = u - e * upe;
            item = uni64(pl.redo[e].item);
            const uint64_t base = uni64(pl.redo[e].base);
            if (k == 0) {
                rstart = base;
                rstop = base + 64;
                rmask = uni64(pl.redo[e].mask);
            } else {
                rstart = base + 64 + (k - 1) * kRedoUnit;
                rstop = rstart + kRedoUnit;
            }
        } else {
            if (first) {
                item = cbeg + blockIdx.x;
                first = false;
            } else {
                if (cbeg + gridDim.x >= cend) break;
                if (lane == 0) item = cbeg + gridDim.x + atomicAdd(&pl.ctr->work_next[pl.cls], 1ull);
                item = uni64(__shfl(item, 0, 64));
            }
            if (item >= cend) break;
        }
        const int q = uni(item_query(pl.qd, nq, item));
        const QueryDesc d = pl.qd[q];
        const QueryState st = pl.qs[q];
        if (st.status & kStNonfinite) continue;
        const int nnz = uni(st.nnz);
        // ground set of the enumeration: all nonzero points, or the
        // candidate points of a restricted query
        const int32_t* kmap = d.kmap;
        const int ng = kmap ? uni(d.kcount) : nnz;
        const uint64_t nsub = uni64(binom_lookup(pl.binom, ng, KS));
        const uint64_t ib = uni64((item - d.item_begin) * (uint64_t)chunk);
        const uint64_t r0 = REDO ? rstart : ib;
        const uint64_t r1 = uni64(min(min(ib + (uint64_t)chunk, nsub), rstop));
        if (r0 >= r1) continue;
        const double* x64 = pl.x64 + d.v_off;
        fc.x64 = x64;
        fc.nrm = pl.nrm + d.n_off;
        fc.idx_bits = d.idx_bits;
        int wbest = kBig;
        int qbest = kBig;
        for (uint64_t rb = r0; rb < r1; rb += 64) {
            if constexpr (TIER != kPlain) {
                // running minimum of the query (terms of other work items so
                // far) and, for the bucketed sweep, the bound from the
                // directions +-x_j; refreshed for every batch of 64 subsets
                qbest = uni(__hip_atomic_load(&pl.qs[q].min_term, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                // a term of 0 cannot be lowered: the rest of the item is not needed
                if (pl.prune && min(qbest, wbest) == 0) {
                    // subsets left: the rest of the range, or (float64 pass,
                    // first unit) the marked subsets of its single batch
                    unsigned long long left = r1 - rb;
                    if (REDO && rmask != ~0ull)
                        left = __popcll(rmask & (r1 - rb >= 64 ? ~0ull : (1ull << (r1 - rb)) - 1ull));
                    if (lane == 0) atomicAdd(&pl.ctr->pruned, left);
                    break;
                }
                if constexpr (BUCKET) qbest = min(qbest, uni(st.ub_term));
            }
            const uint64_t myr = rb + (uint64_t)lane;
            Slot& my = slots[lane];
            if (myr < r1 && ((rmask >> lane) & 1ull)) {
                int cc[KS > 0 ? KS : 1];
                cc[0] = 0;
                unrank_colex<KS>(pl.binom, myr, ng, cc);
                if (kmap) {
#pragma unroll
                    for (int c = 0; c < KS; ++c) cc[c] = kmap[cc[c]];
                }
                double A[P][KS > 0 ? KS : 1];
#pragma unroll
                for (int col = 0; col < KS; ++col)
#pragma unroll
                    for (int r = 0; r < P; ++r) A[r][col] = x64[(size_t)cc[col] * P + r];
                Basis<P> Bs;
                build_basis<P>(A, Bs);
                if constexpr (TIER != kPlain) {
                    // float64 minors that cancel badly: double-double rows
                    // (copies, so that only this rare path keeps the basis
                    // and the subset in memory)
                    if (!Bs.certified || Bs.eta > 0x1p-30) {
                        Basis<P> Br = Bs;
                        int cr[KS > 0 ? KS : 1];
#pragma unroll
                        for (int c = 0; c < KS; ++c) cr[c] = cc[c];
                        refine_basis_dd<P>(x64, pl.x64lo + d.v_off, cr, Br);
                        Bs = Br;
                    }
                }
#pragma unroll
                for (int col = 0; col < KS; ++col) my.mem[col] = (int16_t)cc[col];
                if constexpr (TIER == kPlain) {
                    SlotPlain<P>& S = reinterpret_cast<SlotPlain<P>&>(my);
#pragma unroll
                    for (int c = 0; c < P; ++c) { S.e1[c] = Bs.e1[c]; S.e2[c] = Bs.e2[c]; }
                    S.state = Bs.anynz ? 0 : 1;
                } else {
                    SlotFilt<P>& S = reinterpret_cast<SlotFilt<P>&>(my);
                    SlotF64<P>& S64 = slots64[lane];
                    // the float64 basis is kept (in device scratch) only where a
                    // float64 re-check can read it: the full-sort sweeps and
                    // the float64 pass
                    constexpr bool store64 = TIER == kFilt || REDO;
#pragma unroll
                    for (int c = 0; c < P; ++c) {
                        if (store64) {
                            S64.e1[c] = Bs.e1[c];
                            S64.e2[c] = Bs.e2[c];
                        }
                        S.f1[c] = (float)Bs.e1[c];
                        S.f2[c] = (float)Bs.e2[c];
                    }
                    // per coordinate of a unit-length point: rounding of the
                    // point and of the basis to float32, p products and sums,
                    // the float64 centring, and the frame error eta
                    S.beta32 = (float)((((double)P + 4.0) * (double)kU32 + 4.0 * kU64 + Bs.eta) * 1.01);
                    if (store64) S64.beta64 = (((double)P + 3.0) * kU64 + Bs.eta) * 1.01;
                    S.state = (Bs.certified && !pl.force_exact) ? 0 : 3;
                }
            } else {
                // past the item, or (float64 pass) a subset the first pass swept
                my.state = myr < r1 ? 4 : 1;
            }
            __syncthreads();
            // points of the query in registers for the sweeps of this batch,
            // reloaded per batch so that they are not live while bases are
            // built: an opaque zero (a volatile scalar move, no memory access)
            // keeps the loop-invariant loads from being hoisted out of the loop
            uint32_t opaque;
            asm volatile("s_mov_b32 %0, 0" : "=s"(opaque));
            if constexpr (TIER == kPlain) {
                const double* xb = x64 + opaque;
#pragma unroll
                for (int i = 0; i < K; ++i)
#pragma unroll
                    for (int c = 0; c < P; ++c) xd[TIER == kPlain ? i : 0][c] = xb[(size_t)(lane * K + i) * P + c];
            } else {
                const float* x32 = pl.x32 + d.v_off + opaque;
#pragma unroll
                for (int i = 0; i < K; ++i) {
#pragma unroll
                    for (int c = 0; c < P; ++c) xf[TIER == kPlain ? 0 : i][c] = x32[(size_t)(lane * K + i) * P + c];
                }
            }
            const int cnt = (int)min((uint64_t)64, r1 - rb);
            // subsets of the batch that need the float64 pass (first pass, p >= 3)
            uint64_t need = 0;
            for (int s = 0; s < cnt; ++s) {
                const Slot& S = slots[s];
                const int sstate = uni(S.state);
                if (sstate == 1) { ++ninvalid; continue; }
                if (REDO && sstate == 4) continue;
                int term;
                if constexpr (TIER == kPlain) {
                    term = sweep_plain<P, K>(xd, reinterpret_cast<const SlotPlain<P>&>(S), nnz);
                } else {
                    if (sstate == 3) {
                        term = kDefer;
                    } else {
                        if constexpr (BUCKET) {
                            // a walk gathers at most kListMax points: the
                            // exact tier takes the sweeps that exceed it (a
                            // bucket's crossing field counts at most 1023, and
                            // with n <= 1024 a sweep has at most 1023 points)
                            term = kFallback;
                            if (nnz - KS <= 1024) {
                                const int ub = min(qbest, wbest);
                                const SlotFilt<P>& SF = reinterpret_cast<const SlotFilt<P>&>(S);
                                term = sweep_bucket<P, K, REDO>(xf, SF, slots64[s], nnz, fc, hist, glist, sg, ub,
                                                                rechecks, nwalked);
                                if (term == kNeed64) {
                                    // marked for the float64 pass; no branch
                                    // out of the loop here (one makes the
                                    // compiler turn the sweep's loops into
                                    // exec-masked code: 11% at p = 5)
                                    need |= 1ull << s;
                                    continue;
                                }
                            }
                            if (term == kFallback) term = kDefer;
                        } else {
                            term = sweep_filt<P, K>(xf, reinterpret_cast<const SlotFilt<P>&>(S), slots64[s], nnz,
                                                    fc, side, sg, rechecks);
                        }
                    }
                }
                if (term == kDefer) {
                    if (lane == 0) push_deferred<P>(pl, q, rb + (uint64_t)s);
                    ++ndefer;
                    continue;
                }
                if (term == kSkip) {
                    // bounded below by a term already reached or by ub_term:
                    // the subset is valid (certified basis) and its term is at
                    // least that bound, which it records
                    ++swept;
                    wbest = min(wbest, qbest);
                    continue;
                }
                ++swept;
                wbest = min(wbest, term);
            }
            __syncthreads();
            if constexpr (BUCKET && !REDO) {
                if (need) {
                    // hand the marked subsets and the rest of the item to the
                    // float64 pass; with its list full, the marked subsets go
                    // to the exact tier and the item goes on here
                    unsigned long long pos = 0;
                    if (lane == 0) pos = atomicAdd(&pl.ctr->redo_count[pl.cls], 1ull);
                    pos = uni64(__shfl(pos, 0, 64));
                    if (pos < pl.redo_cap) {
                        if (lane == 0) {
                            RedoItem ri;
                            ri.item = item;
                            ri.base = rb;
                            ri.mask = need;
                            pl.redo[pos] = ri;
                        }
                        break;
                    }
                    for (int s = 0; s < 64; ++s) {
                        if ((need >> s) & 1ull) {
                            if (lane == 0) push_deferred<P>(pl, q, rb + (uint64_t)s);
                            ++ndefer;
                        }
                    }
                }
            }
        }
        if (lane == 0 && wbest < kBig) atomicMin(&pl.qs[q].min_term, wbest);
    }
    // counters (ninvalid counts subsets seen as invalid by the float64 basis)
    unsigned long long rc = rechecks;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) rc += __shfl_xor(rc, o, 64);
    if (lane == 0) {
        if (swept) atomicAdd(&pl.ctr->swept, swept);
        if (rc) atomicAdd(&pl.ctr->fp64_rechecks, rc);
        if (ndefer) atomicAdd(&pl.ctr->deferred, ndefer);
        if (ninvalid) atomicAdd(&pl.ctr->invalid, ninvalid);
        if (nwalked) atomicAdd(&pl.ctr->walked, nwalked);
    }
}

}  // namespace td
