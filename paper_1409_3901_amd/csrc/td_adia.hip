// Kernels of the paper's adaptive algorithm (Algorithm 3, Section 4).  The
// host drives the iteration (the queue of critical (p-1)-sets of Steps 3-4);
// every evaluation runs here:
//   adia_seed_kernel : Step 2 (the direction among +-x_j with the fewest
//                      points on its closed side, and the seed subset);
//   adia_eval_kernel : Steps 2(c) and 4(a)(i)-(ii) for a batch of explicit
//                      (p-2)-subsets: the value of Algorithm 2 on each, and
//                      the points next to its minimising states;
//   adia_cand_kernel : Step 5(a), the points on the closed smaller side of
//                      every remaining critical hyperplane, as bit masks;
//   adia_kmap_kernel : those masks compacted into the index maps of the
//                      restricted subset kernels that carry out Step 5(b).
// The evaluations steer the search only: Step 5(b) computes the final value
// with the certified (exact) tiers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "td_adia.hpp"
#include "td_device.hpp"

namespace td {

// min(S, m - S): the smaller side of the line through the origin.
__device__ __forceinline__ int fside(int s, int m) { return min(s, m - s); }

// Block-wide reductions over 256 threads (4 waves) through `red`.
__device__ __forceinline__ long long block_min_ll(long long v, long long* red) {
    for (int o = 32; o >= 1; o >>= 1) {
        const long long w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    long long r = red[0];
    for (int w = 1; w < 4; ++w) r = red[w] < r ? red[w] : r;
    __syncthreads();
    return r;
}

__device__ __forceinline__ int block_sum_i(int v, int* red) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const int r = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return r;
}

// Sign of x_a . x_b in float64 with a rounding bound: 0 when the bound does
// not settle it (such decisions are taken as zero: a tie).
__device__ __forceinline__ int dot_sign64(const double* x64, int p, int a, int b, double& v) {
    double s = 0.0, ab = 0.0;
    for (int c = 0; c < p; ++c) {
        const double t = x64[(size_t)a * p + c] * x64[(size_t)b * p + c];
        s += t;
        ab += fabs(t);
    }
    v = s;
    const double bound = ab * (double)(2 * p + 4) * kU64 * 1.01;
    return s > bound ? 1 : (s < -bound ? -1 : 0);
}

// Step 2(a) is split over blocks: the keys start at the largest value, then
// block (q, s) takes the directions x_j, j in [64 s, 64 s + 64), of query q;
// its thread (jj, h) counts the points i = h, h + 4, ... on either closed
// side of x_{64 s + jj}, the four partial counts are added in LDS, and the
// smallest key count * 2n' + 2j + (sign < 0) of the block goes to
// seeds[q].best by an atomic minimum (the keys are nonnegative, so the
// minimum over the blocks is the minimum over every direction).
__global__ void adia_best_init_kernel(AdiaSeed* seeds, int nq) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) seeds[q].best = ~0ull;
}

constexpr int kSeedSlices = kMaxN / 64;

__global__ __launch_bounds__(256) void adia_dirs_kernel(Pools pl, AdiaSeed* seeds) {
    __shared__ int s_cp[4][64];
    __shared__ int s_cn[4][64];
    __shared__ long long s_red[4];
    const int q = blockIdx.x / kSeedSlices;
    const int sl = blockIdx.x % kSeedSlices;
    if (q >= pl.cp->num_queries) return;
    const int nnz = pl.qs[q].nnz;
    const int p = pl.qd[q].p;
    if (nnz <= 0 || p < 3 || sl * 64 >= nnz) return;
    const double* x64 = pl.x64 + pl.qd[q].v_off;
    const int tid = threadIdx.x;
    const int jj = tid & 63, h = tid >> 6;
    const int j = sl * 64 + jj;
    int cp = 0, cn = 0;
    if (j < nnz) {
        for (int i = h; i < nnz; i += 4) {
            double v;
            const int sg = dot_sign64(x64, p, j, i, v);
            cp += sg <= 0 ? 1 : 0;
            cn += sg >= 0 ? 1 : 0;
        }
    }
    s_cp[h][jj] = cp;
    s_cn[h][jj] = cn;
    __syncthreads();
    long long key = 0x7fffffffffffffffll;
    if (h == 0 && j < nnz) {
        const int tp = s_cp[0][jj] + s_cp[1][jj] + s_cp[2][jj] + s_cp[3][jj];
        const int tn = s_cn[0][jj] + s_cn[1][jj] + s_cn[2][jj] + s_cn[3][jj];
        const long long kp = (long long)tp * (2ll * nnz) + 2ll * j;
        const long long kn = (long long)tn * (2ll * nnz) + 2ll * j + 1;
        key = kp < kn ? kp : kn;
    }
    key = block_min_ll(key, s_red);
    if (tid == 0) atomicMin(&seeds[q].best, (unsigned long long)key);
}

// Step 2, one block per query, after adia_dirs_kernel.  (a) u_min: over j
// and the sign (x_j before -x_j), the fewest points with u . x_i <= 0,
// smallest j first (the key of seeds[q].best); (b) the p - 2 points with the
// smallest nonnegative u_min . x_i (by value, then index).
__global__ __launch_bounds__(256) void adia_seed_kernel(Pools pl, AdiaSeed* seeds) {
    __shared__ double s_pr[kMaxN];
    __shared__ long long s_red[4];
    __shared__ int s_ired[4];
    __shared__ int s_pick[kMaxP];
    const int q = blockIdx.x;
    if (q >= pl.cp->num_queries) return;
    const QueryDesc d = pl.qd[q];
    const int nnz = pl.qs[q].nnz;
    const int p = d.p;
    const double* x64 = pl.x64 + d.v_off;
    const int tid = threadIdx.x;
    AdiaSeed out;
    out.kneg = 0;
    out.ok = 0;
    for (int c = 0; c < kMaxP - 2; ++c) out.idx[c] = -1;
    out.best = ~0ull;
    if (nnz <= 0 || p < 3) {
        if (tid == 0) seeds[q] = out;
        return;
    }
    // (a) key = count * 2n + 2j + (sign < 0): the smallest key, found by
    // adia_dirs_kernel (nnz > 0: at least one direction)
    const long long best = (long long)seeds[q].best;
    const int r = (int)(best % (2ll * nnz));
    const int bj = r >> 1;
    const double sgn = (r & 1) ? -1.0 : 1.0;
    // (b) projections on u_min (a tie with 0 counts as nonnegative)
    int kneg = 0;
    for (int i = tid; i < nnz; i += blockDim.x) {
        double v;
        const int sg = dot_sign64(x64, p, bj, i, v);
        s_pr[i] = sgn * v;
        kneg += (sgn * (double)sg < 0.0) ? 1 : 0;
    }
    __syncthreads();
    kneg = block_sum_i(kneg, s_ired);
    out.kneg = kneg;
    if (kneg == 0) {
        if (tid == 0) seeds[q] = out;
        return;
    }
    const int ks = p - 2;
    int ok = 1;
    for (int c = 0; c < ks; ++c) {
        // smallest (value, index) among the nonnegative points not taken;
        // the order key packs the rank of the value below the index
        long long bk = 0x7fffffffffffffffll;
        for (int i = tid; i < nnz; i += blockDim.x) {
            bool taken = false;
            for (int e = 0; e < c; ++e) taken = taken || (s_pick[e] == i);
            double v;
            const int sg = dot_sign64(x64, p, bj, i, v);
            if (taken || sgn * (double)sg < 0.0) continue;
            const double pv = sg == 0 ? 0.0 : s_pr[i];
            // nonnegative doubles order like their bits
            const long long key = (long long)(__double_as_longlong(pv) >> 11) * 1024 + i;
            bk = key < bk ? key : bk;
        }
        bk = block_min_ll(bk, s_red);
        if (tid == 0) s_pick[c] = bk == 0x7fffffffffffffffll ? -1 : (int)(bk % 1024);
        __syncthreads();
        if (s_pick[c] < 0) ok = 0;
    }
    if (tid == 0) {
        out.ok = ok;
        for (int c = 0; c < ks; ++c) out.idx[c] = s_pick[c];
        seeds[q] = out;
    }
}

// Steps 2(c) and 4(a)(i)-(ii), one wave per job: the float64 basis of the
// subset, Algorithm 2 with ties grouped on equal keys, its value
// (b + points projecting to the origin), and the points of the runs next to
// a state where min(S, m - S) is smallest (state r lies between runs r - 1
// and r; the first and the last state both lie next to the first and the
// last run, the sweep being circular).
template <int P, int K>
__global__ __launch_bounds__(64) void adia_eval_kernel(Pools pl, const AdiaJob* jobs, int njobs, AdiaRes* res) {
    constexpr int KS = P - 2;
    constexpr int M = 64 * K;
    __shared__ int s_after[M];
    __shared__ int s_t[kAdiaTMax];
    __shared__ int s_tc;
    const int jb = blockIdx.x;
    if (jb >= njobs) return;
    const int lane = lane_id();
    const AdiaJob job = jobs[jb];
    const int q = job.q;
    const QueryDesc d = pl.qd[q];
    const int nnz = pl.qs[q].nnz;
    const double* x64 = pl.x64 + d.v_off;
    int mem[KS > 0 ? KS : 1];
    mem[0] = 0;
#pragma unroll
    for (int c = 0; c < KS; ++c) mem[c] = job.idx[c];
    double A[P][KS > 0 ? KS : 1];
#pragma unroll
    for (int col = 0; col < KS; ++col)
#pragma unroll
        for (int r = 0; r < P; ++r) A[r][col] = x64[(size_t)mem[col] * P + r];
    Basis<P> Bs;
    build_basis<P>(A, Bs);
    if (lane == 0) s_tc = 0;
    if (!Bs.anynz) {
        if (lane == 0) {
            res[jb].term = -1;
            res[jb].tcount = 0;
        }
        return;
    }
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
            const double v = valid ? x64[(size_t)idx * P + c] : 0.0;
            y1 = fma(Bs.e1[c], v, y1);
            y2 = fma(Bs.e2[c], v, y2);
        }
        uint64_t kk = ~0ull;
        if (valid) {
            if (y1 == 0.0 && y2 == 0.0) {
                ++zc;
            } else {
                const bool pos = (y1 > 0.0) || (y1 == 0.0 && y2 > 0.0);
                const double h1 = pos ? y1 : -y1;
                const double h2 = pos ? y2 : -y2;
                const double t = h2 / (h1 + fabs(h2)) + 1.0;   // in (0, 2]
                // angle key in the high bits, point index and fold below
                kk = ((uint64_t)__double_as_longlong(t) & ~0x7ffull) | ((uint64_t)idx << 1) | (pos ? 0ull : 1ull);
                nplus += pos ? 1 : 0;
            }
        }
        key[i] = kk;
    }
    wave_sort<K>(key);
    const int ztot = wave_sum(zc);
    const int m = nnz - KS - ztot;
    const int S0 = wave_sum(nplus);
    // runs of equal angle key, and the state after every element
    const uint64_t nxt = ((uint64_t)(uint32_t)lane_next((int)(key[0] >> 32), 0) << 32) |
                         (uint32_t)lane_next((int)(uint32_t)key[0], 0);
    const uint64_t prv = ((uint64_t)(uint32_t)lane_prev((int)(key[K - 1] >> 32), 0) << 32) |
                         (uint32_t)lane_prev((int)(uint32_t)key[K - 1], 0);
    int loc = 0, starts = 0;
    bool st[K], en[K];
    int sv[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const bool real = key[i] != ~0ull;
        const uint64_t pk = (i > 0) ? key[i - 1] : ((lane == 0) ? ~0ull : prv);
        const uint64_t nk = (i + 1 < K) ? key[i + 1] : ((lane == 63) ? ~0ull : nxt);
        st[i] = real && (pk == ~0ull || (pk >> 11) != (key[i] >> 11));
        en[i] = real && (nk == ~0ull || (nk >> 11) != (key[i] >> 11));
        loc += real ? ((key[i] & 1ull) ? 1 : -1) : 0;
        starts += st[i] ? 1 : 0;
    }
    int s = S0 + wave_excl_sum(loc);
    int rid = wave_excl_sum(starts) - 1;
    const int nruns = wave_sum(starts);
    int best = (lane == 0) ? fside(S0, m) : 0x7fffffff;
    int rids[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const bool real = key[i] != ~0ull;
        s += real ? ((key[i] & 1ull) ? 1 : -1) : 0;
        rid += st[i] ? 1 : 0;
        sv[i] = s;
        rids[i] = rid;
        if (en[i]) {
            s_after[rid] = s;
            best = min(best, fside(s, m));
        }
    }
    best = wave_min(best);
    __syncthreads();
    const int S_end = nruns > 0 ? s_after[nruns - 1] : S0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (key[i] == ~0ull) continue;
        const int r = rids[i];
        const int before = (r == 0) ? S0 : s_after[r - 1];
        const int after = s_after[r];
        const bool hot = fside(before, m) == best || fside(after, m) == best ||
                         (r == 0 && fside(S_end, m) == best) || (r == nruns - 1 && fside(S0, m) == best);
        if (hot) {
            const int slot = atomicAdd(&s_tc, 1);
            if (slot < kAdiaTMax) s_t[slot] = (int)((key[i] >> 1) & 1023ull);
        }
    }
    __syncthreads();
    if (lane == 0) {
        const int tc = min(s_tc, kAdiaTMax);
        res[jb].term = best + ztot;
        res[jb].tcount = s_tc;
        for (int e = 0; e < tc; ++e) res[jb].t[e] = s_t[e];
    }
    (void)sv;
}

// Step 5(a), one wave per node: the normal u of the hyperplane through the
// node's p - 1 points (generalised cross product: the signed cofactors,
// float64 elimination with partial pivoting), the sides of all points
// (|u . x| within 1e-9 of the sum of |u_c x_c| counts as on the hyperplane),
// and the closed side holding fewer points (the side u . x <= 0 on a tie)
// marked in the query's mask.  A node with fewer points (mark-only) marks
// just its points.
__global__ __launch_bounds__(64) void adia_cand_kernel(Pools pl, const AdiaNode* nodes, int nnodes, uint32_t* kmask) {
    __shared__ double s_u[kMaxP];
    __shared__ int s_cnt[2];
    const int b = blockIdx.x;
    if (b >= nnodes) return;
    const int lane = lane_id();
    const AdiaNode nd = nodes[b];
    const int q = nd.q;
    const QueryDesc d = pl.qd[q];
    const int nnz = pl.qs[q].nnz;
    const int p = d.p;
    const double* x64 = pl.x64 + d.v_off;
    uint32_t* mask = kmask + (size_t)q * (kMaxN / 32);
    if (nd.count < p - 1) {
        if (lane < nd.count) atomicOr(&mask[nd.idx[lane] >> 5], 1u << (nd.idx[lane] & 31));
        return;
    }
    if (lane < 2) s_cnt[lane] = 0;
    const int k = p - 1;
    if (lane < p) {
        // cofactor of row `lane` in the last column of [x_F | e]:
        // (-1)^(lane + p - 1) det(x_F without row lane)
        double a[kMaxP - 1][kMaxP - 1];
        int rr = 0;
        for (int row = 0; row < p; ++row) {
            if (row == lane) continue;
            for (int c = 0; c < k; ++c) a[rr][c] = x64[(size_t)nd.idx[c] * p + row];
            ++rr;
        }
        double det = 1.0;
        for (int c = 0; c < k; ++c) {
            int piv = c;
            for (int r2 = c + 1; r2 < k; ++r2)
                if (fabs(a[r2][c]) > fabs(a[piv][c])) piv = r2;
            if (piv != c) {
                for (int c2 = 0; c2 < k; ++c2) {
                    const double t = a[c][c2];
                    a[c][c2] = a[piv][c2];
                    a[piv][c2] = t;
                }
                det = -det;
            }
            const double pv = a[c][c];
            det *= pv;
            if (pv == 0.0) break;
            for (int r2 = c + 1; r2 < k; ++r2) {
                const double f = a[r2][c] / pv;
                for (int c2 = c + 1; c2 < k; ++c2) a[r2][c2] -= f * a[c][c2];
            }
        }
        s_u[lane] = ((lane + p - 1) & 1) ? -det : det;
    }
    __syncthreads();
    int sgv[kMaxN / 64];
    int cneg = 0, cpos = 0;
    for (int t = 0; t < kMaxN / 64; ++t) {
        const int l = lane + 64 * t;
        int sg = 0;
        if (l < nnz) {
            double v = 0.0, ab = 0.0;
            for (int c = 0; c < p; ++c) {
                const double w = s_u[c] * x64[(size_t)l * p + c];
                v += w;
                ab += fabs(w);
            }
            bool member = false;
            for (int c = 0; c < k; ++c) member = member || (nd.idx[c] == l);
            if (!member) sg = v > 1e-9 * ab ? 1 : (v < -1e-9 * ab ? -1 : 0);
            cneg += sg < 0 ? 1 : 0;
            cpos += sg > 0 ? 1 : 0;
        }
        sgv[t] = sg;
    }
    cneg = wave_sum(cneg);
    cpos = wave_sum(cpos);
    const int side = (cneg <= cpos) ? -1 : 1;
    for (int t = 0; t < kMaxN / 64; ++t) {
        const int l = lane + 64 * t;
        if (l < nnz && (sgv[t] == 0 || sgv[t] == side)) atomicOr(&mask[l >> 5], 1u << (l & 31));
    }
}

// Compaction of each query's mask into an ascending index map (one wave per
// query); kcount[q] receives the number of candidate points.
__global__ __launch_bounds__(64) void adia_kmap_kernel(int nq, const uint32_t* kmask, int32_t* kmap, int32_t* kcount) {
    const int q = blockIdx.x;
    if (q >= nq) return;
    const int lane = lane_id();
    const uint32_t* mask = kmask + (size_t)q * (kMaxN / 32);
    int32_t* out = kmap + (size_t)q * kMaxN;
    int base = 0;
    for (int w0 = 0; w0 < kMaxN / 32; w0 += 2) {
        // lane L covers bit L of words w0 and w0 + 1
        const uint32_t wa = mask[w0], wb = mask[w0 + 1];
        const uint64_t bits = (uint64_t)wa | ((uint64_t)wb << 32);
        const bool on = (bits >> lane) & 1ull;
        const uint64_t below = lane == 0 ? 0ull : (bits & ((1ull << lane) - 1ull));
        if (on) out[base + __popcll(below)] = w0 * 32 + lane;
        base += __popcll(bits);
    }
    if (lane == 0) kcount[q] = base;
}

__global__ void adia_clear_kernel(uint32_t* kmask, int words) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x) kmask[i] = 0u;
}

}  // namespace td

namespace {
using EvalFn = void (*)(td::Pools, const td::AdiaJob*, int, td::AdiaRes*);

template <int P>
EvalFn eval_for(int K) {
    switch (K) {
        case 1: return td::adia_eval_kernel<P, 1>;
        case 2: return td::adia_eval_kernel<P, 2>;
        case 4: return td::adia_eval_kernel<P, 4>;
        case 8: return td::adia_eval_kernel<P, 8>;
        case 16: return td::adia_eval_kernel<P, 16>;
    }
    return nullptr;
}

EvalFn pick_eval(int P, int K) {
    switch (P) {
        case 3: return eval_for<3>(K);
        case 4: return eval_for<4>(K);
        case 5: return eval_for<5>(K);
        case 6: return eval_for<6>(K);
        case 7: return eval_for<7>(K);
        case 8: return eval_for<8>(K);
    }
    return nullptr;
}
}  // namespace

extern "C" hipError_t td_launch_adia_seed(const td::Pools* pl, int nq, td::AdiaSeed* seeds, hipStream_t s) {
    hipLaunchKernelGGL(td::adia_best_init_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, seeds, nq);
    hipLaunchKernelGGL(td::adia_dirs_kernel, dim3((unsigned)nq * td::kSeedSlices), dim3(256), 0, s, *pl, seeds);
    hipLaunchKernelGGL(td::adia_seed_kernel, dim3(nq), dim3(256), 0, s, *pl, seeds);
    return hipGetLastError();
}

extern "C" hipError_t td_launch_adia_eval(int P, int K, const td::Pools* pl, const td::AdiaJob* jobs, int njobs,
                                          td::AdiaRes* res, hipStream_t s) {
    EvalFn f = pick_eval(P, K);
    if (!f || njobs <= 0) return f ? hipSuccess : hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(njobs), dim3(64), 0, s, *pl, jobs, njobs, res);
    return hipGetLastError();
}

extern "C" hipError_t td_launch_adia_cand(const td::Pools* pl, int nq, const td::AdiaNode* nodes, int nnodes,
                                          uint32_t* kmask, int32_t* kmap, int32_t* kcount, hipStream_t s) {
    const int words = nq * (td::kMaxN / 32);
    hipLaunchKernelGGL(td::adia_clear_kernel, dim3(std::max(1, std::min(1024, (words + 255) / 256))), dim3(256), 0,
                       s, kmask, words);
    if (nnodes > 0) hipLaunchKernelGGL(td::adia_cand_kernel, dim3(nnodes), dim3(64), 0, s, *pl, nodes, nnodes, kmask);
    hipLaunchKernelGGL(td::adia_kmap_kernel, dim3(nq), dim3(64), 0, s, nq, kmask, kmap, kcount);
    return hipGetLastError();
}
