// Preparation, initialisation and finalisation kernels.
#include <hip/hip_runtime.h>

#include "td_common.hpp"
#include "td_device.hpp"

namespace td {

// Clears the per-call counters (a kernel, not a memset, so the whole call can
// be captured in a graph and replayed).
__global__ void init_kernel(Counters* ctr) {
    unsigned long long* c = reinterpret_cast<unsigned long long*>(ctr);
    const int n = (int)(sizeof(Counters) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0ull;
}

// The thread's part of the bound from the directions +-x_j: for its rows j,
// the closed-side counts of u = s_x[j] over all nnz rows (p = P, rows of P
// floats in LDS), a count taken whenever the product is within e of the side.
template <int P>
__device__ int dir_bound(const float* s_x, int nnz, int tid, float e) {
    int ub = 0x7fffffff;
    for (int j = tid; j < nnz; j += blockDim.x) {
        float u[P];
#pragma unroll
        for (int c = 0; c < P; ++c) u[c] = s_x[j * P + c];
        int le = 0, ge = 0;
        for (int i = 0; i < nnz; ++i) {
            float dot = 0.0f;
#pragma unroll
            for (int c = 0; c < P; ++c) dot = fmaf(u[c], s_x[i * P + c], dot);
            le += dot <= e ? 1 : 0;
            ge += dot >= -e ? 1 : 0;
        }
        ub = min(ub, min(le, ge));
    }
    return ub;
}

// One block of 256 threads per query (persistent over queries).  Shift to the
// query (Section 2: x_i = X_i - z), drop the observations equal to it (they
// lie on every hyperplane through z and add n0 to every count), and store
// the nonzero points compacted in input order:
//   x64 : float64 centred values (one rounding), x64lo: the remainder,
//   x32 : float32 copies scaled to unit length,
//   nrm : float32 upper bound of ||x||_2 of the float64 values,
//   xi  : exact integers (X - z) * 2^-E, E the lowest bit exponent over the
//         query's inputs (two's complement, 128 bits).
// p = 1 needs no subsets: the count is n0 + min(#{x > 0}, #{x < 0}).
__global__ __launch_bounds__(256) void prep_kernel(Pools pl) {
    __shared__ int s_flag[kMaxN];
    __shared__ int s_pos[kMaxN];
    __shared__ float s_x[kMaxN * kMaxP];
    __shared__ int s_red[8];
    __shared__ int s_wsum[4];
    __shared__ int s_q;
    __shared__ double s_z[kMaxP];
    const int tid = threadIdx.x;
    // block b takes query b first, then the shared counter the queries past
    // the grid
    bool first = true;
    while (true) {
        int q;
        if (first) {
            q = (int)blockIdx.x;
            first = false;
        } else {
            if ((int)gridDim.x >= pl.cp->num_queries) break;
            if (tid == 0) s_q = (int)gridDim.x + (int)atomicAdd(&pl.ctr->prep_next, 1ull);
            __syncthreads();
            q = s_q;
            __syncthreads();
        }
        if (q >= pl.cp->num_queries) break;
        const QueryDesc d = pl.qd[q];
        const int n = d.n, p = d.p, M = d.M;
        if (tid < p) s_z[tid] = d.z[tid];
        __syncthreads();
        int bad = 0;
        if (tid < p && !isfinite(s_z[tid])) bad = 1;
        // nonzero flags
        for (int i = tid; i < n; i += blockDim.x) {
            int nz = 0;
            for (int c = 0; c < p; ++c) {
                const double v = d.X[(size_t)i * p + c];
                if (!isfinite(v)) bad = 1;
                if (v != s_z[c]) nz = 1;
            }
            s_flag[i] = nz;
        }
        // lowest / highest bit exponents over the inputs (for the exact copy)
        int emin = 1 << 20, emax = -(1 << 20);
        for (int i = tid; i < n * p; i += blockDim.x) {
            const double v = d.X[i];
            if (v != 0.0 && isfinite(v)) {
                emin = min(emin, low_exp(v));
                emax = max(emax, high_exp(v));
            }
        }
        if (tid < p && s_z[tid] != 0.0 && isfinite(s_z[tid])) {
            emin = min(emin, low_exp(s_z[tid]));
            emax = max(emax, high_exp(s_z[tid]));
        }
        __syncthreads();
        // block reductions: bad (or), emin, emax
        {
            int v = bad;
            for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, 64);
            int a = wave_min(emin), b = wave_max(emax);
            if ((tid & 63) == 0) { s_red[tid >> 6] = v; s_red[4 + (tid >> 6)] = a; }
            __syncthreads();
            if (tid == 0) {
                int o = 0, mn = 1 << 20;
                for (int w = 0; w < 4; ++w) { o |= s_red[w]; mn = min(mn, s_red[4 + w]); }
                s_red[0] = o;
                s_red[1] = mn;
            }
            __syncthreads();
            bad = s_red[0];
            emin = s_red[1];
            __syncthreads();
            if ((tid & 63) == 0) s_red[4 + (tid >> 6)] = b;
            __syncthreads();
            if (tid == 0) {
                int mx = -(1 << 20);
                for (int w = 0; w < 4; ++w) mx = max(mx, s_red[4 + w]);
                s_red[2] = mx;
            }
            __syncthreads();
            emax = s_red[2];
        }
        // order-preserving compaction: exclusive scan of the flags, four
        // consecutive flags per thread (n <= kMaxN = 4 * blockDim.x)
        int nnz = 0;
        {
            constexpr int kPer = kMaxN / 256;
            const int b0 = tid * kPer;
            int f[kPer];
            int sum = 0;
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                f[k] = b0 + k < n ? s_flag[b0 + k] : 0;
                sum += f[k];
            }
            const int ex = wave_excl_sum(sum);
            if ((tid & 63) == 63) s_wsum[tid >> 6] = ex + sum;
            __syncthreads();
            int acc = ex;
            for (int w = 0; w < 4; ++w) {
                acc += w < (tid >> 6) ? s_wsum[w] : 0;
                nnz += s_wsum[w];
            }
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                if (b0 + k < n) s_pos[b0 + k] = acc;
                acc += f[k];
            }
        }
        __syncthreads();
        double* x64 = pl.x64 + d.v_off;
        double* x64lo = pl.x64lo + d.v_off;
        float* x32 = pl.x32 + d.v_off;
        float* nrm = pl.nrm + d.n_off;
        uint64_t* xi = pl.xi + d.v_off * 2;
        const bool ints_ok = (emax - emin + 2) <= 125 && emin < (1 << 19);
        for (int i = tid; i < M; i += blockDim.x) {
            // padding rows beyond nnz are zero
            if (i >= nnz) {
                for (int c = 0; c < p; ++c) {
                    x64[(size_t)i * p + c] = 0.0;
                    x64lo[(size_t)i * p + c] = 0.0;
                    x32[(size_t)i * p + c] = 0.0f;
                    xi[((size_t)i * p + c) * 2] = 0;
                    xi[((size_t)i * p + c) * 2 + 1] = 0;
                }
                nrm[i] = 0.0f;
            }
        }
        for (int i = tid; i < n; i += blockDim.x) {
            if (!s_flag[i]) continue;
            const int j = s_pos[i];
            double ss = 0.0;
#pragma unroll
            for (int c = 0; c < kMaxP; ++c)
                if (c < p) {
                    const double v = d.X[(size_t)i * p + c] - s_z[c];
                    ss = fma(v, v, ss);
                }
            // float32 copy scaled to unit length: the float32 filter only
            // needs directions (the pseudo-angle and the fold of a point do
            // not change under positive scaling), and unit length makes its
            // error radius the same for every point
            const double inv = 1.0 / sqrt(ss);
            for (int c = 0; c < p; ++c) {
#pragma clang fp contract(off)
                const double xv = d.X[(size_t)i * p + c];
                const double v = xv - s_z[c];
                // exact remainder of the subtraction (TwoSum of xv and -z)
                const double zz = v - xv;
                x64lo[(size_t)j * p + c] = (xv - (v - zz)) + (-s_z[c] - zz);
                x64[(size_t)j * p + c] = v;
                x32[(size_t)j * p + c] = (float)(v * inv);
                uint64_t lo = 0, hi = 0;
                if (ints_ok) {
                    uint64_t alo, ahi, blo, bhi;
                    to_i128(xv, emin, alo, ahi);
                    to_i128(s_z[c], emin, blo, bhi);
                    lo = alo - blo;
                    hi = ahi - bhi - (alo < blo ? 1ull : 0ull);
                }
                xi[((size_t)j * p + c) * 2] = lo;
                xi[((size_t)j * p + c) * 2 + 1] = hi;
            }
            // rounding-safe upper bound: relative slack far above the few ulps
            // of the sum, the square root and the conversion to float32
            nrm[j] = (float)(sqrt(ss) * (1.0 + 1e-6));
        }
        // Upper bound of the minimum from the 2n' directions +-x_j (Algorithm
        // 3, Step 2(a)): the depth is at most the closed halfspace count of
        // any direction.  The directions are the float32 unit copies u = x32_j
        // (any direction gives a valid bound), and the signs are those of
        // <u, x32_i>: x32_i is x_i / ||x_i|| up to u32 per coordinate, both
        // vectors have norm at most 1 + p u32, so the float32 inner product
        // is within e = (p + 4) u32 of the sign-deciding <u, x_i / ||x_i||>.
        // A point within e of a side is counted on it, so a count can only be
        // too high and the bound stays valid.
        // (p >= 3 only: at p = 2 a query has one sweep, cheaper than the
        // n'^2 p products of the bound)
        int ub = 0x7fffffff;
        if (pl.prune && p >= 3 && nnz > 0) {
            __syncthreads();
            for (int k = tid; k < nnz * p; k += blockDim.x) s_x[k] = x32[k];
            __syncthreads();
            const float e = ((float)p + 4.0f) * kU32;
            switch (p) {
                case 3: ub = dir_bound<3>(s_x, nnz, tid, e); break;
                case 4: ub = dir_bound<4>(s_x, nnz, tid, e); break;
                case 5: ub = dir_bound<5>(s_x, nnz, tid, e); break;
                case 6: ub = dir_bound<6>(s_x, nnz, tid, e); break;
                case 7: ub = dir_bound<7>(s_x, nnz, tid, e); break;
                default: ub = dir_bound<8>(s_x, nnz, tid, e); break;
            }
            ub = wave_min(ub);
            __syncthreads();
            if ((tid & 63) == 0) s_red[tid >> 6] = ub;
            __syncthreads();
            ub = min(min(s_red[0], s_red[1]), min(s_red[2], s_red[3]));
            __syncthreads();
        }
        // p = 1: closed form
        int pos1 = 0, neg1 = 0;
        if (p == 1) {
            for (int i = tid; i < n; i += blockDim.x) {
                const double v = d.X[i] - s_z[0];
                pos1 += v > 0.0;
                neg1 += v < 0.0;
            }
            pos1 = wave_sum(pos1);
            neg1 = wave_sum(neg1);
            __syncthreads();
            if ((tid & 63) == 0) { s_red[tid >> 6] = pos1; s_red[4 + (tid >> 6)] = neg1; }
            __syncthreads();
            if (tid == 0) {
                pos1 = s_red[0] + s_red[1] + s_red[2] + s_red[3];
                neg1 = s_red[4] + s_red[5] + s_red[6] + s_red[7];
            }
        }
        if (tid == 0) {
            QueryState st;
            st.nnz = nnz;
            st.n0 = n - nnz;
            st.status = (bad ? kStNonfinite : 0) | (ints_ok ? 0 : kStNoExactInts);
            st.min_term = d.zero_term ? 0 : 0x7fffffff;
            st.ub_term = ub;
            if (p == 1) st.min_term = min(pos1, neg1);
            if (nnz == 0) st.min_term = 0;
            pl.qs[q] = st;
        }
        __syncthreads();
    }
}

// counts[q] = n0 + min over subsets, or -1 with a status bit.
__global__ void finalize_kernel(Pools pl) {
    const int nq = pl.cp->num_queries;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        QueryState st = pl.qs[q];
        int bad = st.status & (kStNonfinite | kStDeferOverflow | kStExactRange | kStDegenLimit | kStNotGeneral);
        int out;
        if (bad) {
            out = -1;
        } else if (st.min_term == 0x7fffffff) {
            out = -1;
            st.status |= kStNoValid;
            pl.qs[q].status = st.status;
        } else {
            // some valid subset recorded a term; a subset skipped against the
            // bound ub_term recorded a value at or above it, so the minimum may
            // be the bound itself
            out = st.n0 + min(st.min_term, st.ub_term);
        }
        *pl.qd[q].count = out;
    }
}

}  // namespace td

extern "C" hipError_t td_launch_init(const td::Pools* pl, hipStream_t s) {
    hipLaunchKernelGGL(td::init_kernel, dim3(1), dim3(64), 0, s, pl->ctr);
    return hipGetLastError();
}

extern "C" hipError_t td_launch_prep(const td::Pools* pl, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(td::prep_kernel, dim3(blocks), dim3(256), 0, s, *pl);
    return hipGetLastError();
}

extern "C" hipError_t td_launch_finalize(const td::Pools* pl, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(td::finalize_kernel, dim3(blocks), dim3(256), 0, s, *pl);
    return hipGetLastError();
}
