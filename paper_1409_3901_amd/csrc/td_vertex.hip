// The vertex-form check (td_options.method = TD_METHOD_VERTEX): Proposition 1
// with r = p - 1 on the device.  One wave per workgroup, persistent over the
// work items of its class (chunks of colex ranks of (p-1)-subsets of one
// query): every lane builds the cofactors of one subset of a batch of 64,
// then the wave counts the sides of every point of the query for each of
// them.  No scratch buffers: the subsets' cofactors live in LDS, the points
// in registers (8 per lane, n <= 512; 16 per lane, n <= 1024, at p <= 4).
#include <hip/hip_runtime.h>

#include "td_device.hpp"
#include "td_vertex.hpp"

namespace td {

template <int P>
struct VertexSlot {
    double u[P];    // cofactors of the subset (the hyperplane's normal)
    double b[P];    // their permanents (error bound)
    int16_t mem[P > 1 ? P - 1 : 1];
    int32_t state;  // 0: subset of the batch, 1: past the item
};

template <int P, int K>
__global__ __launch_bounds__(64) void vertex_kernel(Pools pl) {
    constexpr int KS = P - 1;
    __shared__ VertexSlot<P> slots[64];
    const int lane = lane_id();
    const uint64_t cbeg = pl.cp->cls_begin[pl.cls];
    const uint64_t cend = pl.cp->cls_end[pl.cls];
    const uint32_t chunk = pl.cp->cls_chunk[pl.cls];
    const int nq = pl.cp->num_queries;
    unsigned long long swept = 0;
    // block b takes item b first, then the shared counter the items past the grid
    bool first = true;
    while (true) {
        unsigned long long item = 0;
        if (first) {
            item = cbeg + blockIdx.x;
            first = false;
        } else {
            if (cbeg + gridDim.x >= cend) break;
            if (lane == 0) item = cbeg + gridDim.x + atomicAdd(&pl.ctr->work_next[pl.cls], 1ull);
            item = uni64(__shfl(item, 0, 64));
        }
        if (item >= cend) break;
        const int q = uni(item_query(pl.qd, nq, item));
        const QueryDesc d = pl.qd[q];
        const QueryState st = pl.qs[q];
        if (st.status & kStNonfinite) continue;
        const int nnz = uni(st.nnz);
        const uint64_t nsub = uni64(binom_lookup(pl.binom, nnz, KS));
        const uint64_t r0 = uni64((item - d.item_begin) * (uint64_t)chunk);
        const uint64_t r1 = uni64(min(r0 + (uint64_t)chunk, nsub));
        if (r0 >= r1) continue;
        const double* x64 = pl.x64 + d.v_off;
        int wbest = 0x7fffffff;
        bool undecided = false;
        for (uint64_t rb = r0; rb < r1; rb += 64) {
            const uint64_t myr = rb + (uint64_t)lane;
            VertexSlot<P>& my = slots[lane];
            if (myr < r1) {
                int cc[KS > 0 ? KS : 1];
                cc[0] = 0;
                unrank_colex<KS>(pl.binom, myr, nnz, cc);
                double A[P][KS > 0 ? KS : 1];
#pragma unroll
                for (int col = 0; col < KS; ++col)
#pragma unroll
                    for (int r = 0; r < P; ++r) A[r][col] = x64[(size_t)cc[col] * P + r];
                double u[P], b[P];
                vertex_cofactors<P>(A, u, b);
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    my.u[k] = u[k];
                    my.b[k] = b[k];
                }
#pragma unroll
                for (int col = 0; col < KS; ++col) my.mem[col] = (int16_t)cc[col];
                my.state = 0;
            } else {
                my.state = 1;
            }
            __syncthreads();
            // the query's points (rows past nnz are zero and not counted),
            // loaded per batch so that they are not live while the cofactors
            // are built
            double xr[K][P];
#pragma unroll
            for (int i = 0; i < K; ++i)
#pragma unroll
                for (int c = 0; c < P; ++c) xr[i][c] = x64[(size_t)(lane * K + i) * P + c];
            const int cnt = (int)min((uint64_t)64, r1 - rb);
            for (int s = 0; s < cnt; ++s) {
                const VertexSlot<P>& S = slots[s];
                double u[P], b[P];
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    u[k] = S.u[k];
                    b[k] = S.b[k];
                }
                int mem[KS > 0 ? KS : 1];
#pragma unroll
                for (int c = 0; c < KS; ++c) mem[c] = S.mem[c];
                int npos = 0, nneg = 0;
                bool unc = false;
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const int idx = lane * K + i;
                    bool valid = idx < nnz;
#pragma unroll
                    for (int c = 0; c < KS; ++c) valid = valid && (idx != mem[c]);
                    const int side = vertex_side<P>(xr[i], u, b);
                    npos += __popcll(__ballot(valid && side > 0));
                    nneg += __popcll(__ballot(valid && side < 0));
                    unc = unc || (valid && side == 0);
                }
                if (__any(unc)) undecided = true;
                wbest = min(wbest, min(npos, nneg));
                ++swept;
            }
            __syncthreads();
        }
        if (lane == 0) {
            if (wbest < 0x7fffffff) atomicMin(&pl.qs[q].min_term, wbest);
            if (undecided) atomicOr(&pl.qs[q].status, kStNotGeneral);
        }
    }
    if (lane == 0 && swept) atomicAdd(&pl.ctr->swept, swept);
}

}  // namespace td

namespace {
typedef void (*KernelFn)(td::Pools);

template <int P>
KernelFn pick_k(int K) {
    switch (K) {
        case 1: return td::vertex_kernel<P, 1>;
        case 2: return td::vertex_kernel<P, 2>;
        case 4: return td::vertex_kernel<P, 4>;
        case 8: return td::vertex_kernel<P, 8>;
        case 16:
            if constexpr (P <= 4) return td::vertex_kernel<P, 16>;
            return nullptr;
    }
    return nullptr;
}

KernelFn pick(int P, int K) {
    switch (P) {
        case 2: return pick_k<2>(K);
        case 3: return pick_k<3>(K);
        case 4: return pick_k<4>(K);
        case 5: return pick_k<5>(K);
        case 6: return pick_k<6>(K);
        case 7: return pick_k<7>(K);
        case 8: return pick_k<8>(K);
    }
    return nullptr;
}
}  // namespace

// Blocks of the (P, K) vertex kernel one compute unit holds (0 if none).
extern "C" int td_resident_blocks_vertex(int P, int K) {
    KernelFn f = pick(P, K);
    int n = 0;
    if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64, 0) != hipSuccess) return 0;
    return n;
}

extern "C" hipError_t td_launch_vertex(int P, int K, int blocks, hipStream_t s, const td::Pools* pl) {
    KernelFn f = pick(P, K);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(blocks), dim3(64), 0, s, *pl);
    return hipGetLastError();
}
