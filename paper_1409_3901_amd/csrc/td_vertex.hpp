// The vertex form of the depth count: Proposition 1 with r = p - 1 (the
// instance that the critical-direction algorithm of Dyckerhoff and
// Mozharovskyi rests on, Section 2).  For a (p-1)-subset J of the nonzero
// centred points, S_J = span(x_J) is a hyperplane through the query with
// normal u_J, the generalised cross product of the columns x_J (their
// cofactors), and n D_n(S_J) is the smaller of the two closed half-space
// counts it bounds.  With the sample and the query in general position the
// only points on S_J are the p - 1 points of J, so
//     n D_n(0) = n0 + min over J of min(#{x : u_J.x > 0}, #{x : u_J.x < 0}),
// O(n^p) work: an independent check of the (p-2)-subset sweep.
//
// Arithmetic: float64 with a certified error bound.  The cofactors come from
// a Laplace expansion by columns over row subsets (minors of the first c
// columns from those of the first c - 1), evaluated together with the same
// expansion over absolute values, perm(|A|) by row subset.  A minor over c
// columns is a sum of c products of an entry and a minor over c - 1 columns;
// by induction its computed value errs by at most gamma_2c perm(|A_R|)
// (gamma_n = n u / (1 - n u), u = 2^-53).  The side of a point x is the sign
// of sum_k x_k u_k, within gamma_p sum |x_k| |u_k| of the computed sum; with
// the cofactor error that is gamma_3p sum |x_k| perm_k.  The centred points
// are float64 roundings of X - z (relative error u per coordinate), which
// moves the p x p determinant by at most gamma_p sum |x_k| perm_k more.  The
// computed permanents and the computed bound are themselves within
// (1 -+ gamma) of the true ones; the bound below takes gamma_{5p+4} and a
// factor 1.01 over the computed sum.  A point inside that bound is not
// decided: the query then reports TD_DEV_NOT_GENERAL (the data are not in
// the general position that Proposition 1 assumes, or too close to it for
// float64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace td {

__host__ __device__ constexpr double vertex_gamma(int n) {
    return (double)n * 0x1p-53 / (1.0 - (double)n * 0x1p-53);
}

// Bound factor of the side test at dimension P: |computed - exact| of
// sum_k x_k u_k is at most vertex_err_factor<P>() * sum_k |x_k| b_k.
template <int P>
__host__ __device__ constexpr double vertex_err_factor() {
    return 1.01 * vertex_gamma(5 * P + 4);
}

__host__ __device__ constexpr int vertex_popcount(int v) {
    return v == 0 ? 0 : (v & 1) + vertex_popcount(v >> 1);
}

// Cofactors of the P x (P-1) matrix A whose columns are the points of J:
// u[k] = (-1)^k det(A without row k) (one global sign for every J, which the
// count ignores), and b[k] the permanent of |A| without row k.  Row subsets
// are bit masks; m[mask] holds the minor of those rows and the first
// popcount(mask) columns.
template <int P>
__host__ __device__ inline void vertex_cofactors(const double (&A)[P][P > 1 ? P - 1 : 1], double (&u)[P],
                                                 double (&b)[P]) {
    constexpr int NM = 1 << P;
    double m[NM], a[NM];
    m[0] = 1.0;
    a[0] = 1.0;
#pragma unroll
    for (int c = 1; c < P; ++c) {
#pragma unroll
        for (int mask = 1; mask < NM; ++mask) {
            if (vertex_popcount(mask) != c) continue;
            // expansion along column c - 1: the i-th row of the mask (in
            // increasing order) carries the sign (-1)^(i + c - 1)
            double s = 0.0, t = 0.0;
            int i = 0;
#pragma unroll
            for (int r = 0; r < P; ++r) {
                if (!((mask >> r) & 1)) continue;
                const double e = A[r][c - 1];
                const double term = e * m[mask ^ (1 << r)];
                s = ((i + c - 1) & 1) ? s - term : s + term;
                t += (e < 0.0 ? -e : e) * a[mask ^ (1 << r)];
                ++i;
            }
            m[mask] = s;
            a[mask] = t;
        }
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int mask = (NM - 1) ^ (1 << k);
        u[k] = (k & 1) ? -m[mask] : m[mask];
        b[k] = a[mask];
    }
}

// Side of x against the hyperplane with cofactors (u, b): +1 or -1 when
// certified, 0 when the computed value lies within the error bound.
template <int P>
__host__ __device__ inline int vertex_side(const double (&x)[P], const double (&u)[P], const double (&b)[P]) {
    double v = 0.0, e = 0.0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        v += x[k] * u[k];
        e += (x[k] < 0.0 ? -x[k] : x[k]) * b[k];
    }
    e *= vertex_err_factor<P>();
    return v > e ? 1 : (v < -e ? -1 : 0);
}

}  // namespace td
