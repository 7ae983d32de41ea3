// Fixed-width two's-complement integers for the exact tier (single lane).
//
// Inputs are the centred observations as exact integers below 2^125 in
// magnitude (two 64-bit words).  Every exact quantity of the method is a
// determinant of order <= p in such integers, or a product of two of them, so
// fixed widths derived from p suffice; no operation can overflow them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace td {

template <int NL>
struct BigI {
    uint32_t w[NL];   // little-endian two's complement
};

template <int NL>
__device__ inline void big_zero(BigI<NL>& a) {
    for (int i = 0; i < NL; ++i) a.w[i] = 0;
}

template <int NL>
__device__ inline bool big_is_zero(const BigI<NL>& a) {
    uint32_t o = 0;
    for (int i = 0; i < NL; ++i) o |= a.w[i];
    return o == 0;
}

template <int NL>
__device__ inline int big_sign(const BigI<NL>& a) {
    if ((int32_t)a.w[NL - 1] < 0) return -1;
    return big_is_zero(a) ? 0 : 1;
}

template <int NL>
__device__ inline void big_from_i128(BigI<NL>& a, uint64_t lo, uint64_t hi) {
    a.w[0] = (uint32_t)lo;
    a.w[1] = (uint32_t)(lo >> 32);
    a.w[2] = (uint32_t)hi;
    a.w[3] = (uint32_t)(hi >> 32);
    const uint32_t ext = ((int64_t)hi < 0) ? 0xffffffffu : 0u;
    for (int i = 4; i < NL; ++i) a.w[i] = ext;
}

template <int NL>
__device__ inline void big_from_int(BigI<NL>& a, int v) {
    const uint32_t ext = v < 0 ? 0xffffffffu : 0u;
    a.w[0] = (uint32_t)v;
    for (int i = 1; i < NL; ++i) a.w[i] = ext;
}

template <int NL>
__device__ inline void big_neg(BigI<NL>& a) {
    uint64_t c = 1;
    for (int i = 0; i < NL; ++i) {
        c += (uint64_t)(~a.w[i]);
        a.w[i] = (uint32_t)c;
        c >>= 32;
    }
}

template <int NL>
__device__ inline void big_add(BigI<NL>& a, const BigI<NL>& b) {
    uint64_t c = 0;
    for (int i = 0; i < NL; ++i) {
        c += (uint64_t)a.w[i] + b.w[i];
        a.w[i] = (uint32_t)c;
        c >>= 32;
    }
}

template <int NL>
__device__ inline void big_sub(BigI<NL>& a, const BigI<NL>& b) {
    BigI<NL> t = b;
    big_neg(t);
    big_add(a, t);
}

// |a| into mag (NL words), returns the sign (-1, 0, 1)
template <int NL>
__device__ inline int big_abs(const BigI<NL>& a, uint32_t* mag) {
    const int s = big_sign(a);
    if (s < 0) {
        uint64_t c = 1;
        for (int i = 0; i < NL; ++i) {
            c += (uint64_t)(~a.w[i]);
            mag[i] = (uint32_t)c;
            c >>= 32;
        }
    } else {
        for (int i = 0; i < NL; ++i) mag[i] = a.w[i];
    }
    return s;
}

// r = a * b (widths NA, NB -> NR); the caller sizes NR so the product fits.
template <int NR, int NA, int NB>
__device__ inline void big_mul(BigI<NR>& r, const BigI<NA>& a, const BigI<NB>& b) {
    uint32_t ma[NA], mb[NB];
    const int sa = big_abs(a, ma);
    const int sb = big_abs(b, mb);
    for (int i = 0; i < NR; ++i) r.w[i] = 0;
    if (sa == 0 || sb == 0) return;
    int la = NA, lb = NB;
    while (la > 0 && ma[la - 1] == 0) --la;
    while (lb > 0 && mb[lb - 1] == 0) --lb;
    for (int i = 0; i < la; ++i) {
        uint64_t c = 0;
        for (int j = 0; j < lb && i + j < NR; ++j) {
            const uint64_t t = (uint64_t)ma[i] * mb[j] + r.w[i + j] + c;
            r.w[i + j] = (uint32_t)t;
            c = t >> 32;
        }
        for (int k = i + lb; k < NR && c; ++k) {
            const uint64_t t = (uint64_t)r.w[k] + c;
            r.w[k] = (uint32_t)t;
            c = t >> 32;
        }
    }
    if (sa * sb < 0) big_neg(r);
}

// a += s * b * x (x a 128-bit two's-complement integer, s = +-1)
template <int NL>
__device__ inline void big_fma_i128(BigI<NL>& acc, const BigI<NL>& b, uint64_t xlo, uint64_t xhi, int s) {
    BigI<4> x;
    x.w[0] = (uint32_t)xlo;
    x.w[1] = (uint32_t)(xlo >> 32);
    x.w[2] = (uint32_t)xhi;
    x.w[3] = (uint32_t)(xhi >> 32);
    BigI<NL> t;
    big_mul<NL, NL, 4>(t, b, x);
    if (s < 0) big_neg(t);
    big_add(acc, t);
}

// Nearest-ish double (relative error below 2^-50) of a nonzero integer.
template <int NL>
__device__ inline double big_to_double(const BigI<NL>& a) {
    uint32_t m[NL];
    const int s = big_abs(a, m);
    if (s == 0) return 0.0;
    int top = NL - 1;
    while (top > 0 && m[top] == 0) --top;
    double v = 0.0;
    // three leading words give at least 65 significant bits
    for (int i = top; i >= 0 && i >= top - 2; --i) v = v * 4294967296.0 + (double)m[i];
    const int shift = 32 * (top >= 2 ? top - 2 : 0);
    v = ldexp(v, shift);
    return s < 0 ? -v : v;
}

}  // namespace td
