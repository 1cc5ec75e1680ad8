// Device-side B-spline pieces for the uniform periodic grid of Section 3.1.
//
// On cell c with local coordinate t in [0, 1), the degree-D splines that do not
// vanish are N^D_{c-m}(x) = B_D(t + m), m = 0..D.  Each piece is a polynomial,
// written here in monomials from the truncated-power form of the cardinal
// B-spline,
//     B_D(u) = 1/D! sum_{k=0}^{D+1} (-1)^k C(D+1, k) (u - k)_+^D,
// so on [m, m+1):  B_D(t + m) = sum_i c[m][i] t^i with
//     c[m][i] = C(D, i)/D! sum_{k=0}^{m} (-1)^k C(D+1, k) (m - k)^(D - i).
// The coefficients are generated at compile time; nothing here is shared with
// the CPU oracle (which evaluates splines by the Cox-de Boor recursion).
//
// Line means.  The Subsystem I scheme (Section 4.2) needs the time average
// of Lambda1 along the straight step x(tau), which for a step inside one cell
// from t = a to t = b is (Q(b) - Q(a))/(b - a) with Q the antiderivative of the
// piece.  For each monomial (b^(i+1) - a^(i+1)) / ((i+1)(b - a)) = h_i(a, b)/(i+1)
// with h_i(a, b) = sum_{j=0}^{i} a^j b^(i-j): a polynomial in (a, b), so the
// mean has no 0/0 when the step is tiny or zero (which the paper's first remark
// of Section 4.2 handles approximately).  A step that enters a neighbouring
// cell is split at the knot and the two piece means are combined with the
// length fractions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecpic {

constexpr int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

constexpr int64_t binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

constexpr int64_t factorial(int n) {
    int64_t r = 1;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

template <int D>
struct Pieces {
    double c[D + 1][D + 1];   // c[m][i]: coefficient of t^i of B_D(t + m)
    double q[D + 1][D + 1];   // q[m][i] = c[m][i] / (i + 1): weights of h_i in the line mean
    constexpr Pieces() : c{}, q{} {
        for (int m = 0; m <= D; ++m) {
            for (int i = 0; i <= D; ++i) {
                int64_t s = 0;
                for (int k = 0; k <= m; ++k) {
                    int64_t term = binom(D + 1, k) * ipow(m - k, D - i);
                    s += (k % 2 == 0) ? term : -term;
                }
                c[m][i] = (double)(binom(D, i) * s) / (double)factorial(D);
                q[m][i] = c[m][i] / (double)(i + 1);
            }
        }
    }
};

// B[m] = B_D(t + m), m = 0..D (the D+1 splines alive on the cell, index c - m).
template <int D, typename T>
__device__ __forceinline__ void basis_values(T t, T (&B)[D + 1]) {
    constexpr Pieces<D> P{};
#pragma unroll
    for (int m = 0; m <= D; ++m) {
        T v = (T)P.c[m][D];
#pragma unroll
        for (int i = D - 1; i >= 0; --i) v = v * t + (T)P.c[m][i];
        B[m] = v;
    }
}

// Complete homogeneous polynomials h_0..h_D of (a, b).
template <int D, typename T>
__device__ __forceinline__ void homog(T a, T b, T (&h)[D + 1]) {
    h[0] = (T)1;
    T ai = (T)1;
#pragma unroll
    for (int i = 1; i <= D; ++i) {
        ai = ai * a;
        h[i] = h[i - 1] * b + ai;
    }
}

// Mean over [a, b] (0 <= a <= b <= 1, possibly a == b) of B_D(t + m), m = 0..D.
template <int D, typename T>
__device__ __forceinline__ void piece_means(T a, T b, T (&avg)[D + 1]) {
    constexpr Pieces<D> P{};
    T h[D + 1];
    homog<D>(a, b, h);
#pragma unroll
    for (int m = 0; m <= D; ++m) {
        T v = (T)0;
#pragma unroll
        for (int i = 0; i <= D; ++i) v = v + (T)P.q[m][i] * h[i];
        avg[m] = v;
    }
}

// Geometry of a step from t0 in [0, 1) of cell c to t1 in (-1, 2) (c frame):
// the main piece stays in cell c, the side piece (if any) lies in cell c + s.
// sA, sB are the signed lengths of the pieces, [aA, bA] and [aB, bB] their
// (unsigned) extents in the local coordinate of their own cell.
template <typename T>
struct Seg {
    T aA, bA, sA, aB, bB, sB;
};

template <typename T>
__device__ __forceinline__ Seg<T> make_seg(T t0, T t1, int s) {
    const T one = (T)1, zero = (T)0;
    Seg<T> g;
    const T t1c = t1 < zero ? zero : (t1 > one ? one : t1);
    g.aA = t0 < t1c ? t0 : t1c;
    g.bA = t0 < t1c ? t1c : t0;
    g.sA = t1c - t0;
    g.aB = s > 0 ? zero : (s < 0 ? t1 + one : zero);
    g.bB = s > 0 ? t1 - one : (s < 0 ? one : zero);
    g.sB = t1 - t1c;
    return g;
}

// Integrals of the V1 basis (degree P-1) along a step, in cell units:
// I[k] = int Lambda1_{c-P+k} dxi, k = 0..P+1, as the signed piece lengths times
// the piece means (the same formulas the sweep accumulates as moments).
template <int P, typename T>
__device__ __forceinline__ void segment_integrals(T t0, T t1, int s, T (&I)[P + 2]) {
    constexpr int D = P - 1;
    constexpr Pieces<D> Q{};
    const Seg<T> g = make_seg(t0, t1, s);
    T hA[D + 1], hB[D + 1];
    homog<D>(g.aA, g.bA, hA);
    homog<D>(g.aB, g.bB, hB);
#pragma unroll
    for (int k = 0; k <= P + 1; ++k) I[k] = (T)0;
#pragma unroll
    for (int m = 0; m <= D; ++m) {
        T vA = (T)0, vB = (T)0;
#pragma unroll
        for (int i = 0; i <= D; ++i) { vA += (T)Q.q[m][i] * hA[i]; vB += (T)Q.q[m][i] * hB[i]; }
        I[P - m] += g.sA * vA;                  // index c - m
        if (s > 0) I[P + 1 - m] += g.sB * vB;   // index c + 1 - m
        if (s < 0) I[P - 1 - m] += g.sB * vB;   // index c - 1 - m
    }
}

}  // namespace ecpic
