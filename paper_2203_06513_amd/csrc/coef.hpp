// Per-cell polynomial coefficient tables.
//
// Every particle block works on one cell c, so every field it needs is a fixed
// polynomial in the particle's local coordinate t.  These tables hold, per cell,
//   A-record  (2 (P+1) doubles): A_y(t), A_z(t) = sum_i a[i] t^i on the cell,
//             a[i] = sum_m a_{c-m} c[m][i]  (V0 pieces of degree P);
//   E-record  (P doubles): weights of the V1 piece means of a V1 field e,
//             mean of e over [a, b] = sum_i w[i] h_i(a, b),  w[i] = sum_m e_{c-m} q[m][i]
//             (V1 pieces of degree P-1, q = c/(i+1)).
// With them the gathers, the divided differences (A(b) - A(a))/(b - a) =
// sum_{i>=1} a[i] h_{i-1}(a, b) and the line means of Subsystem I become a few
// Horner / dot steps per particle, with coefficients loaded once per block.
// Tables carry one padding record on each side (record r <-> cell r - 1,
// periodic), so cells c-1, c, c+1 are three consecutive records.
#pragma once

#include "common.hpp"
#include "spline.hpp"

namespace ecpic {

template <int P>
struct RecA {
    static constexpr int N = 2 * (P + 1);
};
template <int P>
struct RecE {
    static constexpr int N = P;
};

__device__ __forceinline__ int rec_index(int c) { return c + 1; }

// Write record of cell c (and its periodic padding alias) into table t with
// record size n.
__device__ __forceinline__ void store_record(double *t, int M, int c, int n, int i, double v) {
    t[(size_t)rec_index(c) * n + i] = v;
    if (c == M - 1) t[(size_t)0 * n + i] = v;
    if (c == 0) t[(size_t)(M + 1) * n + i] = v;
}

// A-record of cell c from padded V0 coefficient arrays.
template <int P>
__device__ __forceinline__ void make_recA(const double *ay, const double *az, int c, double (&ry)[P + 1],
                                          double (&rz)[P + 1]) {
    constexpr Pieces<P> B{};
#pragma unroll
    for (int i = 0; i <= P; ++i) {
        double sy = 0.0, sz = 0.0;
#pragma unroll
        for (int m = 0; m <= P; ++m) {
            sy += ay[c - m + HALO] * B.c[m][i];
            sz += az[c - m + HALO] * B.c[m][i];
        }
        ry[i] = sy;
        rz[i] = sz;
    }
}

template <int P, typename F>
__device__ __forceinline__ void make_recE(F e_at, int c, double (&r)[P]) {
    constexpr Pieces<P - 1> B{};
#pragma unroll
    for (int i = 0; i < P; ++i) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < P; ++m) s += e_at(c - m) * B.q[m][i];
        r[i] = s;
    }
}

template <int N, typename T>
__device__ __forceinline__ T horner(const T *c, T t) {
    T v = c[N - 1];
#pragma unroll
    for (int i = N - 2; i >= 0; --i) v = fma(v, t, c[i]);
    return v;
}

// (A(b) - A(a))/(b - a) for A = sum_{i=0}^{P} c_i t^i, given h_0..h_{P-1} of (a, b).
// (h_0 = 1 for every pair, so the sums start from the first coefficient.)
template <int P, typename T>
__device__ __forceinline__ T divdiff(const T *c, const T (&h)[P]) {
    T v = c[1];
#pragma unroll
    for (int i = 2; i <= P; ++i) v = fma(c[i], h[i - 1], v);
    return v;
}

// (A'(b) - A'(a))/(b - a) for A = sum_{i=0}^{P} c_i t^i, A' = dA/dt, given h_0..h_{P-1}
// of (a, b): sum_{i=2}^{P} i c_i h_{i-2}.
template <int P, typename T>
__device__ __forceinline__ T divdiff2(const T *c, const T (&h)[P]) {
    T v = (T)2 * c[2];
#pragma unroll
    for (int i = 3; i <= P; ++i) v = fma((T)i * c[i], h[i - 2], v);
    return v;
}

template <int P, typename T>
__device__ __forceinline__ T pmean(const T *w, const T (&h)[P]) {
    T v = w[0];
#pragma unroll
    for (int i = 1; i < P; ++i) v = fma(w[i], h[i], v);
    return v;
}

// Reciprocal and square root accurate to a few ulp without the IEEE range
// handling (arguments here are positive and O(1)); Newton / Goldschmidt steps
// refine the hardware approximations.
#ifdef ECPIC_IEEE_DIVSQRT
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ double fsqrt(double q) { return sqrt(q); }
#else
__device__ __forceinline__ double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double fsqrt(double q) {   // q >= 1
    // two Newton steps on the root from the hardware reciprocal square root y
    // (relative error e): s = q y, then s += (q - s^2) h with h = y / 2 fixed;
    // the error goes e -> ~e^2 -> ~e^3, below rounding
    const double y = __builtin_amdgcn_rsq(q);
    const double h = 0.5 * y;
    double s = q * y;
    s = fma(fma(-s, s, q), h, s);
    return fma(fma(-s, s, q), h, s);
}
#endif

// One particle of a Subsystem II iterate (Section 4.2): the deposit
// coefficients c = (A^(k) + A^n)/(gamma^n + gamma^(k)) at local coordinate t0
// with momentum p0; any, anz (ak*) are the cell's polynomial coefficients of
// a^n (of a^(k)).
template <int P>
__device__ __forceinline__ void sub2_coef(const double *any, const double *anz, const double *aky, const double *akz,
                                          double t0, double p0, double &cy, double &cz) {
    const double Any = horner<P + 1>(any, t0), Anz = horner<P + 1>(anz, t0);
    const double Aky = horner<P + 1>(aky, t0), Akz = horner<P + 1>(akz, t0);
    const double q = fma(p0, p0, 1.0);
    const double gn = fsqrt(q + Any * Any + Anz * Anz);
    const double gk = fsqrt(q + Aky * Aky + Akz * Akz);
    const double inv = frcp(gn + gk);
    cy = (Aky + Any) * inv;
    cz = (Akz + Anz) * inv;
}

// Single precision: the hardware square root and reciprocal (about 1 ulp).
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float q) { return __builtin_amdgcn_sqrtf(q); }

}  // namespace ecpic
