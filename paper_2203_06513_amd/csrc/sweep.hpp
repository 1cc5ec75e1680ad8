// Pieces shared by the particle passes of Subsystem I (the sweeps in sub1.hip
// and the warm-start predictor in mlp.hip): the moments of the current
// deposit, step end points, the per-wave reduction into partial slots, and the
// split of an item's rows among the waves of a block.
#pragma once

#include "coef.hpp"

namespace ecpic {

template <int P>
struct Moments {
    double A[P], R[P], L[P];   // sum over particles of (signed piece length) h_i(piece)
};

// End point of a step: xi0 in [c, c+1), t1 = (xi0 + d) - c is exact in floating
// point, so the committed position and the deposited segment agree.  A step of
// a cell or more (or NaN) is flagged and its end point clamped into (-1, 2),
// which leaves every valid one unchanged and keeps the neighbour index in range.
__device__ __forceinline__ void end_point(double xi0, double d, int c, double &t1, int &s, int &flags) {
    t1 = (xi0 + d) - (double)c;
    wave_flag(flags, !(fabs(t1 - 0.5) < 1.5), FLAG_CFL);
    t1 = fmin(fmax(t1, -0.99999999999999989), 1.9999999999999998);
    s = (int)floor(t1);
}

// The P+2 V1 slots of the wave's particles (slot q <-> V1 index c - P + q):
// each lane converts its own moments (linear, cell c: m = P - q, c+1:
// m = P + 1 - q, c-1: m = P - 1 - q), the P+2 values are summed over the
// wave, and lane q < P+2 returns slot q.
template <int P>
__device__ __forceinline__ double moments_to_slots(const Moments<P> &mo) {
    constexpr Pieces<P - 1> Q{};
    double v[P + 2];
#pragma unroll
    for (int q = 0; q < P + 2; ++q) {
        double s = 0.0;
#pragma unroll
        for (int ii = 0; ii < P; ++ii) {
            if (P - q >= 0 && P - q < P) s = fma(Q.q[P - q < P ? P - q : 0][ii], mo.A[ii], s);
            if (P + 1 - q >= 0 && P + 1 - q < P) s = fma(Q.q[P + 1 - q < P ? P + 1 - q : 0][ii], mo.R[ii], s);
            if (P - 1 - q >= 0 && P - 1 - q < P) s = fma(Q.q[P - 1 - q >= 0 ? P - 1 - q : 0][ii], mo.L[ii], s);
        }
        v[q] = wave_sum_dpp(s);
    }
    const int lane = threadIdx.x & (WAVE - 1);
    double out = 0.0;
#pragma unroll
    for (int q = 0; q < P + 2; ++q) out = lane == q ? v[q] : out;
    return out;
}

// Values per wave in the partials of a sweep: P+2 current slots, the residual
// max and the flags.
template <int P>
struct UnitI {
    static constexpr int N = P + 4;
};

// The rows (64 particles) of an item are split into nw contiguous runs, one per
// wave of the block, so that a wave's particles are consecutive in the sorted
// order (the commit relies on it to keep the order stable).
__device__ __forceinline__ void wave_range(int beg, int end, int wid, int nw, int &wb, int &we) {
    const int rows = (end - beg + WAVE - 1) / WAVE;
    const int rpw = (rows + nw - 1) / nw;
    wb = min(beg + wid * rpw * WAVE, end);
    we = min(wb + rpw * WAVE, end);
}

// Cell-local end point and cell change of a step (single precision sweeps).
__device__ __forceinline__ void end_point(float t0, float d, float &t1, int &s, int &flags) {
    t1 = t0 + d;
    wave_flag(flags, !(fabsf(t1 - 0.5f) < 1.5f), FLAG_CFL);
    t1 = fminf(fmaxf(t1, -0.99999994f), 1.9999999f);
    s = (int)floorf(t1);
}

// Single precision moments with Knuth's TwoSum compensation: every product and
// every addition leaves its rounding error in the companion sum.
template <int P>
struct Moments32 {
    float A[P], R[P], L[P];
    float cA[P], cR[P], cL[P];
};

__device__ __forceinline__ void acc_two_sum(float &s, float &c, float a, float b) {
#pragma clang fp contract(off)
    const float x = a * b;
    const float ex = fmaf(a, b, -x);
    const float t = s + x;
    const float bp = t - s;
    const float e = (s - (t - bp)) + (x - bp);
    s = t;
    c += e + ex;
}

__device__ __forceinline__ void acc(double &s, double a, double b) { s = fma(a, b, s); }

template <int P>
__device__ __forceinline__ void acc_A(Moments<P> &mo, int i, double a, double b) { acc(mo.A[i], a, b); }
template <int P>
__device__ __forceinline__ void acc_R(Moments<P> &mo, int i, double a, double b) { acc(mo.R[i], a, b); }
template <int P>
__device__ __forceinline__ void acc_L(Moments<P> &mo, int i, double a, double b) { acc(mo.L[i], a, b); }
template <int P>
__device__ __forceinline__ void acc_A(Moments32<P> &mo, int i, float a, float b) { acc_two_sum(mo.A[i], mo.cA[i], a, b); }
template <int P>
__device__ __forceinline__ void acc_R(Moments32<P> &mo, int i, float a, float b) { acc_two_sum(mo.R[i], mo.cR[i], a, b); }
template <int P>
__device__ __forceinline__ void acc_L(Moments32<P> &mo, int i, float a, float b) { acc_two_sum(mo.L[i], mo.cL[i], a, b); }

// Moments of a step from t0 to t1 (end in cell c + s); scale 0 drops it.
template <int P, typename T, typename MO>
__device__ __forceinline__ void stage_deposit(MO &mo, bool anycross, T t0, T t1, int s, T scale) {
    const T zero = (T)0, one = (T)1;
    const T t1c = fmin(fmax(t1, zero), one);
    T h[P];
    homog<P - 1>(fmin(t0, t1c), fmax(t0, t1c), h);
    const T sA = scale * (t1c - t0);
#pragma unroll
    for (int i = 0; i < P; ++i) acc_A<P>(mo, i, sA, h[i]);
    if (anycross) {
        const T tl = t1 - (T)s;
        homog<P - 1>(s > 0 ? zero : (s < 0 ? tl : zero), s > 0 ? tl : (s < 0 ? one : zero), h);
        const T sB = scale * (t1 - t1c);
        const T sr = s > 0 ? sB : zero, sl = s < 0 ? sB : zero;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            acc_R<P>(mo, i, sr, h[i]);
            acc_L<P>(mo, i, sl, h[i]);
        }
    }
}

}  // namespace ecpic
