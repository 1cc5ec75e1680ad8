// Small device helpers: wave/block reductions, padded stores, scans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

// Instantiate CALL(P) for the spline degrees the library is built for.
#define ECPIC_DISPATCH(P, CALL) \
    switch (P) {                \
        case 2: CALL(2); break; \
        case 3: CALL(3); break; \
        case 4: CALL(4); break; \
        case 5: CALL(5); break; \
    }

namespace ecpic {

constexpr int WAVE = 64;
constexpr int MAX_BLOCK = 256;
constexpr int MAX_WAVES = MAX_BLOCK / WAVE;

__device__ __forceinline__ double dbits(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ unsigned long long bitsd(double v) { return (unsigned long long)__double_as_longlong(v); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Cross-lane moves by DPP (no LDS).  Rows disabled by ROWMASK read as 0.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave in a fixed order, returned to every lane
// (quad swaps, half-row and row mirrors, then the two row broadcasts that leave
// the total in lane 63).  All lanes must be active.
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_d<0xB1>(v);         // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);         // quad_perm [2,3,0,1]
    v += dpp_d<0x141>(v);        // row_half_mirror
    v += dpp_d<0x140>(v);        // row_mirror
    v += dpp_d<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_d<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return readlane_d(v, WAVE - 1);
}

// Max over the wave (arguments >= 0), returned to every lane.
__device__ __forceinline__ double wave_max_dpp(double v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x141>(v));
    v = fmax(v, dpp_d<0x140>(v));
    v = fmax(v, dpp_d<0x142, 0xA>(v));
    v = fmax(v, dpp_d<0x143, 0xC>(v));
    return readlane_d(v, WAVE - 1);
}

// Sum NV per-thread values over the block in a fixed order; thread t < NV gets
// total t in out.  lds must hold MAX_WAVES * NV doubles.
template <int NV>
__device__ __forceinline__ double block_sum_slot(const double (&v)[NV], double *lds) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = wave_sum(v[i]);
        if (lane == 0) lds[wid * NV + i] = s;
    }
    __syncthreads();
    double out = 0.0;
    if ((int)threadIdx.x < NV) {
        for (int w = 0; w < nw; ++w) out += lds[w * NV + threadIdx.x];
    }
    __syncthreads();
    return out;
}

// OR over the wave of flag words of the low NB bits, one ballot per bit (no
// cross-lane data movement).  All lanes must be active.
template <int NB = 3>
__device__ __forceinline__ int wave_or_bits(int v) {
    int r = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b)
        if (__builtin_amdgcn_ballot_w64((v >> b) & 1)) r |= 1 << b;
    return r;
}

// Max and OR (of flag bits) over the block; result valid in thread 0.  All
// lanes must be active.
__device__ __forceinline__ void block_max_or(double &m, int &f, double *ldsd, int *ldsi) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
    m = wave_max_dpp(m);
    f = wave_or_bits(f);
    if (lane == 0) { ldsd[wid] = m; ldsi[wid] = f; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nw; ++w) { m = fmax(m, ldsd[w]); f |= ldsi[w]; }
    }
    __syncthreads();
}

// Set flag bit f for the whole wave if cond holds in any active lane (the
// flags are OR-reduced per wave anyway; the test stays in the scalar unit).
__device__ __forceinline__ void wave_flag(int &flags, bool cond, int f) {
    if (__builtin_amdgcn_ballot_w64(cond)) flags |= f;
}

// Status of a substep about to start; gate_src (the substep it follows) must
// have committed without a flag, else every kernel of this substep skips.
__device__ __forceinline__ void init_status(DevStatus *st, const DevStatus *gate_src) {
    st->rx_bits[0] = 0ull;
    st->rx_bits[1] = 0ull;
    st->re_bits[0] = 0ull;
    st->re_bits[1] = 0ull;
    st->kconv = -1;
    st->committed = 0;
    st->flags = 0;
    st->fp32_sweeps = 0;
    st->scan_multi = 0;
    st->queued = 0;
    st->res = 0.0;
    for (int i = 0; i < 4; ++i) st->res_first[i] = 0.0;
    st->gate = gate_src ? (gate_src->committed && gate_src->flags == 0) : 1;
}

// Write v as coefficient j in [0, M) of a padded periodic array (all aliases).
__device__ __forceinline__ void store_padded(double *f, int M, int j, double v) {
    const int r = (HALO + M - 1) / M;
    for (int q = -r; q <= r; ++q) {
        int idx = j + q * M;
        if (idx >= -HALO && idx < M + HALO) f[idx + HALO] = v;
    }
}

// j mod M in [0, M); one compare and add for j in [-M, 2M), a division only
// beyond (an integer division is tens of instructions).
__device__ __forceinline__ int imod(int j, int M) {
    const int w = j < 0 ? j + M : (j >= M ? j - M : j);
    if (w >= 0 && w < M) return w;
    const int r = j % M;
    return r < 0 ? r + M : r;
}

// Exclusive scan of one int per thread over a block of blockDim.x <= 1024
// threads; returns the exclusive prefix, *total gets the block sum.  Each wave
// scans its values, then every thread adds the wave totals before its own.
__device__ __forceinline__ int block_exscan(int v, int *lds /* >= 16 */, int *total) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
    int x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int y = __shfl_up(x, o, WAVE);
        if (lane >= o) x += y;
    }
    if (lane == WAVE - 1) lds[wid] = x;
    __syncthreads();
    int pre = 0, sum = 0;
#pragma unroll
    for (int w = 0; w < 1024 / WAVE; ++w) {
        const int t = w < nw ? lds[w] : 0;
        pre += w < wid ? t : 0;
        sum += t;
    }
    *total = sum;
    __syncthreads();   // lds may be reused after the return
    return pre + x - v;
}

// Neighbours of cell c in [0, M) on the periodic grid (no division).
__device__ __forceinline__ int cell_prev(int c, int M) { return c == 0 ? M - 1 : c - 1; }
__device__ __forceinline__ int cell_next(int c, int M) { return c == M - 1 ? 0 : c + 1; }

// Items of a cell of n particles: ceil(n / chunk), 0 for an empty cell.
__device__ __forceinline__ int items_of(int n, int chunk) {
    return n <= chunk ? (n > 0 ? 1 : 0) : (n + chunk - 1) / chunk;
}

// Build an item list from per-cell counts (single block): cell c gets
// ceil(count[c] / chunk) items of near-equal size.  start[c] must hold the
// exclusive scan of counts, start[M] = N.  Returns the item count (in every
// thread).
__device__ inline int build_items(const int32_t *count, const int32_t *start, int M, int chunk, int64_t N,
                                  ItemList out, int *lds) {
    // items per cell, exclusive scan -> cell_first
    const int per = (M + blockDim.x - 1) / blockDim.x;
    const int c0 = threadIdx.x * per;
    int local = 0, one_each = 1;
    for (int c = c0; c < c0 + per && c < M; ++c) {
        const int ni = items_of(count[c], chunk);
        local += ni;
        one_each &= ni == 1;
    }
    one_each = __syncthreads_and(one_each);
    int total;
    int off = block_exscan(local, lds, &total);
    for (int c = c0; c < c0 + per && c < M; ++c) {
        const int n = count[c];
        const int ni = items_of(n, chunk);
        out.cell_first[c] = off;
        if (ni > 0) {
            out.cell[off] = c;
            out.begin[off] = start[c];
        }
        for (int q = 1; q < ni; ++q) {
            out.cell[off + q] = c;
            out.begin[off + q] = start[c] + (int)(((int64_t)n * q) / ni);
        }
        off += ni;
    }
    if (threadIdx.x == 0) {
        out.cell_first[M] = total;
        out.begin[total] = (int)N;
        out.n_items[0] = total;
        out.n_items[1] = one_each;   // item c is cell c's only item
    }
    return total;
}

// Exclusive scan of count[0..M) into start[0..M] (single block).
__device__ inline void scan_cells(const int32_t *count, int32_t *start, int M, int *lds) {
    const int per = (M + blockDim.x - 1) / blockDim.x;
    const int c0 = threadIdx.x * per;
    int local = 0;
    for (int c = c0; c < c0 + per && c < M; ++c) local += count[c];
    int total;
    int off = block_exscan(local, lds, &total);
    for (int c = c0; c < c0 + per && c < M; ++c) { start[c] = off; off += count[c]; }
    if (threadIdx.x == 0) start[M] = total;
}

}  // namespace ecpic
