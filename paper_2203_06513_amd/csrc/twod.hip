// Reduced 2D model (Sections 2.2, 3.2 and 4.3), without and with the spin terms
// (hbar): kernels, spectral solves and the C ABI of include/ecpic2d.h.
//
// Data layout in HBM (one context):
//   particles  SoA, grouped by tile (TW cells of one row) in tile order, double
//              buffered: xi_k = x_k / dx_k in [0, M_k) (f64), p1, p2 (f64), id
//              (i32, the index given at set_particles).  Inside a tile the
//              cell-sorted sequence is stored transposed (see tile_pos), so a
//              coalesced read hands the lanes of a wave particles of different
//              cells.  start[c] is where cell c's share of its tile begins in the
//              sorted count (start[first cell of a tile] is the tile's offset).
//              The Picard iterate d = x^{n+1} - x^n (physical units) and p^{k+1}
//              live in more buffers; with spin, sx, sy, sz (f64) are double
//              buffered with the particles.
//   fields     row-major M1 x M2 coefficient grids, index i1 M2 + i2 (no halo;
//              the tile kernels wrap indices while staging).
//   spectra    M1 x M2 complex grids for the linear solves.
//
// Tiles.  A tile is TW consecutive cells of one row (x1 fixed); its particles
// are contiguous in the sorted order.  One thread block per tile stages the
// field coefficients the tile's particles can touch (rows r-p-1 .. r+1, columns
// c0-p-1 .. c0+TW, enough for a step of less than one cell) in LDS, gathers
// from there, accumulates its deposits in LDS with atomics, and adds the patch
// to the global grid with atomics at the end.
//
// Linear solves.  Every linear operator of the 2D scheme is a sum of tensor
// products of circulants (periodic B-spline mass matrices and differences), so
// the 2D discrete Fourier transform diagonalises it: M1, M0 + dt^2 K/4 and the
// Maxwell system are solved exactly by a forward transform, a division by the
// symbol and an inverse transform.  The transforms are Stockham FFTs with the
// values in registers (radix 8) and LDS between stages (rows in one kernel,
// columns with the spectral step fused in the next, inverse rows with an
// epilogue).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/ecpic2d.h"
#include "coef.hpp"
#include "common.hpp"
#include "spline.hpp"

namespace ecpic2d {

using ecpic::basis_values;
using ecpic::frcp;
using ecpic::fsqrt;
using ecpic::piece_means;
using ecpic::wave_sum_dpp;

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int TWMAX = 64;        // tile width (cells along x2)
constexpr int MAXM = 512;        // largest grid size per direction (LDS of the transforms)
constexpr int MAXK = 64;         // residual slots per substep (Picard cap)
constexpr int FLAG_NONFINITE = 1, FLAG_CFL = 2;

__device__ __forceinline__ int wrapi(int j, int M) {
    const int w = j < 0 ? j + M : (j >= M ? j - M : j);
    if (w >= 0 && w < M) return w;
    const int r = j % M;
    return r < 0 ? r + M : r;
}

__device__ __forceinline__ unsigned long long bitsd(double v) { return (unsigned long long)__double_as_longlong(v); }

// Max of v >= 0 over the block, then one atomic max (as bits) into *slot.
__device__ __forceinline__ void block_max_to(double v, unsigned long long *slot) {
    __shared__ double red[BLOCK / WAVE];
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < (int)(blockDim.x / WAVE); ++w) m = fmax(m, red[w]);
        if (m > 0.0) atomicMax(slot, bitsd(m));
    }
}

// Sum over the block in a fixed order; thread 0 writes it to *out.
__device__ __forceinline__ void block_sum_to(double v, double *out) {
    __shared__ double red[BLOCK / WAVE];
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) s += red[w];
        *out = s;
    }
}

// Block -> tile, keeping each XCD (blocks are dealt to the 8 XCDs round robin)
// on a contiguous band of rows so neighbouring tiles share its L2.
__device__ __forceinline__ int tile_of_block() {
    const int b = blockIdx.x, n = gridDim.x;
    if (n % 8 != 0) return b;
    return (b % 8) * (n / 8) + b / 8;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

// Number of lanes below this one set in mask.
__device__ __forceinline__ int rank_in(unsigned long long mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Walk over a tile's particles.  The sort stores each tile transposed: with
// cnt = 64 Q + R particles, the particle of rank t = l Q + j (t < 64 Q) in the
// cell-sorted order sits at position j 64 + l, the last R in order.  Reading
// position j 64 + lane is then coalesced, while lane l works through the run of
// ranks [l Q, (l+1) Q), so the lanes of one wave sit in different cells and
// their LDS deposits rarely hit the same address.  Waves take j = wave, wave +
// waves, ... while j 64 < cnt (the last pass holds the R remaining particles).
__device__ __forceinline__ int tile_pos(int t, int cnt) {
    const int Q = cnt / WAVE;
    return t < WAVE * Q ? (t % Q) * WAVE + t / Q : t;
}

// Slot of this lane in the range of its cell, one atomic per run of equal
// consecutive cells: the first lane of a run adds the run's length to
// cursor[c] and hands the old value to the run (ds_bpermute).  Live lanes must be
// a prefix of the wave; every lane must execute this.
__device__ __forceinline__ int claim_slot(int c, bool live, int32_t *cursor) {
    const int lane = lane_id();
    const int prev = __shfl_up(c, 1, WAVE);
    const bool head = live && (lane == 0 || prev != c);
    const unsigned long long heads = __builtin_amdgcn_ballot_w64(head);
    const unsigned long long lives = __builtin_amdgcn_ballot_w64(live);
    const unsigned long long upto = lane == WAVE - 1 ? ~0ull : ((2ull << lane) - 1ull);   // lanes <= this one
    const int leader = WAVE - 1 - __builtin_clzll((heads & upto) | 1ull);
    int b = 0;
    if (head) {
        const unsigned long long later = (heads & ~upto) | ~lives;   // next head or first dead lane
        const int next = later ? __builtin_ctzll(later) : WAVE;
        b = atomicAdd(&cursor[c], next - lane);
    }
    b = __builtin_amdgcn_ds_bpermute(leader << 2, b);
    return b + lane - leader;
}

// Slot of this lane in counter[key] for the lanes with flag set, one atomic per
// distinct key among them (the lowest such lane adds the key's lane count and
// hands the old value on); lanes without flag get an unspecified value.
__device__ __forceinline__ int wave_claim(int32_t *counter, int key, bool flag) {
    unsigned long long rem = __builtin_amdgcn_ballot_w64(flag);
    int slot = 0;
    while (rem) {
        const int leader = __builtin_ctzll(rem);
        const int lk = __shfl(key, leader, WAVE);
        const bool mine = flag && key == lk;
        const unsigned long long m = __builtin_amdgcn_ballot_w64(mine);
        int b = 0;
        if (lane_id() == leader) b = atomicAdd(&counter[lk], __builtin_popcountll(m));
        b = __shfl(b, leader, WAVE);
        if (mine) slot = b + rank_in(m);
        rem &= ~m;
    }
    return slot;
}

// Gauss-Legendre rule with P points on [0, 1] (exact to degree 2P - 1, the degree
// of a product of a degree-P and a degree-(P-1) spline along a straight path).
template <int P>
struct GL;
template <> struct GL<2> {
    static constexpr double x[2] = {0.21132486540518713, 0.7886751345948129};
    static constexpr double w[2] = {0.5, 0.5};
};
template <> struct GL<3> {
    static constexpr double x[3] = {0.1127016653792583, 0.5, 0.8872983346207417};
    static constexpr double w[3] = {0.27777777777777785, 0.4444444444444444, 0.27777777777777785};
};
template <> struct GL<4> {
    static constexpr double x[4] = {0.06943184420297371, 0.33000947820757187, 0.6699905217924281,
                                    0.9305681557970262};
    static constexpr double w[4] = {0.17392742256872684, 0.3260725774312731, 0.3260725774312731,
                                    0.17392742256872684};
};
template <> struct GL<5> {
    static constexpr double x[5] = {0.04691007703066802, 0.23076534494715845, 0.5, 0.7692346550528415,
                                    0.9530899229693319};
    static constexpr double w[5] = {0.11846344252809471, 0.2393143352496831, 0.2844444444444445,
                                    0.2393143352496831, 0.11846344252809471};
};

// ---------------------------------------------------------------------------
// Small grid and particle kernels
// ---------------------------------------------------------------------------

__global__ void k2_fill(double *a, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

__global__ void k2_fill_u64(unsigned long long *a, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = 0ull;
}

__global__ void k2_fill_i32(int32_t *a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

__global__ void k2_copy(double *__restrict__ dst, const double *__restrict__ src, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// (G a)_1 = (a_{i1,i2} - a_{i1-1,i2}) / dx1, (G a)_2 = (a_{i1,i2} - a_{i1,i2-1}) / dx2.
__global__ void k2_grad(const double *__restrict__ a, double *__restrict__ g1, double *__restrict__ g2, int M1,
                        int M2, double inv_dx1, double inv_dx2) {
    const int N = M1 * M2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const int i1 = i / M2, i2 = i - i1 * M2;
        const double v = a[i];
        g1[i] = (v - a[wrapi(i1 - 1, M1) * M2 + i2]) * inv_dx1;
        g2[i] = (v - a[i1 * M2 + wrapi(i2 - 1, M2)]) * inv_dx2;
    }
}

// Positions of new particles: wrap into [0, M) (cell units), record the cell and
// count it.
__global__ __launch_bounds__(BLOCK) void k2_bin_new(const double *__restrict__ x1, const double *__restrict__ x2,
                                                    double *__restrict__ xi1, double *__restrict__ xi2,
                                                    int32_t *__restrict__ cell, int32_t *__restrict__ count, int64_t n,
                                                    int M1, int M2, double inv_dx1, double inv_dx2, int *flags) {
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const bool live = i < n;
        int c = 0;
        if (live) {
            double u1 = x1[i] * inv_dx1, u2 = x2[i] * inv_dx2;
            if (!isfinite(u1) || !isfinite(u2)) { atomicOr(flags, FLAG_NONFINITE); u1 = 0.0; u2 = 0.0; }
            u1 = fmod(u1, (double)M1);
            u2 = fmod(u2, (double)M2);
            if (u1 < 0.0) u1 += (double)M1;
            if (u2 < 0.0) u2 += (double)M2;
            if (u1 >= (double)M1) u1 = 0.0;
            if (u2 >= (double)M2) u2 = 0.0;
            xi1[i] = u1;
            xi2[i] = u2;
            c = (int)u1 * M2 + (int)u2;
            cell[i] = c;
        }
        claim_slot(c, live, count);
    }
}

// Exclusive scan of count[0..Nc) into start[0..Nc], count <- 0, in three passes:
// block sums (SCAN_TILE cells per block), a scan of the block sums (one block),
// and the block-local scans plus their offsets.
constexpr int SCAN_THREADS = 1024, SCAN_PER = 4, SCAN_TILE = SCAN_THREADS * SCAN_PER;

__device__ __forceinline__ int block_exscan1024(int v, int *total) {
    __shared__ int wsum[SCAN_THREADS / WAVE];
    const int lane = lane_id(), wid = threadIdx.x / WAVE;
    int x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const int y = __shfl_up(x, o, WAVE);
        if (lane >= o) x += y;
    }
    if (lane == WAVE - 1) wsum[wid] = x;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) {
        pre += w < wid ? wsum[w] : 0;
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k2_scan_sums(const int32_t *__restrict__ count, int32_t *bsum,
                                                             int Nc) {
    const int c0 = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER;
    int v = 0;
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) v += c0 + q < Nc ? count[c0 + q] : 0;
    int tot;
    block_exscan1024(v, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_THREADS) void k2_scan_top(int32_t *bsum, int nb, int32_t *start_end) {
    // nb <= SCAN_THREADS (Nc <= 512 * 512 = 64 tiles)
    const int v = (int)threadIdx.x < nb ? bsum[threadIdx.x] : 0;
    int tot;
    const int pre = block_exscan1024(v, &tot);
    if ((int)threadIdx.x < nb) bsum[threadIdx.x] = pre;
    if (threadIdx.x == 0) *start_end = tot;
}

__global__ __launch_bounds__(SCAN_THREADS) void k2_scan_apply(int32_t *__restrict__ count, int32_t *__restrict__ start,
                                                              const int32_t *__restrict__ bsum, int Nc) {
    const int c0 = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER;
    int k[SCAN_PER], v = 0;
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
        k[q] = c0 + q < Nc ? count[c0 + q] : 0;
        v += k[q];
    }
    int tot;
    int off = bsum[blockIdx.x] + block_exscan1024(v, &tot);
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q)
        if (c0 + q < Nc) {
            start[c0 + q] = off;
            off += k[q];
            count[c0 + q] = 0;
        }
}

// Move every particle to its cell's range of the destination buffers.
__global__ __launch_bounds__(BLOCK) void k2_scatter(const double *__restrict__ s1, const double *__restrict__ s2,
                                                    const double *__restrict__ q1, const double *__restrict__ q2,
                                                    const int32_t *__restrict__ sid, double *__restrict__ d1,
                                                    double *__restrict__ d2, double *__restrict__ r1,
                                                    double *__restrict__ r2, int32_t *__restrict__ did,
                                                    const int32_t *__restrict__ cell, const int32_t *__restrict__ start,
                                                    int32_t *__restrict__ cursor, int64_t n, int M2, int TW) {
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const bool live = i < n;
        const int c = live ? cell[i] : 0;
        const int slot = claim_slot(c, live, cursor);
        if (live) {
            const int r = c / M2, first = r * M2 + ((c - r * M2) / TW) * TW;   // tile's first cell
            const int tb = start[first], cnt = start[first + TW] - tb;
            const int j = tb + tile_pos(start[c] - tb + slot, cnt);
            d1[j] = s1[i];
            d2[j] = s2[i];
            r1[j] = q1[i];
            r2[j] = q2[i];
            did[j] = sid[i];
        }
    }
}

// out[id[i]] = v[i] (positions back to physical units when scale != 1).
__global__ void k2_unsort(const double *__restrict__ v, const int32_t *__restrict__ id, double *__restrict__ out,
                          int64_t n, double scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[id[i]] = v[i] * scale;
}

__global__ void k2_iota(int32_t *id, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        id[i] = (int32_t)i;
}

// Value of the degree (P, P) field at a point in cell (c1, c2), local (t1, t2),
// from the global grid.
template <int P>
__device__ __forceinline__ double gather00(const double *__restrict__ f, int M1, int M2, int c1, int c2, double t1,
                                           double t2) {
    double b1[P + 1], b2[P + 1];
    basis_values<P>(t1, b1);
    basis_values<P>(t2, b2);
    double s = 0.0;
#pragma unroll
    for (int m1 = 0; m1 <= P; ++m1) {
        const double *row = f + wrapi(c1 - m1, M1) * M2;
        double t = 0.0;
#pragma unroll
        for (int m2 = 0; m2 <= P; ++m2) t += b2[m2] * row[wrapi(c2 - m2, M2)];
        s += b1[m1] * t;
    }
    return s;
}

// sum f_{i1,i2} N^{D1}_{i1}(x1) N^{D2}_{i2}(x2) at a point of cell (c1, c2), from
// global memory (diagnostics).
template <int D1, int D2>
__device__ __forceinline__ double gatherg(const double *__restrict__ f, int M1, int M2, int c1, int c2, double t1,
                                          double t2) {
    double b1[D1 + 1], b2[D2 + 1];
    basis_values<D1>(t1, b1);
    basis_values<D2>(t2, b2);
    double s = 0.0;
#pragma unroll
    for (int m1 = 0; m1 <= D1; ++m1) {
        const double *row = f + wrapi(c1 - m1, M1) * M2;
        double t = 0.0;
#pragma unroll
        for (int m2 = 0; m2 <= D2; ++m2) t += b2[m2] * row[wrapi(c2 - m2, M2)];
        s += b1[m1] * t;
    }
    return s;
}

// Zeeman sum w s . B_h(x) over the particles (times hbar on the host), B_h =
// (dA_z/dx2, -dA_z/dx1, B_z) from G a_z (g1, g2) and b_z.
template <int P>
__global__ __launch_bounds__(BLOCK) void k2_zeeman(const double *__restrict__ xi1, const double *__restrict__ xi2,
                                                   const double *__restrict__ sx, const double *__restrict__ sy,
                                                   const double *__restrict__ sz, const double *__restrict__ g1,
                                                   const double *__restrict__ g2, const double *__restrict__ bz,
                                                   int64_t n, int M1, int M2, double w, double *__restrict__ partial) {
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double u1 = xi1[i], u2 = xi2[i];
        const int c1 = (int)u1, c2 = (int)u2;
        const double t1 = u1 - c1, t2 = u2 - c2;
        const double Bx = gatherg<P, P - 1>(g2, M1, M2, c1, c2, t1, t2);
        const double By = -gatherg<P - 1, P>(g1, M1, M2, c1, c2, t1, t2);
        const double Bz = gatherg<P - 1, P - 1>(bz, M1, M2, c1, c2, t1, t2);
        s += w * (sx[i] * Bx + sy[i] * By + sz[i] * Bz);
    }
    block_sum_to(s, &partial[blockIdx.x]);
}

// out[i] = in[id[i]]: values given in the caller's order, put into the sorted order.
__global__ void k2_gather_id(const double *__restrict__ in, const int32_t *__restrict__ id, double *__restrict__ out,
                             int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[id[i]];
}

// Spin deposits over tiles (no motion): mode 0: Dx += w s_x N^P(x1) N^{P-1}(x2) and
// Dy += w s_y N^{P-1}(x1) N^P(x2) (Lambda1*^T W S_xy); mode 1: Dz += w s_z
// N^{P-1}(x1) N^{P-1}(x2) (Lambda2^T W S_z).  Targets zero on entry.
template <int P>
__global__ __launch_bounds__(BLOCK) void k2_deposit_spin(const double *__restrict__ xi1,
                                                         const double *__restrict__ xi2,
                                                         const double *__restrict__ sx,
                                                         const double *__restrict__ sy,
                                                         const double *__restrict__ sz,
                                                         const int32_t *__restrict__ start, double *__restrict__ Dx,
                                                         double *__restrict__ Dy, double *__restrict__ Dz, int M1,
                                                         int M2, int TW, double w, int mode) {
    constexpr int PR = P + 1, PCM = TWMAX + P, PS = PR * PCM;
    __shared__ double sX[PS], sY[PS];
    const int nseg = M2 / TW;
    const int tile = tile_of_block();
    const int r = tile / nseg, c0 = (tile - r * nseg) * TW;
    const int PC = TW + P;
    const int R0 = r - P, C0 = c0 - P;
    for (int t = threadIdx.x; t < PR * PC; t += blockDim.x) {
        sX[t] = 0.0;
        sY[t] = 0.0;
    }
    __syncthreads();
    const int begin = start[tile], end = start[tile + 1];
    for (int i = begin + threadIdx.x; i < end; i += blockDim.x) {
        const double u1 = xi1[i], u2 = xi2[i];
        const int c2 = (int)u2;
        double a1[P + 1], a2[P + 1], b1[P], b2[P];
        basis_values<P>(u1 - r, a1);
        basis_values<P>(u2 - c2, a2);
        basis_values<P - 1>(u1 - r, b1);
        basis_values<P - 1>(u2 - c2, b2);
        if (mode == 0) {
            const double qx = w * sx[i], qy = w * sy[i];
#pragma unroll
            for (int m1 = 0; m1 <= P; ++m1)
#pragma unroll
                for (int m2 = 0; m2 <= P; ++m2) {
                    const int k = (r - m1 - R0) * PC + c2 - m2 - C0;
                    if (m2 < P) atomicAdd(&sX[k], qx * a1[m1] * b2[m2]);
                    if (m1 < P) atomicAdd(&sY[k], qy * b1[m1] * a2[m2]);
                }
        } else {
            const double qz = w * sz[i];
#pragma unroll
            for (int m1 = 0; m1 < P; ++m1)
#pragma unroll
                for (int m2 = 0; m2 < P; ++m2) atomicAdd(&sX[(r - m1 - R0) * PC + c2 - m2 - C0], qz * b1[m1] * b2[m2]);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < PR * PC; t += blockDim.x) {
        const int i = t / PC, j = t - i * PC;
        const int g = wrapi(R0 + i, M1) * M2 + wrapi(C0 + j, M2);
        if (mode == 0) {
            if (sX[t] != 0.0) atomicAdd(&Dx[g], sX[t]);
            if (sY[t] != 0.0) atomicAdd(&Dy[g], sY[t]);
        } else if (sX[t] != 0.0) {
            atomicAdd(&Dz[g], sX[t]);
        }
    }
}

// src = G*^T (Dx, Dy) = G2^T Dx - G1^T Dy, the transposes of the backward
// differences: (G1^T u)_i = (u_{i1,i2} - u_{i1+1,i2}) / dx1, likewise in x2.
__global__ __launch_bounds__(BLOCK) void k2_spin_src(const double *__restrict__ Dx, const double *__restrict__ Dy,
                                                     double *__restrict__ src, int M1, int M2, double inv_dx1,
                                                     double inv_dx2) {
    const int N = M1 * M2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const int i1 = i / M2, i2 = i - i1 * M2;
        src[i] = (Dx[i] - Dx[i1 * M2 + wrapi(i2 + 1, M2)]) * inv_dx2 -
                 (Dy[i] - Dy[wrapi(i1 + 1, M1) * M2 + i2]) * inv_dx1;
    }
}

// ---------------------------------------------------------------------------
// Subsystem I sweep (Section 4.3): gather, push, deposit, one tile per block
// ---------------------------------------------------------------------------
struct SweepArgs {
    const double *xi1, *xi2, *p1, *p2;   // sorted particles
    double *d1, *d2;                     // increment d^(k) (physical); formed and stored by sweep 0
    double *dn1, *dn2;                   // increment d^(k+1)
    double *pk1, *pk2;                   // momentum p^(k+1)
    const int32_t *start;                // first particle of each tile (ntiles + 1)
    const double *eb1, *eb2;             // (e^n + e^(k)) / 2
    const double *az, *g1a, *g2a;        // a_z and G a_z
    double *J1, *J2;                     // current of d^(k) (accumulated, zero on entry)
    unsigned long long *res;             // max |d^(k+1) - d^(k)|, as bits
    int *flags;
    const int *gate;                     // nonzero: an earlier sweep converged, nothing to do
    int M1, M2, TW;
    double inv_dx1, inv_dx2, dt, w;
    const double *sx, *sy, *sz, *bz;     // spins and b_z (the sweep with spin)
    double hbar;
    double *azn, *gamn;                  // A_z(x^n) and gamma(x^n, p^n): formed by sweep 0, read by the rest
};

// Line mean of the V1 basis (degree P-1) along one leg of the step, from t0 in
// [0, 1) of cell c0 to t1 in (-1, 2) (cell units, c0 frame); s = +1 / -1 / 0
// tells whether t1 lies in cell c0+1 / c0-1 / c0, and rlen is 1 / |t1 - t0|
// (used only when s != 0).  lb[k], k = 0..P+1, is the mean of Lambda1_{c0-P+k}:
// the mean over each piece of the leg (the part in c0 and the part in c0+s),
// weighted by the piece's share of the length.
template <int P>
__device__ __forceinline__ void leg_mean_v1(double t0, double t1, int s, double rlen, double (&lb)[P + 2]) {
    constexpr int D = P - 1;
    const double t1c = fmin(fmax(t1, 0.0), 1.0);
    double avgA[D + 1], avgB[D + 1];
    piece_means<D>(fmin(t0, t1c), fmax(t0, t1c), avgA);
    // the piece in the neighbour cell: [0, t1 - 1] (s = +1) or [t1 + 1, 1] (s = -1)
    const double as = s < 0 ? t1 + 1.0 : 0.0, bs = s > 0 ? t1 - 1.0 : (s < 0 ? 1.0 : 0.0);
    piece_means<D>(as, bs, avgB);
    const double wB = s != 0 ? (bs - as) * rlen : 0.0, wA = 1.0 - wB;
#pragma unroll
    for (int k = 0; k <= P + 1; ++k) {
        const double v = (k >= 1 && k <= P) ? wA * avgA[P - k] : 0.0;   // index c0 - m, k = P - m
        double vb = 0.0;                                                 // index c0 + s - m
        if (s > 0 && P + 1 - k >= 0 && P + 1 - k <= D) vb = avgB[P + 1 - k < 0 ? 0 : (P + 1 - k > D ? D : P + 1 - k)];
        if (s < 0 && P - 1 - k >= 0 && P - 1 - k <= D) vb = avgB[P - 1 - k < 0 ? 0 : (P - 1 - k > D ? D : P - 1 - k)];
        lb[k] = v + wB * vb;
    }
}

// 1 / |s| for a leg of s cells, with |s| raised to a tiny normal floor: a leg
// that crosses a grid line is longer than that unless it starts within the
// floor of the line, where the split of its (vanishing) length does not matter.
__device__ __forceinline__ double leg_rcp(double s) { return frcp(fmax(fabs(s), 1.0e-290)); }

// Path integrals of the V1 basis on one piece of the straight step (between two
// grid-line crossings, inside cell (k1, k2)), both components, by the P-point
// Gauss-Legendre rule in the piece's own frame: W1[u][v] is the integral over
// the piece (parameter length len) of N^{P-1}_{k1-(P-1)+u}(x1) N^P_{k2-P+v}(x2),
// W2[u][v] that of N^P_{k1-P+u}(x1) N^{P-1}_{k2-(P-1)+v}(x2).
template <int P>
__device__ __forceinline__ void piece_integrals(double x1, double x2, double s1, double s2, int k1, int k2,
                                                double sa, double len, double (&W1)[P][P + 1],
                                                double (&W2)[P + 1][P]) {
#pragma unroll
    for (int u = 0; u < P; ++u)
#pragma unroll
        for (int v = 0; v < P + 1; ++v) { W1[u][v] = 0.0; W2[v][u] = 0.0; }
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const double s = sa + len * GL<P>::x[q];
        const double g = len * GL<P>::w[q];
        const double t1 = x1 + s * s1 - k1, t2 = x2 + s * s2 - k2;
        double b0x[P + 1], b1x[P], b0y[P + 1], b1y[P];
        basis_values<P>(t1, b0x);       // b0x[m]: N^P_{k1-m}
        basis_values<P - 1>(t1, b1x);   // b1x[m]: N^{P-1}_{k1-m}
        basis_values<P>(t2, b0y);
        basis_values<P - 1>(t2, b1y);
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const double gx = g * b1x[P - 1 - u], gy = g * b1y[P - 1 - u];
#pragma unroll
            for (int v = 0; v < P + 1; ++v) {
                W1[u][v] += gx * b0y[P - v];
                W2[v][u] += gy * b0x[P - v];
            }
        }
    }
}

// The field patch of a tile in LDS (rows r-P-1 .. r+1, columns c0-P-1 .. c0+TW).
struct Patch {
    double *E1, *E2, *A, *G1, *G2, *J1, *J2, *Bz;
    int PC, R0, C0, r;
};

// One particle's step geometry (cell units): start x, increment s, end y, the
// start/end cells, the lower-left cell of the step and the path parameters lo <=
// hi of its grid-line crossings (1 when there is none).
struct Geo {
    double x1, x2, q1, q2, D1, D2, s1, s2, y1, y2, lo, hi;
    int ca2, cb1, cb2, mn1, mn2;
};

__device__ __forceinline__ Geo geometry(const SweepArgs &a, double x1, double x2, double q1, double q2, double D1,
                                        double D2, bool live, int r, int &flags) {
    Geo g;
    g.x1 = x1;
    g.x2 = x2;
    g.q1 = q1;
    g.q2 = q2;
    g.D1 = live ? D1 : 0.0;
    g.D2 = live ? D2 : 0.0;
    g.s1 = g.D1 * a.inv_dx1;
    g.s2 = g.D2 * a.inv_dx2;
    g.y1 = g.x1 + g.s1;
    g.y2 = g.x2 + g.s2;
    const int ca1 = r;
    g.ca2 = (int)g.x2;
    g.cb1 = (int)floor(g.y1);
    g.cb2 = (int)floor(g.y2);
    if (g.cb1 < ca1 - 1 || g.cb1 > ca1 + 1 || g.cb2 < g.ca2 - 1 || g.cb2 > g.ca2 + 1 || !isfinite(g.s1 + g.s2)) {
        if (live) flags |= isfinite(g.s1 + g.s2) ? FLAG_CFL : FLAG_NONFINITE;
        g.cb1 = ca1;
        g.cb2 = g.ca2;
    }
    g.mn1 = min(ca1, g.cb1);
    g.mn2 = min(g.ca2, g.cb2);
    const double bA = g.cb1 != ca1 ? ((double)max(ca1, g.cb1) - g.x1) * copysign(leg_rcp(g.s1), g.s1) : 1.0;
    const double bB = g.cb2 != g.ca2 ? ((double)max(g.ca2, g.cb2) - g.x2) * copysign(leg_rcp(g.s2), g.s2) : 1.0;
    g.lo = fmin(bA, bB);
    g.hi = fmax(bA, bB);
    return g;
}

// Pieces first..last of the path (0: [0, lo], 1: [lo, hi], 2: [hi, 1]): the mean
// field is accumulated into E1, E2 and w d times the path integrals of the V1 basis
// are added to the current patch.  Pieces no lane of the wave needs are skipped.
template <int P>
__device__ __forceinline__ void pieces(const Geo &g, bool live, int first, int last, const Patch &t, double w,
                                       double &E1, double &E2) {
    const double j1 = w * g.D1, j2 = w * g.D2;
    const int PC = t.PC;
#pragma unroll 1
    for (int piece = first; piece <= last; ++piece) {
        const double sa = piece == 0 ? 0.0 : (piece == 1 ? g.lo : g.hi);
        const double sb = piece == 0 ? g.lo : (piece == 1 ? g.hi : 1.0);
        const double len = live ? sb - sa : 0.0;
        if (!__builtin_amdgcn_ballot_w64(len > 0.0)) continue;
        const double sm = 0.5 * (sa + sb);
        const int k1 = min(max((int)floor(g.x1 + sm * g.s1), g.mn1), g.mn1 + 1);
        const int k2 = min(max((int)floor(g.x2 + sm * g.s2), g.mn2), g.mn2 + 1);
        double W1[P][P + 1], W2[P + 1][P];
        piece_integrals<P>(g.x1, g.x2, g.s1, g.s2, k1, k2, sa, len, W1, W2);
        const int o1 = (k1 - (P - 1) - t.R0) * PC + k2 - P - t.C0;   // W1[0][0] in the patch
        const int o2 = (k1 - P - t.R0) * PC + k2 - (P - 1) - t.C0;   // W2[0][0]
#pragma unroll
        for (int u = 0; u < P; ++u)
#pragma unroll
            for (int v = 0; v < P + 1; ++v) {
                E1 += W1[u][v] * t.E1[o1 + u * PC + v];
                E2 += W2[v][u] * t.E2[o2 + v * PC + u];
            }
        if (len > 0.0) {
#pragma unroll
            for (int u = 0; u < P; ++u)
#pragma unroll
                for (int v = 0; v < P + 1; ++v) {
                    atomicAdd(&t.J1[o1 + u * PC + v], j1 * W1[u][v]);
                    atomicAdd(&t.J2[o2 + v * PC + u], j2 * W2[v][u]);
                }
        }
    }
}

// A_z at a start point x (x1 in the tile's row) from the patch.
template <int P>
__device__ __forceinline__ double start_A(const Patch &t, double x1, double x2) {
    const int c2 = (int)x2;
    double b1[P + 1], b2[P + 1];
    basis_values<P>(x1 - t.r, b1);
    basis_values<P>(x2 - c2, b2);
    double A = 0.0;
#pragma unroll
    for (int m1 = 0; m1 <= P; ++m1) {
        double ta = 0.0;
#pragma unroll
        for (int m2 = 0; m2 <= P; ++m2) ta += b2[m2] * t.A[(t.r - m1 - t.R0) * t.PC + c2 - m2 - t.C0];
        A += b1[m1] * ta;
    }
    return A;
}

// gamma(x, p) from A_z(x) = A and p = (q1, q2).
__device__ __forceinline__ double gamma_of(double q1, double q2, double A) {
    return fsqrt(1.0 + q1 * q1 + q2 * q2 + A * A);
}

// A_z at the end point, the means of dA_z/dx2 along the vertical leg (at x1^n) and
// of dA_z/dx1 along the horizontal leg (at x2^{n+1}), the push of the Subsystem I
// scheme, and the stores of particle i.  Aa = A_z(x^n) and gA = gamma(x^n, p^n)
// are fixed over the iteration.
template <int P, bool SPIN>
__device__ __forceinline__ void finish(const Geo &g, bool live, int i, double E1, double E2, double Aa, double gA,
                                       const Patch &t, const SweepArgs &a, double &rmax, int &flags) {
    const int PC = t.PC, R0 = t.R0, C0 = t.C0, ca1 = t.r, ca2 = g.ca2, cb1 = g.cb1, cb2 = g.cb2;
    double ba1[P + 1], bb1[P + 1], bb2[P + 1];
    basis_values<P>(g.x1 - ca1, ba1);
    basis_values<P>(g.y1 - cb1, bb1);
    basis_values<P>(g.y2 - cb2, bb2);
    double Ab = 0.0;
#pragma unroll
    for (int m1 = 0; m1 <= P; ++m1) {
        double tb = 0.0;
#pragma unroll
        for (int m2 = 0; m2 <= P; ++m2) tb += bb2[m2] * t.A[(cb1 - m1 - R0) * PC + cb2 - m2 - C0];
        Ab += bb1[m1] * tb;
    }
    const double rl2 = leg_rcp(g.s2), rl1 = leg_rcp(g.s1);
    double lm2[P + 2], lm1[P + 2];
    leg_mean_v1<P>(g.x2 - ca2, g.y2 - ca2, cb2 - ca2, rl2, lm2);   // indices ca2 - P + k
    leg_mean_v1<P>(g.x1 - ca1, g.y1 - ca1, cb1 - ca1, rl1, lm1);   // indices ca1 - P + k
    double Dv = 0.0, Dh = 0.0;
#pragma unroll
    for (int m1 = 0; m1 <= P; ++m1) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < P + 2; ++k) s += lm2[k] * t.G2[(ca1 - m1 - R0) * PC + ca2 - P + k - C0];
        Dv += ba1[m1] * s;
    }
#pragma unroll
    for (int k = 0; k < P + 2; ++k) {
        double s = 0.0;
#pragma unroll
        for (int m2 = 0; m2 <= P; ++m2) s += bb2[m2] * t.G1[(ca1 - P + k - R0) * PC + cb2 - m2 - C0];
        Dh += lm1[k] * s;
    }
    double F1 = 0.0, F2 = 0.0;   // spin force / hbar
    if constexpr (SPIN) {
        // Means along the same two legs of the derivatives of dA_z/dx2 (coefficients
        // G2 = (G a)_2, degrees (P, P-1)), dA_z/dx1 (G1, (P-1, P)) and B_z ((P-1, P-1)):
        // each derivative's coefficients are backward differences of the field's.
        double lq2[P + 1], lq1[P + 1], bm1[P], bmb2[P];
        leg_mean_v1<P - 1>(g.x2 - ca2, g.y2 - ca2, cb2 - ca2, rl2, lq2);   // degree P-2, indices ca2 - P + 1 + k
        leg_mean_v1<P - 1>(g.x1 - ca1, g.y1 - ca1, cb1 - ca1, rl1, lq1);   // degree P-2, indices ca1 - P + 1 + k
        basis_values<P - 1>(g.x1 - ca1, bm1);
        basis_values<P - 1>(g.y2 - cb2, bmb2);
        const double i1 = a.inv_dx1, i2 = a.inv_dx2;
        // Summation by parts: sum_k m_k (F_k - F_{k-1}) = sum_j F_j (m_j - m_{j+1}), so
        // every patch value is read once, with difference weights formed once.
        // x2 leg at x1^n: columns ca2 - P - 1 + j, j = 0..P+2.
        double wa[P + 3], wb[P + 3];   // weights of lm2 (degree P-1) and lq2 (degree P-2)
#pragma unroll
        for (int j = 0; j <= P + 2; ++j) {
            const double m0 = j >= 1 ? lm2[j - 1] : 0.0, m1 = j <= P + 1 ? lm2[j] : 0.0;
            const double q0 = j >= 2 ? lq2[j - 2] : 0.0, q1 = (j >= 1 && j <= P + 1) ? lq2[j - 1] : 0.0;
            wa[j] = m0 - m1;
            wb[j] = q0 - q1;
        }
        double Sy2 = 0.0, Sx2 = 0.0, Sb2 = 0.0;
#pragma unroll
        for (int m1 = 0; m1 <= P; ++m1) {
            const int row = (ca1 - m1 - R0) * PC - C0 + ca2 - P - 1;
            double ty = 0.0, tx = 0.0, tb = 0.0;
#pragma unroll
            for (int j = 0; j <= P + 2; ++j) {
                if (j >= 1) ty += wb[j] * t.G2[row + j];
                tx += wa[j] * t.G1[row + j];
                if (j >= 1) tb += wb[j] * t.Bz[row + j];
            }
            Sy2 += ba1[m1] * ty;
            if (m1 < P) {
                Sx2 += bm1[m1] * tx;
                Sb2 += bm1[m1] * tb;
            }
        }
        // x1 leg at x2^{n+1}: rows ca1 - P - 1 + j, j = 0..P+2; per row the x2 sums first.
        double Sy1 = 0.0, Sx1 = 0.0, Sb1 = 0.0;
#pragma unroll
        for (int j = 0; j <= P + 2; ++j) {
            const double m0 = j >= 1 ? lm1[j - 1] : 0.0, m1 = j <= P + 1 ? lm1[j] : 0.0;
            const double q0 = j >= 2 ? lq1[j - 2] : 0.0, q1 = (j >= 1 && j <= P + 1) ? lq1[j - 1] : 0.0;
            const int row = (ca1 - P - 1 + j - R0) * PC - C0;
            double ty = 0.0, tx = 0.0, tb = 0.0;
#pragma unroll
            for (int m2 = 0; m2 <= P; ++m2) {
                const int c = row + cb2 - m2;
                tx += bb2[m2] * t.G1[c];
                if (m2 < P) {
                    ty += bmb2[m2] * t.G2[c];
                    tb += bmb2[m2] * t.Bz[c];
                }
            }
            Sy1 += (m0 - m1) * ty;
            Sx1 += (q0 - q1) * tx;
            Sb1 += (q0 - q1) * tb;
        }
        const double sx = a.sx[i], sy = a.sy[i], sz = a.sz[i];
        F1 = (sx * Sy1 - sy * Sx1 + sz * Sb1) * i1;
        F2 = (sx * Sy2 - sy * Sx2 + sz * Sb2) * i2;
    }
    const double q1 = g.q1, q2 = g.q2;
    const double gB = gamma_of(q1, q2, Ab);
    const double f = -(Aa + Ab) * frcp(gA + gB);
    double n1, n2;
    if constexpr (SPIN) {
        n1 = q1 + a.dt * (E1 + f * Dh - a.hbar * F1);
        n2 = q2 + a.dt * (E2 + f * Dv - a.hbar * F2);
    } else {
        n1 = q1 + a.dt * (E1 + f * Dh);
        n2 = q2 + a.dt * (E2 + f * Dv);
    }
    const double gC = gamma_of(n1, n2, Ab);
    const double sc = a.dt * frcp(gB + gC);
    const double e1 = (q1 + n1) * sc, e2 = (q2 + n2) * sc;
    if (live) {
        if (!isfinite(e1 + e2 + n1 + n2)) flags |= FLAG_NONFINITE;
        a.dn1[i] = e1;
        a.dn2[i] = e2;
        a.pk1[i] = n1;
        a.pk2[i] = n2;
        rmax = fmax(rmax, fmax(fabs(e1 - g.D1), fabs(e2 - g.D2)));
    }
}

// One sweep over a tile.  Every particle integrates the first piece of its path
// inline; a step that crosses a grid line needs one or two more pieces, and such
// particles (about one in ten) are parked, with their position, increment and
// partial mean field, in a per-wave LDS queue and finished 64 at a time, so that
// the waves do not run the extra pieces for lanes that have none (only the
// momentum is read again).
constexpr int QCAP = 2 * WAVE;
constexpr int QV = 6;   // x1, x2, d1, d2, E1, E2

// FIRST (sweep 0): the increment is the explicit start d^(0) = dt p^n /
// gamma(x^n, p^n), formed from A_z on the patch and stored with A_z(x^n) and
// gamma(x^n, p^n), which the later sweeps read instead; that variant is held
// to three waves per SIMD (168 VGPRs) at p = 3, like the others.  SPIN: the
// spin force as well; held to three waves per SIMD for p <= 3 (a few registers
// spilled) after the first sweep, two in it.
template <int P, bool FIRST, bool SPIN>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(!SPIN ? (FIRST && P == 3 ? 3 : 1)
                                                                            : (P <= 3 ? (FIRST ? 2 : 3) : 1)))) void k2_sweep_I(
    SweepArgs a) {
    if (*a.gate) return;   // uniform over the grid
    constexpr int PR = P + 3, PCM = TWMAX + P + 2, PS = PR * PCM;
    __shared__ double sE1[PS], sE2[PS], sA[PS], sG1[PS], sG2[PS], sJ1[PS], sJ2[PS], sBz[SPIN ? PS : 1];
    __shared__ int qI[BLOCK / WAVE][QCAP];
    __shared__ double qV[BLOCK / WAVE][QV][QCAP];
    const int nseg = a.M2 / a.TW;
    const int tile = tile_of_block();
    const int r = tile / nseg, c0 = (tile - r * nseg) * a.TW;
    const int PC = a.TW + P + 2;
    const Patch t{sE1, sE2, sA, sG1, sG2, sJ1, sJ2, sBz, PC, r - P - 1, c0 - P - 1, r};
    for (int k = threadIdx.x; k < PR * PC; k += blockDim.x) {
        const int i = k / PC, j = k - i * PC;
        const int g = wrapi(t.R0 + i, a.M1) * a.M2 + wrapi(t.C0 + j, a.M2);
        sE1[k] = a.eb1[g];
        sE2[k] = a.eb2[g];
        sA[k] = a.az[g];
        sG1[k] = a.g1a[g];
        sG2[k] = a.g2a[g];
        sJ1[k] = 0.0;
        sJ2[k] = 0.0;
        if constexpr (SPIN) sBz[k] = a.bz[g];
    }
    __syncthreads();
    const int begin = a.start[tile], end = a.start[tile + 1];
    const int wid = threadIdx.x / WAVE, lane = lane_id();
    int *const qi = qI[wid];
    double(*const qv)[QCAP] = qV[wid];
    double rmax = 0.0;
    int flags = 0;
    int head = 0, tail = 0;   // queue of this wave (uniform)
    // finish the n <= 64 oldest queued particles, one per lane
    auto drain = [&](int n) {
        const bool valid = lane < n;
        const int slot = (head + lane) & (QCAP - 1);
        double v[QV];
#pragma unroll
        for (int q = 0; q < QV; ++q) v[q] = valid ? qv[q][slot] : 0.0;
        const int i = valid ? qi[slot] : begin;
        if (!valid) v[0] = (double)r, v[1] = (double)c0;   // any point of the tile
        double E1 = v[4], E2 = v[5];
        const double q1 = a.p1[i], q2 = a.p2[i];
        const Geo g = geometry(a, v[0], v[1], q1, q2, v[2], v[3], valid, r, flags);
        pieces<P>(g, valid, 1, 2, t, a.w, E1, E2);
        const double An = start_A<P>(t, v[0], v[1]);   // formed again rather than queued
        finish<P, SPIN>(g, valid, i, E1, E2, An, gamma_of(q1, q2, An), t, a, rmax, flags);
        head += n;
    };
    const int nw = blockDim.x / WAVE, passes = (end - begin + WAVE - 1) / WAVE;   // none for an empty tile
    for (int jr = wid; jr < passes; jr += nw) {
        const int i = begin + jr * WAVE + lane;
        const bool live = i < end;
        const int ii = live ? i : begin;
        const double x1 = a.xi1[ii], x2 = a.xi2[ii], q1 = a.p1[ii], q2 = a.p2[ii];
        double D1, D2, An, gn;
        if constexpr (FIRST) {
            An = start_A<P>(t, x1, x2);
            gn = gamma_of(q1, q2, An);
            const double sc = a.dt * frcp(gn);
            D1 = q1 * sc;
            D2 = q2 * sc;
            if (live) {
                a.d1[i] = D1;
                a.d2[i] = D2;
                a.azn[i] = An;
                a.gamn[i] = gn;
            }
        } else {
            D1 = a.d1[ii];
            D2 = a.d2[ii];
            An = a.azn[ii];
            gn = a.gamn[ii];
        }
        const Geo g = geometry(a, x1, x2, q1, q2, D1, D2, live, r, flags);
        double E1 = 0.0, E2 = 0.0;
        pieces<P>(g, live, 0, 0, t, a.w, E1, E2);
        const bool cross = live && g.lo < 1.0;
        const unsigned long long cm = __builtin_amdgcn_ballot_w64(cross);
        if (cross) {
            const int slot = (tail + rank_in(cm)) & (QCAP - 1);
            qi[slot] = i;
            qv[0][slot] = x1;
            qv[1][slot] = x2;
            qv[2][slot] = D1;
            qv[3][slot] = D2;
            qv[4][slot] = E1;
            qv[5][slot] = E2;
        }
        tail += __builtin_popcountll(cm);
        if (live && !cross) finish<P, SPIN>(g, live, i, E1, E2, An, gn, t, a, rmax, flags);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (tail - head >= WAVE) drain(WAVE);
    }
    if (tail > head) drain(tail - head);
    if (flags) atomicOr(a.flags, flags);
    block_max_to(rmax, a.res);
    __syncthreads();
    for (int k = threadIdx.x; k < PR * PC; k += blockDim.x) {
        const int i = k / PC, j = k - i * PC;
        const int g = wrapi(t.R0 + i, a.M1) * a.M2 + wrapi(t.C0 + j, a.M2);
        if (sJ1[k] != 0.0) atomicAdd(&a.J1[g], sJ1[k]);
        if (sJ2[k] != 0.0) atomicAdd(&a.J2[g], sJ2[k]);
    }
}

// Tile starts from cell starts (after the full cell sort of set_particles): the
// first cell of tile T is (T / nseg) M2 + (T % nseg) TW.
__global__ void k2_tiles_from_cells(const int32_t *__restrict__ start, int32_t *__restrict__ tstart, int ntiles,
                                    int nseg, int M2, int TW, int Nc) {
    for (int T = blockIdx.x * blockDim.x + threadIdx.x; T <= ntiles; T += gridDim.x * blockDim.x)
        tstart[T] = T == ntiles ? start[Nc] : start[(T / nseg) * M2 + (T - (T / nseg) * nseg) * TW];
}

// New cell coordinate of a particle from its committed increment, wrapped into
// [0, M); the commit and the re-sort form it with the same operations.
__device__ __forceinline__ double new_coord(double u, double d, double inv_dx, int M) {
    double v = fma(d, inv_dx, u);
    if (v < 0.0) v += (double)M;
    if (v >= (double)M) v -= (double)M;
    if (!(v < (double)M) || v < 0.0) v = 0.0;   // -tiny + M rounded to M
    return v;
}

// Subsystem I commit, first half (one block per tile): the new tile Tn and the
// column c of every particle inside it, packed as Tn 64 + c in word[i]; per
// tile the particles that stay and (by atomics) those that arrive.  The new
// positions and momenta are written by the re-sort.
__global__ __launch_bounds__(BLOCK) void k2_commit_tiles(const double *__restrict__ xi1,
                                                         const double *__restrict__ xi2,
                                                         const double *__restrict__ d1, const double *__restrict__ d2,
                                                         int32_t *__restrict__ word,
                                                         const int32_t *__restrict__ tstart, int32_t *__restrict__ tstay,
                                                         int32_t *__restrict__ tarr, int M1, int M2, int TW,
                                                         double inv_dx1, double inv_dx2) {
    __shared__ int red[BLOCK / WAVE];
    const int T = blockIdx.x, nseg = M2 / TW;
    const int begin = tstart[T], end = tstart[T + 1];
    int stay = 0;
    for (int i = begin + threadIdx.x; i < end; i += blockDim.x) {
        const double u1 = new_coord(xi1[i], d1[i], inv_dx1, M1), u2 = new_coord(xi2[i], d2[i], inv_dx2, M2);
        const int c2 = (int)u2, sg = c2 / TW;
        const int Tn = (int)u1 * nseg + sg;
        word[i] = (Tn << 6) | (c2 - sg * TW);
        if (Tn == T) ++stay;
        wave_claim(tarr, Tn, Tn != T);
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) stay += __shfl_xor(stay, o, WAVE);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = stay;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) t += red[w];
        tstay[T] = t;
    }
}

// count[T] = stay[T] + arrivals[T]; the arrival counts and cursors start at zero again.
__global__ void k2_tile_counts(const int32_t *__restrict__ tstay, int32_t *__restrict__ tarr,
                               int32_t *__restrict__ tcnt, int32_t *__restrict__ tcur, int ntiles) {
    for (int T = blockIdx.x * blockDim.x + threadIdx.x; T < ntiles; T += gridDim.x * blockDim.x) {
        tcnt[T] = tstay[T] + tarr[T];
        tarr[T] = 0;
        tcur[T] = 0;
    }
}

// Arrivals listed per new tile: a particle of old tile T whose new tile Tn
// differs puts its index at mig[tnew[Tn] + tstay[Tn] + k], k from Tn's cursor
// (the slots after Tn's stayers in the new order).
__global__ __launch_bounds__(BLOCK) void k2_list_arrivals(const int32_t *__restrict__ word,
                                                          const int32_t *__restrict__ told,
                                                          const int32_t *__restrict__ tnew,
                                                          const int32_t *__restrict__ tstay, int32_t *__restrict__ tcur,
                                                          int32_t *__restrict__ mig) {
    const int T = blockIdx.x;
    for (int i = told[T] + threadIdx.x; i < told[T + 1]; i += blockDim.x) {
        const int Tn = word[i] >> 6;
        const int k = wave_claim(tcur, Tn, Tn != T);
        if (Tn != T) mig[tnew[Tn] + tstay[Tn] + k] = i;
    }
}

// Subsystem I commit, second half, and the re-sort in one pass (one block per
// new tile): the tile's particles are the stayers of its old range and its
// listed arrivals; an LDS histogram of their new columns and its prefix give
// each its rank in the cell-sorted order, and the tile is written in the
// transposed layout (tile_pos), so that a coalesced read hands the lanes of a
// wave particles of different cells.  Each particle is written with its new
// position (formed again from x^n and the increment), its momentum p^(k+1)
// and its id.  When the tile's sources and particles fit INVCAP, every output
// array passes through LDS (sources read in order, values placed at their new
// positions, the tile written in order); a fuller tile writes each particle to
// its position directly.
constexpr int INVCAP = 6144;

constexpr int SORT_THREADS = 512;

struct Resort {
    const double *xi1, *xi2, *d1, *d2, *pk1, *pk2;
    const int32_t *sid, *word, *mig, *told, *tnew, *tstay;
    double *o1, *o2, *r1, *r2;
    int32_t *did;
    int M1, M2;
    double inv_dx1, inv_dx2;
    const double *ss[3];   // spins (null without spin)
    double *os[3];
    __device__ __forceinline__ void put(int j, int i) const {
        o1[j] = new_coord(xi1[i], d1[i], inv_dx1, M1);
        o2[j] = new_coord(xi2[i], d2[i], inv_dx2, M2);
        r1[j] = pk1[i];
        r2[j] = pk2[i];
        did[j] = sid[i];
        if (ss[0])
            for (int q = 0; q < 3; ++q) os[q][j] = ss[q][i];
    }
};

// Particles per thread whose loads the re-sort issues together.
constexpr int RB = 4;

__global__ __launch_bounds__(SORT_THREADS) void k2_tile_resort(Resort a) {
    constexpr int NW = SORT_THREADS / WAVE;
    __shared__ int hist[WAVE], cur[WAVE];
    __shared__ int wcnt[NW][WAVE], woff[NW][WAVE];
    __shared__ int pos[INVCAP];      // new position in the tile of source q (-1: it left)
    __shared__ double val[INVCAP];   // one output array of the tile, by new position
    const int T = tile_of_block();
    const int ob = a.told[T], nold = a.told[T + 1] - ob;
    const int base = a.tnew[T], cnt = a.tnew[T + 1] - base, arr0 = base + a.tstay[T];
    const int nsrc = nold + cnt - a.tstay[T];
    const int nt = blockDim.x, wv = threadIdx.x / WAVE;
    // source q < nold: old position q of the tile; q >= nold: listed arrival
    auto source = [&](int q) { return q < nold ? ob + q : a.mig[arr0 + q - nold]; };
    if (threadIdx.x < WAVE) hist[threadIdx.x] = 0;
    for (int k = threadIdx.x; k < NW * WAVE; k += nt) wcnt[k / WAVE][k % WAVE] = 0;
    __syncthreads();
    // column counts (any order)
    for (int q0 = threadIdx.x; q0 < nsrc; q0 += RB * nt) {
        int w[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) w[k] = q0 + k * nt < nsrc ? a.word[source(q0 + k * nt)] : -1;
#pragma unroll
        for (int k = 0; k < RB; ++k)
            if (w[k] >= 0 && (w[k] >> 6) == T) atomicAdd(&hist[w[k] & 63], 1);
    }
    __syncthreads();
    if (threadIdx.x < WAVE) {   // exclusive prefix over the 64 columns
        const int v = hist[threadIdx.x];
        int inc = v;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const int u = __shfl_up(inc, o, WAVE);
            if ((int)threadIdx.x >= o) inc += u;
        }
        cur[threadIdx.x] = inc - v;
    }
    __syncthreads();
    // Stable ranks: the sources in the old cell-sorted order (old rank t at
    // position tile_pos(t)), then the arrivals, a block of them at a time;
    // inside a wave the lanes of one column count the lower lanes of that
    // column, across waves a per-column prefix.  Rank r goes to position
    // tile_pos(r) of the new tile.
    const bool direct = cnt > INVCAP || nsrc > INVCAP;
    for (int t0 = 0; t0 < nsrc; t0 += nt) {   // uniform over the block
        const int t = t0 + threadIdx.x;
        int q = -1, key = -1;
        if (t < nsrc) {
            q = t < nold ? tile_pos(t, nold) : t;
            const int w = a.word[source(q)];
            if ((w >> 6) == T) key = w & 63;
        }
        unsigned long long rem = __builtin_amdgcn_ballot_w64(key >= 0);
        int wr = 0;
        while (rem) {
            const int leader = __builtin_ctzll(rem);
            const int lk = __shfl(key, leader, WAVE);
            const unsigned long long m = __builtin_amdgcn_ballot_w64(key == lk);
            if (key == lk) wr = rank_in(m);
            if (lane_id() == leader) wcnt[wv][lk] = __builtin_popcountll(m);
            rem &= ~m;
        }
        __syncthreads();
        if (threadIdx.x < WAVE) {
            int run = cur[threadIdx.x];
            for (int v = 0; v < NW; ++v) {
                const int c = wcnt[v][threadIdx.x];
                wcnt[v][threadIdx.x] = 0;
                woff[v][threadIdx.x] = run;
                run += c;
            }
            cur[threadIdx.x] = run;
        }
        __syncthreads();
        if (q >= 0) {
            const int p = key >= 0 ? tile_pos(woff[wv][key] + wr, cnt) : -1;
            if (direct) {
                if (p >= 0) a.put(base + p, source(q));
            } else {
                pos[q] = p;
            }
        }
    }
    if (direct) return;   // uniform over the block
    // One output array at a time: the old tile read in order (and the
    // arrivals), each value placed in LDS at its new position, the tile written
    // in order.
    const int nf = a.ss[0] ? 8 : 5;   // with spin: s_x, s_y, s_z as well
    for (int f = 0; f < nf; ++f) {
        __syncthreads();
        for (int q0 = threadIdx.x; q0 < nsrc; q0 += RB * nt) {
            int i[RB], p[RB];
            double v[RB];
#pragma unroll
            for (int k = 0; k < RB; ++k) {
                const int q = q0 + k * nt;
                p[k] = q < nsrc ? pos[q] : -1;
                i[k] = p[k] >= 0 ? source(q) : -1;
            }
#pragma unroll
            for (int k = 0; k < RB; ++k) {
                if (i[k] < 0) continue;
                switch (f) {
                    case 0: v[k] = new_coord(a.xi1[i[k]], a.d1[i[k]], a.inv_dx1, a.M1); break;
                    case 1: v[k] = new_coord(a.xi2[i[k]], a.d2[i[k]], a.inv_dx2, a.M2); break;
                    case 2: v[k] = a.pk1[i[k]]; break;
                    case 3: v[k] = a.pk2[i[k]]; break;
                    case 4: v[k] = (double)a.sid[i[k]]; break;
                    default: v[k] = a.ss[f - 5][i[k]]; break;
                }
            }
#pragma unroll
            for (int k = 0; k < RB; ++k)
                if (i[k] >= 0) val[p[k]] = v[k];
        }
        __syncthreads();
        double *out = f == 0 ? a.o1 : f == 1 ? a.o2 : f == 2 ? a.r1 : f == 3 ? a.r2 : f == 4 ? nullptr : a.os[f - 5];
        for (int p = threadIdx.x; p < cnt; p += nt) {
            if (f != 4) out[base + p] = val[p];
            else a.did[base + p] = (int32_t)val[p];
        }
    }
}

// ---------------------------------------------------------------------------
// Subsystem III particle term and the charge deposit (tiles, no motion)
// ---------------------------------------------------------------------------
struct DepArgs {
    const double *xi1, *xi2, *p1, *p2;
    const int32_t *start;   // first particle of each tile (ntiles + 1)
    const double *an;    // a_z^n                     (III)
    const double *ezn;   // e_z^n                     (III)
    const double *ezk;   // e_z^(k)                   (III)
    double *S;           // deposit target (zero on entry)
    double *anp;         // A^n at each particle (III): written on the first iteration, read after
    int M1, M2, TW;
    double dt, w;
    int mode;            // 0: charge w Lambda0; 1: Subsystem III source
    int first;           // III: first iteration of the substep
    const int *gate;     // III: nonzero once an earlier iteration converged (nothing to do)
};

// mode 1: S += w (A^n + A^(k)) / (gamma(p, A^n) + gamma(p, A^(k))) Lambda0(x_a),
// with A^(k) the field of a^(k) = a^n - dt (e^n + e^(k)) / 2.
template <int P>
__global__ __launch_bounds__(BLOCK) void k2_deposit0(DepArgs a) {
    if (a.gate && *a.gate) return;   // uniform over the grid
    constexpr int PR = P + 1, PCM = TWMAX + P, PS = PR * PCM;
    __shared__ double sAn[PS], sAk[PS], sS[PS];
    const int nseg = a.M2 / a.TW;
    const int tile = tile_of_block();
    const int r = tile / nseg, c0 = (tile - r * nseg) * a.TW;
    const int PC = a.TW + P;
    const int R0 = r - P, C0 = c0 - P;
    for (int t = threadIdx.x; t < PR * PC; t += blockDim.x) {
        const int i = t / PC, j = t - i * PC;
        const int g = wrapi(R0 + i, a.M1) * a.M2 + wrapi(C0 + j, a.M2);
        if (a.mode == 1) {
            const double an = a.an[g];
            if (a.first) sAn[t] = an;
            sAk[t] = an - 0.5 * a.dt * (a.ezn[g] + a.ezk[g]);
        }
        sS[t] = 0.0;
    }
    __syncthreads();
    const int begin = a.start[tile], end = a.start[tile + 1];
    const int nw = blockDim.x / WAVE, passes = (end - begin + WAVE - 1) / WAVE;   // none for an empty tile
    for (int jr = threadIdx.x / WAVE; jr < passes; jr += nw) {
        const int i = begin + jr * WAVE + lane_id();
        const bool live = i < end;
        const int ii = live ? i : begin;
        const double u1 = a.xi1[ii], u2 = a.xi2[ii];
        const int c2 = (int)u2;
        double b1[P + 1], b2[P + 1];
        basis_values<P>(u1 - r, b1);
        basis_values<P>(u2 - c2, b2);
        double q = a.w;
        if (a.mode == 1) {
            double An = 0.0, Ak = 0.0;
#pragma unroll
            for (int m1 = 0; m1 <= P; ++m1) {
                double tn = 0.0, tk = 0.0;
#pragma unroll
                for (int m2 = 0; m2 <= P; ++m2) {
                    const int s = (r - m1 - R0) * PC + c2 - m2 - C0;
                    if (a.first) tn += b2[m2] * sAn[s];
                    tk += b2[m2] * sAk[s];
                }
                An += b1[m1] * tn;
                Ak += b1[m1] * tk;
            }
            if (a.first) {
                if (live) a.anp[i] = An;
            } else {
                An = a.anp[ii];
            }
            const double q1 = a.p1[ii], q2 = a.p2[ii], pp = 1.0 + q1 * q1 + q2 * q2;
            q = a.w * (An + Ak) * frcp(fsqrt(pp + An * An) + fsqrt(pp + Ak * Ak));
        }
        if (live) {
#pragma unroll
            for (int m1 = 0; m1 <= P; ++m1) {
                const double qb = q * b1[m1];
#pragma unroll
                for (int m2 = 0; m2 <= P; ++m2) atomicAdd(&sS[(r - m1 - R0) * PC + c2 - m2 - C0], qb * b2[m2]);
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < PR * PC; t += blockDim.x) {
        const int i = t / PC, j = t - i * PC;
        const int g = wrapi(R0 + i, a.M1) * a.M2 + wrapi(C0 + j, a.M2);
        if (sS[t] != 0.0) atomicAdd(&a.S[g], sS[t]);
    }
}

// Subsystem II over tiles: B_z (V2) and A_z (V0) gathered from the tile's LDS
// patch, every momentum turned by the angle B_z dt / gamma.  SPIN: every spin
// also turns about B_h = (dA_z/dx2, -dA_z/dx1, B_z) by the angle -|B_h| dt
// (ds/dt = s x B_h, Rodrigues' formula), with G a_z staged as well.
struct RotArgs {
    const double *xi1, *xi2;
    double *p1, *p2, *sx, *sy, *sz;
    const int32_t *start;
    const double *bz, *az, *g1, *g2;
    int M1, M2, TW;
    double dt;
};

template <int P, bool SPIN>
__global__ __launch_bounds__(BLOCK) void k2_rotate_tiles(RotArgs a) {
    constexpr int PR = P + 1, PCM = TWMAX + P, PS = PR * PCM;
    __shared__ double sA[PS], sB[PS], sG1[SPIN ? PS : 1], sG2[SPIN ? PS : 1];
    const int nseg = a.M2 / a.TW;
    const int tile = tile_of_block();
    const int r = tile / nseg, c0 = (tile - r * nseg) * a.TW;
    const int PC = a.TW + P;
    const int R0 = r - P, C0 = c0 - P;
    for (int t = threadIdx.x; t < PR * PC; t += blockDim.x) {
        const int i = t / PC, j = t - i * PC;
        const int g = wrapi(R0 + i, a.M1) * a.M2 + wrapi(C0 + j, a.M2);
        sA[t] = a.az[g];
        sB[t] = a.bz[g];
        if constexpr (SPIN) {
            sG1[t] = a.g1[g];
            sG2[t] = a.g2[g];
        }
    }
    __syncthreads();
    const int begin = a.start[tile], end = a.start[tile + 1];
    for (int i = begin + threadIdx.x; i < end; i += blockDim.x) {
        const double u1 = a.xi1[i], u2 = a.xi2[i];
        const int c2 = (int)u2;
        const double t1 = u1 - r, t2 = u2 - c2;
        double a1[P + 1], a2[P + 1], b1[P], b2[P];
        basis_values<P>(t1, a1);
        basis_values<P>(t2, a2);
        basis_values<P - 1>(t1, b1);
        basis_values<P - 1>(t2, b2);
        double A = 0.0, B = 0.0, Bx = 0.0, By = 0.0;
#pragma unroll
        for (int m1 = 0; m1 <= P; ++m1) {
            double ta = 0.0, tb = 0.0, tx = 0.0, ty = 0.0;
#pragma unroll
            for (int m2 = 0; m2 <= P; ++m2) {
                const int s = (r - m1 - R0) * PC + c2 - m2 - C0;
                ta += a2[m2] * sA[s];
                if (m1 < P && m2 < P) tb += b2[m2] * sB[s];
                if constexpr (SPIN) {
                    if (m2 < P) tx += b2[m2] * sG2[s];   // dA_z/dx2: degrees (P, P-1)
                    if (m1 < P) ty += a2[m2] * sG1[s];   // dA_z/dx1: degrees (P-1, P)
                }
            }
            A += a1[m1] * ta;
            if (m1 < P) B += b1[m1] * tb;
            if constexpr (SPIN) {
                Bx += a1[m1] * tx;
                if (m1 < P) By -= b1[m1] * ty;
            }
        }
        const double q1 = a.p1[i], q2 = a.p2[i];
        const double th = B * a.dt / sqrt(1.0 + q1 * q1 + q2 * q2 + A * A);
        double sn, cs;
        sincos(th, &sn, &cs);
        a.p1[i] = q1 * cs + q2 * sn;
        a.p2[i] = -q1 * sn + q2 * cs;
        if constexpr (SPIN) {
            const double nb = sqrt(Bx * Bx + By * By + B * B);
            if (nb > 0.0) {
                const double k0 = Bx / nb, k1 = By / nb, k2 = B / nb;
                const double s0 = a.sx[i], s1 = a.sy[i], s2 = a.sz[i];
                const double x0 = k1 * s2 - k2 * s1, x1 = k2 * s0 - k0 * s2, x2 = k0 * s1 - k1 * s0;
                const double ks = k0 * s0 + k1 * s1 + k2 * s2;
                double sb, cb;
                sincos(nb * a.dt, &sb, &cb);
                a.sx[i] = s0 * cb - x0 * sb + k0 * ks * (1.0 - cb);
                a.sy[i] = s1 * cb - x1 * sb + k1 * ks * (1.0 - cb);
                a.sz[i] = s2 * cb - x2 * sb + k2 * ks * (1.0 - cb);
            }
        }
    }
}

// a^{n+1} = a^n - dt (e^n + e^{n+1}) / 2, e_z = e^{n+1}.
__global__ void k2_finish_III(double *__restrict__ az, double *__restrict__ ez, const double *__restrict__ ezn,
                              const double *__restrict__ ezk, int N, double dt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        az[i] -= 0.5 * dt * (ezn[i] + ezk[i]);
        ez[i] = ezk[i];
    }
}

// ---------------------------------------------------------------------------
// Diagnostics: kinetic energy, quadratic forms, Gauss residual
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(BLOCK) void k2_kinetic(const double *__restrict__ xi1, const double *__restrict__ xi2,
                           const double *__restrict__ p1, const double *__restrict__ p2,
                           const double *__restrict__ az, int64_t n, int M1, int M2, double w,
                           double *__restrict__ partial) {
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double u1 = xi1[i], u2 = xi2[i];
        const int c1 = (int)u1, c2 = (int)u2;
        const double A = gather00<P>(az, M1, M2, c1, c2, u1 - c1, u2 - c2);
        const double q1 = p1[i], q2 = p2[i];
        const double pp = q1 * q1 + q2 * q2 + A * A;
        s += w * pp / (sqrt(1.0 + pp) + 1.0);   // gamma - 1 without cancellation
    }
    block_sum_to(s, &partial[blockIdx.x]);
}

struct MassRows {
    double r1[11], r2[11];   // rows of the 1D mass matrices (dimensionless), 2d+1 entries
    int d1, d2;
    double scale;            // dx1 dx2
};

// y = (Mass_{d1} (x) Mass_{d2}) x on the periodic grid.
__global__ __launch_bounds__(BLOCK) void k2_mass(const double *__restrict__ x, double *__restrict__ y, int M1, int M2, MassRows m) {
    const int N = M1 * M2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const int i1 = i / M2, i2 = i - i1 * M2;
        double s = 0.0;
        for (int k1 = -m.d1; k1 <= m.d1; ++k1) {
            const double *row = x + wrapi(i1 + k1, M1) * M2;
            double t = 0.0;
            for (int k2 = -m.d2; k2 <= m.d2; ++k2) t += m.r2[k2 + m.d2] * row[wrapi(i2 + k2, M2)];
            s += m.r1[k1 + m.d1] * t;
        }
        y[i] = m.scale * s;
    }
}

// partial[block] = sum of x_i y_i over the block's nodes.
__global__ void k2_dot(const double *__restrict__ x, const double *__restrict__ y, int N, double *partial) {
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) s += x[i] * y[i];
    block_sum_to(s, &partial[blockIdx.x]);
}

// out = sum of partial[0..n) in order (one block).
__global__ void k2_sum(const double *__restrict__ partial, int n, double *out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
    block_sum_to(s, out);
}

// r = G^T u + rho - dx1 dx2 with u = M1 e (two components); max |r| into *res.
__global__ __launch_bounds__(BLOCK) void k2_gauss(const double *__restrict__ u1, const double *__restrict__ u2,
                         const double *__restrict__ rho, double *__restrict__ r, int M1, int M2, double inv_dx1,
                         double inv_dx2, double cell_area, unsigned long long *res) {
    const int N = M1 * M2;
    double m = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const int i1 = i / M2, i2 = i - i1 * M2;
        const double v = (u1[i] - u1[wrapi(i1 + 1, M1) * M2 + i2]) * inv_dx1 +
                         (u2[i] - u2[i1 * M2 + wrapi(i2 + 1, M2)]) * inv_dx2 + rho[i] - cell_area;
        r[i] = v;
        m = fmax(m, fabs(v));
    }
    block_max_to(m, res);
}

// End of one fixed-point iteration (unless an earlier one converged): its
// residuals ra, rb (rb may be null) and the status flags (may be null) go to
// the host mirror h[0..2], and the gate closes when a flag is set, a residual
// is not finite, or the larger one is at most tol: the conditions on which the
// host stops at this iteration.
__global__ void k2_check(const unsigned long long *ra, const unsigned long long *rb, const int *flags, double tol,
                         int *gate, double *h) {
    if (*gate) return;
    double a, b = 0.0;
    const unsigned long long ba = *ra, bb = rb ? *rb : 0ull;
    memcpy(&a, &ba, sizeof(a));
    memcpy(&b, &bb, sizeof(b));
    const int f = flags ? *flags : 0;
    h[0] = a;
    h[1] = b;
    h[2] = (double)f;
    if (f || !isfinite(a) || !isfinite(b) || fmax(a, b) <= tol) *gate = 1;
}

// ---------------------------------------------------------------------------
// Spectral solves: 2D FFT (rows, then columns with the spectral step fused)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <bool INV>
__device__ __forceinline__ double2 mul_i(double2 a) {   // a exp(-+ i pi / 2): -i a forward, +i a inverse
    return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// DFT of R = 2, 4 or 8 points in registers: X_q = sum_r v_r exp(-+ 2 pi i r q / R)
// (the + sign for INV).
template <int R, bool INV>
__device__ __forceinline__ void dft_reg(double2 (&v)[R]) {
    if constexpr (R == 2) {
        const double2 a = v[0], b = v[1];
        v[0] = make_double2(a.x + b.x, a.y + b.y);
        v[1] = make_double2(a.x - b.x, a.y - b.y);
    } else if constexpr (R == 4) {
        const double2 s02 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
        const double2 d02 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
        const double2 s13 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
        const double2 d13 = mul_i<INV>(make_double2(v[1].x - v[3].x, v[1].y - v[3].y));
        v[0] = make_double2(s02.x + s13.x, s02.y + s13.y);
        v[2] = make_double2(s02.x - s13.x, s02.y - s13.y);
        v[1] = make_double2(d02.x + d13.x, d02.y + d13.y);
        v[3] = make_double2(d02.x - d13.x, d02.y - d13.y);
    } else {
        double2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        dft_reg<4, INV>(e);
        dft_reg<4, INV>(o);
        constexpr double c = 0.70710678118654752440;
        o[1] = cmul(o[1], make_double2(c, INV ? c : -c));
        o[2] = mul_i<INV>(o[2]);
        o[3] = cmul(o[3], make_double2(-c, INV ? c : -c));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = make_double2(e[q].x + o[q].x, e[q].y + o[q].y);
            v[q + 4] = make_double2(e[q].x - o[q].x, e[q].y - o[q].y);
        }
    }
}

// FFT of n = 2^k points (8 <= n <= MAXM), Stockham autosort with radix-8
// stages and one final radix-2 or radix-4 stage when k is not a multiple of 3.
// A transform is spread over T = n / 8 threads; thread t holds the 8 values at
// positions t + m T (m < 8) in x, before and after.  In a stage of radix R
// after Ns points have been combined, butterfly j = t + q T (q < 8 / R) takes
// the inputs j + r n / R (x[q + r 8/R]), multiplies input r by
// w^(r (j mod Ns) n / (Ns R)) with w = exp(-+ 2 pi i / n), and sends output r
// to (j - j mod Ns) R + j mod Ns + r Ns.  Between stages the values pass
// through LDS (position p of this transform at lds[base + p sp]); the last
// stage's outputs are this thread's own positions, so they stay in registers.
// stw holds w^m for m < n / 2.  Every thread of the block takes part (the
// stages synchronise the block).
template <int R, bool INV>
__device__ __forceinline__ void fft_stage(double2 (&x)[8], int t, int T, int n, int Ns, bool last, double2 *lds,
                                          int sp, int base, const double2 *stw) {
    constexpr int Q = 8 / R;
    const int step = n / (Ns * R), h = n >> 1;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = t + q * T, k = j & (Ns - 1);
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double2 a = x[q + r * Q];
            if (r > 0) {
                const int m = r * k * step;
                double2 w = m < h ? stw[m] : make_double2(-stw[m - h].x, -stw[m - h].y);
                if (INV) w.y = -w.y;
                a = cmul(a, w);
            }
            v[r] = a;
        }
        dft_reg<R, INV>(v);
        const int o = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (last)
                x[q + r * Q] = v[r];
            else
                lds[base + (o + r * Ns) * sp] = v[r];
        }
    }
    if (!last) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = lds[base + (t + m * T) * sp];
        __syncthreads();
    }
}

template <bool INV>
__device__ void fft8(double2 (&x)[8], int t, int n, double2 *lds, int sp, int base, const double2 *stw) {
    const int T = n >> 3;
    const int e = 31 - __clz(n), n8 = e / 3, rem = e % 3;
    int Ns = 1;
    for (int s = 0; s < n8; ++s) {
        fft_stage<8, INV>(x, t, T, n, Ns, s == n8 - 1 && rem == 0, lds, sp, base, stw);
        Ns <<= 3;
    }
    if (rem == 1) fft_stage<2, INV>(x, t, T, n, Ns, true, lds, sp, base, stw);
    if (rem == 2) fft_stage<4, INV>(x, t, T, n, Ns, true, lds, sp, base, stw);
}

template <int NB>
struct Ptrs {
    double *p[NB];
};

// Forward transform along x2 of NB real grids, one transform per (grid, row)
// over M2 / 8 threads; bit b of zero_mask zeroes grid b after it is read (the
// accumulators of the next deposit).
template <int NB>
__global__ __launch_bounds__(BLOCK) void k2_fft_rows_fwd(Ptrs<NB> src, int zero_mask, double2 *__restrict__ Z,
                                                         int M1, int M2, const double2 *__restrict__ tw2,
                                                         const int *gate) {
    if (gate && *gate) return;   // uniform over the grid
    __shared__ double2 lds[8 * BLOCK], stw[MAXM / 2];
    const int n = M2, T = n >> 3, per = BLOCK / T;
    const int fl = threadIdx.x / T, t = threadIdx.x - fl * T, f = blockIdx.x * per + fl;
    const bool act = f < NB * M1;
    const int b = act ? f / M1 : 0, row = act ? f - b * M1 : 0;
    for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) stw[i] = tw2[i];
    double *s = src.p[0];
#pragma unroll
    for (int q = 1; q < NB; ++q)
        if (b == q) s = src.p[q];
    s += (size_t)row * M2;
    const bool zero = (zero_mask >> b) & 1;
    double2 x[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        x[m] = make_double2(act ? s[t + m * T] : 0.0, 0.0);
        if (act && zero) s[t + m * T] = 0.0;
    }
    __syncthreads();
    fft8<false>(x, t, n, lds, 1, fl * n, stw);
    if (act) {
        double2 *z = Z + (size_t)b * M1 * M2 + (size_t)row * M2;
#pragma unroll
        for (int m = 0; m < 8; ++m) z[t + m * T] = x[m];
    }
}

// 1D symbols of the spectral step, per direction (length M1 and M2): the mass
// matrices' eigenvalues m0, m1 (dx included) and the backward difference
// (1 - exp(-i theta)) / dx as (cr, ci).
struct Sym {
    const double *m0a, *m1a, *cra, *cia;
    const double *m0b, *m1b, *crb, *cib;
};

// Along x1 for NB grids: forward transform of each grid's column, the spectral
// step op(k1, k2, v) on every frequency (all NB grids at once, in registers),
// then (if op.INVERSE) the inverse transforms, written back to Z.  The block's
// BLOCK / (M1 / 8) columns are adjacent and consecutive threads take
// consecutive columns, so every row access is contiguous; adjacent column
// groups go to blocks on the same XCD.
template <int NB, class Op>
__global__ __launch_bounds__(BLOCK) void k2_fft_cols(double2 *__restrict__ Z, int M1, int M2,
                                                     const double2 *__restrict__ tw1, Op op, const int *gate) {
    if (gate && *gate) return;   // uniform over the grid
    __shared__ double2 lds[8 * BLOCK], stw[MAXM / 2];
    const int n = M1, T = n >> 3, per = BLOCK / T;
    const int c = threadIdx.x % per, t = threadIdx.x / per;
    const int col = tile_of_block() * per + c;
    const bool act = col < M2;
    const size_t N = (size_t)M1 * M2;
    for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) stw[i] = tw1[i];
    double2 x[NB][8];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int m = 0; m < 8; ++m)
            x[b][m] = act ? Z[b * N + (size_t)(t + m * T) * M2 + col] : make_double2(0.0, 0.0);
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) fft8<false>(x[b], t, n, lds, per, c, stw);
    if (act) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            double2 v[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) v[b] = x[b][m];
            op(t + m * T, col, v);
#pragma unroll
            for (int b = 0; b < NB; ++b) x[b][m] = v[b];
        }
    }
    if constexpr (Op::INVERSE) {
#pragma unroll
        for (int b = 0; b < NB; ++b) fft8<true>(x[b], t, n, lds, per, c, stw);
        if (act) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int m = 0; m < 8; ++m) Z[b * N + (size_t)(t + m * T) * M2 + col] = x[b][m];
        }
    }
}

// Inverse transform along x2 of NB grids, scaled by 1/(M1 M2); the real part of
// entry g of grid b goes to epi(b, g, v), whose return values are max-reduced
// into epi.res (if set).
template <int NB, class Epi>
__global__ __launch_bounds__(BLOCK) void k2_fft_rows_inv(const double2 *__restrict__ Z, int M1, int M2,
                                                         const double2 *__restrict__ tw2, double invN, Epi epi,
                                                         const int *gate) {
    if (gate && *gate) return;   // uniform over the grid
    __shared__ double2 lds[8 * BLOCK], stw[MAXM / 2];
    const int n = M2, T = n >> 3, per = BLOCK / T;
    const int fl = threadIdx.x / T, t = threadIdx.x - fl * T, f = blockIdx.x * per + fl;
    const bool act = f < NB * M1;
    const int b = act ? f / M1 : 0, row = act ? f - b * M1 : 0;
    for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) stw[i] = tw2[i];
    const double2 *z = Z + (size_t)b * M1 * M2 + (size_t)row * M2;
    double2 x[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) x[m] = act ? z[t + m * T] : make_double2(0.0, 0.0);
    __syncthreads();
    fft8<true>(x, t, n, lds, 1, fl * n, stw);
    double mx = 0.0;
    if (act) {
#pragma unroll
        for (int m = 0; m < 8; ++m) mx = fmax(mx, epi(b, row * M2 + t + m * T, x[m].x * invN));
    }
    if (epi.res) block_max_to(mx, epi.res);
}

// ---- spectral steps -------------------------------------------------------
// M1^{-1} on the current (Subsystem I): component 1 has symbol m1(t1) m0(t2),
// component 2 m0(t1) m1(t2).
struct OpM1inv {
    static constexpr bool INVERSE = true;
    Sym s;
    __device__ void operator()(int k1, int k2, double2 (&v)[2]) const {
        const double d1 = 1.0 / (s.m1a[k1] * s.m0b[k2]), d2 = 1.0 / (s.m0a[k1] * s.m1b[k2]);
        v[0].x *= d1; v[0].y *= d1;
        v[1].x *= d2; v[1].y *= d2;
    }
};

// e^{(k+1)} = e^n - M1^{-1} J; residual |e^{(k+1)} - e^{(k)}|; ebar = (e^n + e^{(k+1)})/2.
struct EpiI {
    const double *en1, *en2;
    double *ek1, *ek2, *eb1, *eb2;
    unsigned long long *res;
    __device__ double operator()(int b, int g, double v) const {
        const double en = b ? en2[g] : en1[g];
        double *ek = b ? ek2 : ek1;
        double *eb = b ? eb2 : eb1;
        const double e = en - v;
        const double d = fabs(e - ek[g]);
        ek[g] = e;
        eb[g] = 0.5 * (en + e);
        return isfinite(d) ? d : HUGE_VAL;   // a non-finite field shows in the residual
    }
};

__device__ __forceinline__ double kappa(const Sym &s, int k1, int k2) {   // symbol of K = G^T M1 G
    const double c1 = s.cra[k1] * s.cra[k1] + s.cia[k1] * s.cia[k1];
    const double c2 = s.crb[k2] * s.crb[k2] + s.cib[k2] * s.cib[k2];
    return c1 * s.m1a[k1] * s.m0b[k2] + c2 * s.m0a[k1] * s.m1b[k2];
}

// Subsystem III constant part: R = (M0 - q K) e^n + dt K a^n (q = dt^2/4), kept in Fourier space.
struct OpIIIrhs {
    static constexpr bool INVERSE = false;
    Sym s;
    double2 *R;
    int M2;
    double dt;
    __device__ void operator()(int k1, int k2, double2 (&v)[2]) const {
        const double kp = kappa(s, k1, k2), m0 = s.m0a[k1] * s.m0b[k2];
        const double ce = m0 - 0.25 * dt * dt * kp, ca = dt * kp;
        R[(size_t)k1 * M2 + k2] = make_double2(ce * v[0].x + ca * v[1].x, ce * v[0].y + ca * v[1].y);
    }
};

// With spin (v[2] = G*^T Lambda1*^T W S_xy): R gains dt hbar v[2].
struct OpIIIrhsS {
    static constexpr bool INVERSE = false;
    Sym s;
    double2 *R;
    int M2;
    double dt, hbar;
    __device__ void operator()(int k1, int k2, double2 (&v)[3]) const {
        const double kp = kappa(s, k1, k2), m0 = s.m0a[k1] * s.m0b[k2];
        const double ce = m0 - 0.25 * dt * dt * kp, ca = dt * kp, cs = dt * hbar;
        R[(size_t)k1 * M2 + k2] = make_double2(ce * v[0].x + ca * v[1].x + cs * v[2].x,
                                               ce * v[0].y + ca * v[1].y + cs * v[2].y);
    }
};

// Subsystem III solve: e = (R + dt S) / (M0 + q K).
struct OpIII {
    static constexpr bool INVERSE = true;
    Sym s;
    const double2 *R;
    int M2;
    double dt;
    __device__ void operator()(int k1, int k2, double2 (&v)[1]) const {
        const double lam = s.m0a[k1] * s.m0b[k2] + 0.25 * dt * dt * kappa(s, k1, k2);
        const double2 r = R[(size_t)k1 * M2 + k2];
        v[0] = make_double2((r.x + dt * v[0].x) / lam, (r.y + dt * v[0].y) / lam);
    }
};

struct EpiIII {
    double *ezk;
    unsigned long long *res;
    __device__ double operator()(int, int g, double v) const {
        const double d = fabs(v - ezk[g]);
        ezk[g] = v;
        return isfinite(d) ? d : HUGE_VAL;   // a non-finite field shows in the residual
    }
};

// Subsystem IV in Fourier space (v = e1, e2, b): with c_k = (1 - exp(-i t_k))/dx_k and
// sigma = |c1|^2 m1a/m0a + |c2|^2 m1b/m0b the symbol of C M1^{-1} C^T M2,
//   b' = ((1 - q sigma) b - dt (c1 e2 - c2 e1)) / (1 + q sigma),
//   e1' = e1 - dt conj(c2) (m1b/m0b) (b + b')/2,  e2' = e2 + dt conj(c1) (m1a/m0a) (b + b')/2,
// the implicit midpoint step of the Maxwell subsystem eliminated for b.
// One Fourier mode of the Maxwell step (e1, e2, b in place).
__device__ __forceinline__ void maxwell_mode(const Sym &s, double dt, int k1, int k2, double2 &e1, double2 &e2,
                                             double2 &b) {
    const double2 c1 = make_double2(s.cra[k1], s.cia[k1]), c2 = make_double2(s.crb[k2], s.cib[k2]);
    const double ra = s.m1a[k1] / s.m0a[k1], rb = s.m1b[k2] / s.m0b[k2];
    const double sig = (c1.x * c1.x + c1.y * c1.y) * ra + (c2.x * c2.x + c2.y * c2.y) * rb;
    const double q = 0.25 * dt * dt;
    const double2 t1 = cmul(c1, e2), t2 = cmul(c2, e1);
    const double2 ce = make_double2(t1.x - t2.x, t1.y - t2.y);
    const double den = 1.0 / (1.0 + q * sig), num = 1.0 - q * sig;
    const double2 bn = make_double2((num * b.x - dt * ce.x) * den, (num * b.y - dt * ce.y) * den);
    const double2 bm = make_double2(0.5 * (b.x + bn.x), 0.5 * (b.y + bn.y));
    const double2 u1 = cmul(make_double2(c2.x, -c2.y), bm), u2 = cmul(make_double2(c1.x, -c1.y), bm);
    e1 = make_double2(e1.x - dt * rb * u1.x, e1.y - dt * rb * u1.y);
    e2 = make_double2(e2.x + dt * ra * u2.x, e2.y + dt * ra * u2.y);
    b = bn;
}

struct OpIV {
    static constexpr bool INVERSE = true;
    Sym s;
    double dt;
    __device__ void operator()(int k1, int k2, double2 (&v)[3]) const { maxwell_mode(s, dt, k1, k2, v[0], v[1], v[2]); }
};

// With spin the b_z equation carries hbar Lambda2^T W S_z (v[3], constant): with
// b~ = b + hbar M2^{-1} D_z the scheme is the one without spin, so b~ is stepped
// and the shift taken off again.
struct OpIVs {
    static constexpr bool INVERSE = true;
    Sym s;
    double dt, hbar;
    __device__ void operator()(int k1, int k2, double2 (&v)[4]) const {
        const double sh = hbar / (s.m1a[k1] * s.m1b[k2]);
        double2 b = make_double2(v[2].x + sh * v[3].x, v[2].y + sh * v[3].y);
        maxwell_mode(s, dt, k1, k2, v[0], v[1], b);
        v[2] = make_double2(b.x - sh * v[3].x, b.y - sh * v[3].y);
    }
};

// Gauss-law correction (v = e1, e2, rho): r = G^T M1 e + rho (the constant part
// lives in the mean, which phi does not see), phi = r / kappa, e -= G phi.
struct OpPoisson {
    static constexpr bool INVERSE = true;
    Sym s;
    __device__ void operator()(int k1, int k2, double2 (&v)[3]) const {
        if (k1 == 0 && k2 == 0) return;
        const double2 c1 = make_double2(s.cra[k1], s.cia[k1]), c2 = make_double2(s.crb[k2], s.cib[k2]);
        const double w1 = s.m1a[k1] * s.m0b[k2], w2 = s.m0a[k1] * s.m1b[k2];
        const double2 a = cmul(make_double2(c1.x, -c1.y), v[0]), b = cmul(make_double2(c2.x, -c2.y), v[1]);
        const double kp = kappa(s, k1, k2);
        const double2 phi = make_double2((w1 * a.x + w2 * b.x + v[2].x) / kp, (w1 * a.y + w2 * b.y + v[2].y) / kp);
        const double2 g1 = cmul(c1, phi), g2 = cmul(c2, phi);
        v[0] = make_double2(v[0].x - g1.x, v[0].y - g1.y);
        v[1] = make_double2(v[1].x - g2.x, v[1].y - g2.y);
    }
};

template <int NB>
struct EpiStore {
    Ptrs<NB> out;
    unsigned long long *res;
    __device__ double operator()(int b, int g, double v) const {
#pragma unroll
        for (int q = 0; q < NB; ++q)
            if (b == q && out.p[q]) out.p[q][g] = v;
        return 0.0;
    }
};

}  // namespace ecpic2d

// ===========================================================================
// Host side
// ===========================================================================
using namespace ecpic2d;

namespace {

int64_t eulerian2(int n, int k) {   // A(n, k) = sum_j (-1)^j C(n+1, j) (k+1-j)^n
    int64_t s = 0;
    for (int j = 0; j <= k; ++j) {
        int64_t b = 1;
        for (int q = 1; q <= j; ++q) b = b * (n + 1 - j + q) / q;
        int64_t pw = 1;
        for (int q = 0; q < n; ++q) pw *= (k + 1 - j);
        s += (j % 2 == 0) ? b * pw : -b * pw;
    }
    return s;
}

// Row of the degree-d B-spline mass matrix with dx = 1: the cardinal B-spline of
// degree 2d+1 at the integers, A(2d+1, k) / (2d+1)!.
std::vector<double> mass_row2(int d) {
    const int n = 2 * d + 1;
    double f = 1.0;
    for (int q = 2; q <= n; ++q) f *= q;
    std::vector<double> r(n);
    for (int k = 0; k < n; ++k) r[k] = (double)eulerian2(n, k) / f;
    return r;
}

struct Prof2 {
    bool on = false;
    std::map<std::string, std::pair<double, int64_t>> acc;
    std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> pending;
};

constexpr int RED_BLOCKS = 1024;

}  // namespace

struct ecpic2d_ctx {
    ecpic2d_config cfg{};
    int P = 3, M1 = 0, M2 = 0, Nc = 0, TW = 16, kmax = 50, device = 0;
    int64_t N = 0;
    double dx1 = 0, dx2 = 0, w = 0, tol = 0;
    hipStream_t stream = nullptr;
    int cur = 0;
    double *xi1[2] = {}, *xi2[2] = {}, *p1[2] = {}, *p2[2] = {};
    int32_t *id[2] = {};
    double *d1[2] = {}, *d2[2] = {}, *pk1 = nullptr, *pk2 = nullptr;
    double *azn = nullptr, *gamn = nullptr;   // A_z(x^n), gamma^n during Subsystem I (sweep order)
    int32_t *cell = nullptr /* new cell (set_particles) or packed new tile and column (commit) */, *count = nullptr,
            *start = nullptr, *bsum = nullptr;
    int32_t *mig = nullptr;   // arrivals per new tile, after the stayers' slots
    int32_t *tstart[2] = {}, *tstay = nullptr, *tarr = nullptr, *tcnt = nullptr, *tcur = nullptr;
    int ts = 0, ntiles = 0;   // tstart[ts]: first particle of each tile
    double *e1 = nullptr, *e2 = nullptr, *bz = nullptr, *ez = nullptr, *az = nullptr;
    double *en1 = nullptr, *en2 = nullptr, *ek1 = nullptr, *ek2 = nullptr, *eb1 = nullptr, *eb2 = nullptr;
    double *J1 = nullptr, *J2 = nullptr, *g1a = nullptr, *g2a = nullptr, *ezn = nullptr, *ezk = nullptr,
           *S = nullptr, *tmp = nullptr;
    double2 *Z = nullptr, *R = nullptr, *tw1 = nullptr, *tw2 = nullptr;
    double *sym = nullptr;        // m0a m1a cra cia (M1 each) m0b m1b crb cib (M2 each)
    double *partial = nullptr;    // RED_BLOCKS + 8
    unsigned long long *res = nullptr;   // 3 * MAXK + 4 slots
    int *flags = nullptr;
    int *gate = nullptr;                 // set once an iteration has converged (or failed)
    int spin = 0;                        // particles carry spins (hbar terms on)
    double hbar = 0.0;
    double *sx[2] = {}, *sy[2] = {}, *sz[2] = {};   // spins, in the particle buffers' order
    double *Dx = nullptr, *Dy = nullptr, *Dz = nullptr, *ssrc = nullptr;   // spin deposits and G*^T source
    double *hres = nullptr, *hres_dev = nullptr;   // pinned mirror: 3 values per iteration (I, then III)
    hipEvent_t ev[2] = {};
    bool have_particles = false;
    std::vector<double> m0row, m1row;
    Prof2 prof;
    std::vector<void *> allocs;
};

namespace {

template <typename T>
int dalloc(ecpic2d_ctx *c, T **p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc((void **)p, n * sizeof(T)) != hipSuccess) { *p = nullptr; return ECPIC_ENOMEM; }
    c->allocs.push_back((void *)*p);
    return ECPIC_OK;
}

int sync2(ecpic2d_ctx *c) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return ECPIC_EDEVICE;
    if (c->prof.on) {
        for (auto &pe : c->prof.pending) {
            float ms = 0.f;
            hipEventElapsedTime(&ms, pe.second.first, pe.second.second);
            auto &a = c->prof.acc[pe.first];
            a.first += ms;
            a.second += 1;
            hipEventDestroy(pe.second.first);
            hipEventDestroy(pe.second.second);
        }
        c->prof.pending.clear();
    }
    return hipGetLastError() == hipSuccess ? ECPIC_OK : ECPIC_EDEVICE;
}

// Launch with HIP events around it when profiling.
template <class F>
void timed(ecpic2d_ctx *c, const char *name, F launch) {
    if (!c->prof.on) { launch(); return; }
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    hipEventRecord(a, c->stream);
    launch();
    hipEventRecord(b, c->stream);
    c->prof.pending.push_back({name, {a, b}});
}

int grid_for(int64_t n) {
    int64_t g = (n + BLOCK - 1) / BLOCK;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

Sym sym_of(ecpic2d_ctx *c) {
    const double *s = c->sym;
    const int M1 = c->M1, M2 = c->M2;
    return Sym{s, s + M1, s + 2 * M1, s + 3 * M1, s + 4 * M1, s + 4 * M1 + M2, s + 4 * M1 + 2 * M2,
               s + 4 * M1 + 3 * M2};
}

int n_tiles(ecpic2d_ctx *c) { return c->M1 * (c->M2 / c->TW); }

// Full cell sort (set_particles): counts in c->count, cells in c->cell; each tile
// is stored transposed (tile_pos), and the tile starts are taken from the cell starts.
void sort_particles(ecpic2d_ctx *c) {
    const int A = c->cur, B = 1 - c->cur;
    timed(c, "sort", [&] {
        const int nb = (c->Nc + SCAN_TILE - 1) / SCAN_TILE;
        k2_scan_sums<<<nb, SCAN_THREADS, 0, c->stream>>>(c->count, c->bsum, c->Nc);
        k2_scan_top<<<1, SCAN_THREADS, 0, c->stream>>>(c->bsum, nb, c->start + c->Nc);
        k2_scan_apply<<<nb, SCAN_THREADS, 0, c->stream>>>(c->count, c->start, c->bsum, c->Nc);
        k2_scatter<<<grid_for(c->N), BLOCK, 0, c->stream>>>(c->xi1[A], c->xi2[A], c->p1[A], c->p2[A], c->id[A],
                                                           c->xi1[B], c->xi2[B], c->p1[B], c->p2[B], c->id[B],
                                                           c->cell, c->start, c->count, c->N, c->M2, c->TW);
        k2_fill_i32<<<grid_for(c->Nc), BLOCK, 0, c->stream>>>(c->count, c->Nc);
        k2_tiles_from_cells<<<grid_for(c->ntiles + 1), BLOCK, 0, c->stream>>>(
            c->start, c->tstart[c->ts], c->ntiles, c->M2 / c->TW, c->M2, c->TW, c->Nc);
    });
    c->cur = B;
}

// Re-sort after the first half of a Subsystem I commit (packed new tile and
// column in c->cell, stay and arrival counts per tile; increment in buffer di):
// new tile starts, the arrival lists, then each new tile formed and sorted by
// cell into the transposed layout in the other particle buffer.
void sort_tiles(ecpic2d_ctx *c, int di) {
    const int A = c->cur, B = 1 - c->cur, T0 = c->ts, T1 = 1 - c->ts;
    timed(c, "sort", [&] {
        const int nt = c->ntiles, nb = (nt + SCAN_TILE - 1) / SCAN_TILE;
        k2_tile_counts<<<grid_for(nt), BLOCK, 0, c->stream>>>(c->tstay, c->tarr, c->tcnt, c->tcur, nt);
        k2_scan_sums<<<nb, SCAN_THREADS, 0, c->stream>>>(c->tcnt, c->bsum, nt);
        k2_scan_top<<<1, SCAN_THREADS, 0, c->stream>>>(c->bsum, nb, c->tstart[T1] + nt);
        k2_scan_apply<<<nb, SCAN_THREADS, 0, c->stream>>>(c->tcnt, c->tstart[T1], c->bsum, nt);
        k2_list_arrivals<<<nt, BLOCK, 0, c->stream>>>(c->cell, c->tstart[T0], c->tstart[T1], c->tstay, c->tcur,
                                                     c->mig);
        const Resort r{c->xi1[A], c->xi2[A], c->d1[di], c->d2[di], c->pk1, c->pk2, c->id[A], c->cell, c->mig,
                       c->tstart[T0], c->tstart[T1], c->tstay, c->xi1[B], c->xi2[B], c->p1[B], c->p2[B], c->id[B],
                       c->M1, c->M2, 1.0 / c->dx1, 1.0 / c->dx2, {c->sx[A], c->sy[A], c->sz[A]},
                       {c->sx[B], c->sy[B], c->sz[B]}};
        k2_tile_resort<<<nt, SORT_THREADS, 0, c->stream>>>(r);
    });
    c->cur = B;
    c->ts = T1;
}

// Forward rows -> columns with op -> inverse rows with epi, over NB grids.
template <int NB, class Op, class Epi>
void spectral(ecpic2d_ctx *c, const char *name, Ptrs<NB> src, int zero_mask, Op op, Epi epi,
              const int *gate = nullptr) {
    timed(c, name, [&] {
        // transforms per block: BLOCK / (n / 8) for n points
        const int rows = NB * c->M1, per_row = BLOCK / (c->M2 / 8), per_col = BLOCK / (c->M1 / 8);
        const int grow = (rows + per_row - 1) / per_row, gcol = (c->M2 + per_col - 1) / per_col;
        k2_fft_rows_fwd<NB><<<grow, BLOCK, 0, c->stream>>>(src, zero_mask, c->Z, c->M1, c->M2, c->tw2, gate);
        k2_fft_cols<NB, Op><<<gcol, BLOCK, 0, c->stream>>>(c->Z, c->M1, c->M2, c->tw1, op, gate);
        if (Op::INVERSE)
            k2_fft_rows_inv<NB, Epi><<<grow, BLOCK, 0, c->stream>>>(c->Z, c->M1, c->M2, c->tw2, 1.0 / (double)c->Nc,
                                                                  epi, gate);
    });
}

// Host view of one iteration's mirror (residuals h[0], h[1], flags h[2]).
int status_of(const double *h) {
    const int f = (int)h[2];
    if (f & FLAG_NONFINITE) return ECPIC_ENONFINITE;
    if (f & FLAG_CFL) return ECPIC_ECFL;
    if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return ECPIC_ENONFINITE;
    return ECPIC_OK;
}

int flags_status(ecpic2d_ctx *c) {
    int f = 0;
    if (hipMemcpyAsync(&f, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess) return ECPIC_EDEVICE;
    int rc = sync2(c);
    if (rc) return rc;
    if (f & FLAG_NONFINITE) return ECPIC_ENONFINITE;
    if (f & FLAG_CFL) return ECPIC_ECFL;
    return ECPIC_OK;
}

double read_res(ecpic2d_ctx *c, int slot, int *rc) {
    unsigned long long b = 0;
    if (hipMemcpyAsync(&b, c->res + slot, sizeof(b), hipMemcpyDeviceToHost, c->stream) != hipSuccess) {
        *rc = ECPIC_EDEVICE;
        return 0.0;
    }
    *rc = sync2(c);
    double v;
    std::memcpy(&v, &b, sizeof(v));
    return v;
}

#define LAUNCH_P(P, ...)                                      \
    switch (P) {                                              \
        case 2: { constexpr int PP = 2; __VA_ARGS__; } break; \
        case 3: { constexpr int PP = 3; __VA_ARGS__; } break; \
        case 4: { constexpr int PP = 4; __VA_ARGS__; } break; \
        case 5: { constexpr int PP = 5; __VA_ARGS__; } break; \
    }

int substep_I(ecpic2d_ctx *c, double dt, ecpic2d_iter_stats *st) {
    const int A = c->cur, Nc = c->Nc, gC = grid_for(Nc);
    hipStream_t s = c->stream;
    k2_fill_u64<<<1, 2 * MAXK, 0, s>>>(c->res, 2 * MAXK);
    k2_fill_i32<<<1, 1, 0, s>>>(c->flags, 1);
    k2_grad<<<gC, BLOCK, 0, s>>>(c->az, c->g1a, c->g2a, c->M1, c->M2, 1.0 / c->dx1, 1.0 / c->dx2);
    k2_copy<<<gC, BLOCK, 0, s>>>(c->en1, c->e1, Nc);
    k2_copy<<<gC, BLOCK, 0, s>>>(c->en2, c->e2, Nc);
    k2_copy<<<gC, BLOCK, 0, s>>>(c->ek1, c->e1, Nc);
    k2_copy<<<gC, BLOCK, 0, s>>>(c->ek2, c->e2, Nc);
    k2_copy<<<gC, BLOCK, 0, s>>>(c->eb1, c->e1, Nc);
    k2_copy<<<gC, BLOCK, 0, s>>>(c->eb2, c->e2, Nc);
    k2_fill<<<gC, BLOCK, 0, s>>>(c->J1, Nc, 0.0);
    k2_fill<<<gC, BLOCK, 0, s>>>(c->J2, Nc, 0.0);
    k2_fill_i32<<<1, 1, 0, s>>>(c->gate, 1);
    const Sym sy = sym_of(c);
    // Sweep k reads d^(k) from buffer k & 1 and writes d^(k+1) to the other;
    // then the field update, the check, and event ev[k & 1].
    auto iterate = [&](int k) {
        const int di = k & 1;
        SweepArgs a{c->xi1[A], c->xi2[A], c->p1[A], c->p2[A], c->d1[di], c->d2[di], c->d1[1 - di], c->d2[1 - di],
                    c->pk1, c->pk2, c->tstart[c->ts], c->eb1, c->eb2, c->az, c->g1a, c->g2a, c->J1, c->J2,
                    c->res + k, c->flags, c->gate, c->M1, c->M2, c->TW, 1.0 / c->dx1, 1.0 / c->dx2, dt, c->w,
                    c->sx[A], c->sy[A], c->sz[A], c->bz, c->hbar, c->azn, c->gamn};
        timed(c, "sweep_I", [&] {
            if (c->spin) {
                if (k == 0) {
                    LAUNCH_P(c->P, k2_sweep_I<PP, true, true><<<n_tiles(c), BLOCK, 0, s>>>(a));
                } else {
                    LAUNCH_P(c->P, k2_sweep_I<PP, false, true><<<n_tiles(c), BLOCK, 0, s>>>(a));
                }
            } else if (k == 0) {
                LAUNCH_P(c->P, k2_sweep_I<PP, true, false><<<n_tiles(c), BLOCK, 0, s>>>(a));
            } else {
                LAUNCH_P(c->P, k2_sweep_I<PP, false, false><<<n_tiles(c), BLOCK, 0, s>>>(a));
            }
        });
        spectral<2>(c, "solve_I", Ptrs<2>{{c->J1, c->J2}}, 3, OpM1inv{sy},
                    EpiI{c->en1, c->en2, c->ek1, c->ek2, c->eb1, c->eb2, c->res + MAXK + k}, c->gate);
        k2_check<<<1, 1, 0, s>>>(c->res + k, c->res + MAXK + k, c->flags, c->tol, c->gate, c->hres_dev + 3 * k);
        hipEventRecord(c->ev[k & 1], s);
    };
    // Iteration k + 1 is queued before iteration k is read back, so the GPU
    // does not wait for the host; it does nothing if iteration k closed the gate.
    // With kernel timing on, iterations are queued one at a time (every timed
    // launch does its work).
    const bool ahead = !c->prof.on;
    double r = 0.0;
    int k, rc = ECPIC_OK;
    iterate(0);
    for (k = 0; k < c->kmax; ++k) {
        if (ahead && k + 1 < c->kmax) iterate(k + 1);
        if (hipEventSynchronize(c->ev[k & 1]) != hipSuccess) return ECPIC_EDEVICE;
        const double *h = c->hres + 3 * k;
        rc = status_of(h);
        if (rc) break;
        r = std::max(h[0], h[1]);
        if (r <= c->tol) break;
        if (!ahead && k + 1 < c->kmax) iterate(k + 1);
    }
    if (rc) {
        sync2(c);
        return rc;
    }
    const int di = k & 1;
    if (st) { st->sweeps = std::min(k + 1, c->kmax); st->residual = r; st->reserved = 0; }
    if (k == c->kmax) return ECPIC_ENOTCONV;
    // commit x^n + d^(k) (buffer di), p^(k+1), e^(k+1): new tiles and counts, the
    // fields, then the re-sort writes the particles in their new order
    timed(c, "commit_I", [&] {
        k2_commit_tiles<<<c->ntiles, BLOCK, 0, s>>>(c->xi1[A], c->xi2[A], c->d1[di], c->d2[di], c->cell,
                                                    c->tstart[c->ts], c->tstay, c->tarr, c->M1, c->M2, c->TW,
                                                    1.0 / c->dx1, 1.0 / c->dx2);
    });
    k2_copy<<<gC, BLOCK, 0, s>>>(c->e1, c->ek1, Nc);
    k2_copy<<<gC, BLOCK, 0, s>>>(c->e2, c->ek2, Nc);
    sort_tiles(c, di);
    return sync2(c);
}

int substep_II(ecpic2d_ctx *c, double dt) {
    const int A = c->cur;
    if (c->spin)
        k2_grad<<<grid_for(c->Nc), BLOCK, 0, c->stream>>>(c->az, c->g1a, c->g2a, c->M1, c->M2, 1.0 / c->dx1,
                                                          1.0 / c->dx2);
    const RotArgs a{c->xi1[A], c->xi2[A], c->p1[A], c->p2[A], c->sx[A], c->sy[A], c->sz[A], c->tstart[c->ts],
                    c->bz, c->az, c->g1a, c->g2a, c->M1, c->M2, c->TW, dt};
    timed(c, "rotate_II", [&] {
        if (c->spin) {
            LAUNCH_P(c->P, k2_rotate_tiles<PP, true><<<n_tiles(c), BLOCK, 0, c->stream>>>(a));
        } else {
            LAUNCH_P(c->P, k2_rotate_tiles<PP, false><<<n_tiles(c), BLOCK, 0, c->stream>>>(a));
        }
    });
    return ECPIC_OK;
}

int substep_III(ecpic2d_ctx *c, double dt, ecpic2d_iter_stats *st) {
    const int A = c->cur, Nc = c->Nc, gC = grid_for(Nc);
    hipStream_t s = c->stream;
    k2_fill_u64<<<1, MAXK, 0, s>>>(c->res + 2 * MAXK, MAXK);
    k2_copy<<<gC, BLOCK, 0, s>>>(c->ezn, c->ez, Nc);
    k2_copy<<<gC, BLOCK, 0, s>>>(c->ezk, c->ez, Nc);
    k2_fill<<<gC, BLOCK, 0, s>>>(c->S, Nc, 0.0);
    const Sym sy = sym_of(c);
    // constant part in Fourier space (with spin: plus dt hbar G*^T Lambda1*^T W S_xy)
    if (c->spin) {
        k2_fill<<<gC, BLOCK, 0, s>>>(c->Dx, Nc, 0.0);
        k2_fill<<<gC, BLOCK, 0, s>>>(c->Dy, Nc, 0.0);
        LAUNCH_P(c->P, k2_deposit_spin<PP><<<n_tiles(c), BLOCK, 0, s>>>(c->xi1[A], c->xi2[A], c->sx[A], c->sy[A],
                                                                         c->sz[A], c->tstart[c->ts], c->Dx, c->Dy,
                                                                         nullptr, c->M1, c->M2, c->TW, c->w, 0));
        k2_spin_src<<<gC, BLOCK, 0, s>>>(c->Dx, c->Dy, c->ssrc, c->M1, c->M2, 1.0 / c->dx1, 1.0 / c->dx2);
        spectral<3>(c, "solve_III", Ptrs<3>{{c->ezn, c->az, c->ssrc}}, 0, OpIIIrhsS{sy, c->R, c->M2, dt, c->hbar},
                    EpiStore<3>{Ptrs<3>{{nullptr, nullptr, nullptr}}, nullptr});
    } else {
        spectral<2>(c, "solve_III", Ptrs<2>{{c->ezn, c->az}}, 0, OpIIIrhs{sy, c->R, c->M2, dt},
                    EpiStore<2>{Ptrs<2>{{nullptr, nullptr}}, nullptr});
    }
    k2_fill_i32<<<1, 1, 0, s>>>(c->gate, 1);
    auto iterate = [&](int k) {   // as in Subsystem I: deposit, solve, check, event ev[k & 1]
        DepArgs a{c->xi1[A], c->xi2[A], c->p1[A], c->p2[A], c->tstart[c->ts], c->az, c->ezn, c->ezk, c->S,
                  c->pk1, c->M1, c->M2, c->TW, dt, c->w, 1, k == 0, c->gate};
        timed(c, "deposit_III", [&] { LAUNCH_P(c->P, k2_deposit0<PP><<<n_tiles(c), BLOCK, 0, s>>>(a)); });
        spectral<1>(c, "solve_III", Ptrs<1>{{c->S}}, 1, OpIII{sy, c->R, c->M2, dt},
                    EpiIII{c->ezk, c->res + 2 * MAXK + k}, c->gate);
        k2_check<<<1, 1, 0, s>>>(c->res + 2 * MAXK + k, nullptr, nullptr, c->tol, c->gate,
                                 c->hres_dev + 3 * (MAXK + k));
        hipEventRecord(c->ev[k & 1], s);
    };
    const bool ahead = !c->prof.on;
    double r = 0.0;
    int k, rc = ECPIC_OK;
    iterate(0);
    for (k = 0; k < c->kmax; ++k) {
        if (ahead && k + 1 < c->kmax) iterate(k + 1);
        if (hipEventSynchronize(c->ev[k & 1]) != hipSuccess) return ECPIC_EDEVICE;
        const double *h = c->hres + 3 * (MAXK + k);
        rc = status_of(h);
        if (rc) break;
        r = h[0];
        if (r <= c->tol) break;
        if (!ahead && k + 1 < c->kmax) iterate(k + 1);
    }
    if (rc) {
        sync2(c);
        return rc;
    }
    if (st) { st->sweeps = std::min(k + 1, c->kmax); st->residual = r; st->reserved = 0; }
    if (k == c->kmax) return ECPIC_ENOTCONV;
    k2_finish_III<<<gC, BLOCK, 0, s>>>(c->az, c->ez, c->ezn, c->ezk, Nc, dt);
    return ECPIC_OK;
}

int substep_IV(ecpic2d_ctx *c, double dt) {
    if (c->spin) {   // with the constant source hbar C^T Lambda2^T W S_z
        const int A = c->cur;
        k2_fill<<<grid_for(c->Nc), BLOCK, 0, c->stream>>>(c->Dz, c->Nc, 0.0);
        LAUNCH_P(c->P, k2_deposit_spin<PP><<<n_tiles(c), BLOCK, 0, c->stream>>>(
                           c->xi1[A], c->xi2[A], c->sx[A], c->sy[A], c->sz[A], c->tstart[c->ts], nullptr, nullptr,
                           c->Dz, c->M1, c->M2, c->TW, c->w, 1));
        spectral<4>(c, "maxwell_IV", Ptrs<4>{{c->e1, c->e2, c->bz, c->Dz}}, 0, OpIVs{sym_of(c), dt, c->hbar},
                    EpiStore<4>{Ptrs<4>{{c->e1, c->e2, c->bz, nullptr}}, nullptr});
        return ECPIC_OK;
    }
    spectral<3>(c, "maxwell_IV", Ptrs<3>{{c->e1, c->e2, c->bz}}, 0, OpIV{sym_of(c), dt},
                EpiStore<3>{Ptrs<3>{{c->e1, c->e2, c->bz}}, nullptr});
    return ECPIC_OK;
}

void deposit_rho(ecpic2d_ctx *c, double *rho) {
    const int A = c->cur;
    k2_fill<<<grid_for(c->Nc), BLOCK, 0, c->stream>>>(rho, c->Nc, 0.0);
    DepArgs a{c->xi1[A], c->xi2[A], c->p1[A], c->p2[A], c->tstart[c->ts], nullptr, nullptr, nullptr, rho,
              nullptr, c->M1, c->M2, c->TW, 0.0, c->w, 0, 0};
    LAUNCH_P(c->P, k2_deposit0<PP><<<n_tiles(c), BLOCK, 0, c->stream>>>(a));
}

MassRows rows_of(ecpic2d_ctx *c, int d1, int d2) {
    MassRows m{};
    const std::vector<double> &a = d1 == c->P ? c->m0row : c->m1row, &b = d2 == c->P ? c->m0row : c->m1row;
    for (size_t i = 0; i < a.size(); ++i) m.r1[i] = a[i];
    for (size_t i = 0; i < b.size(); ++i) m.r2[i] = b[i];
    m.d1 = d1;
    m.d2 = d2;
    m.scale = c->dx1 * c->dx2;
    return m;
}

// x^T Mass x for a grid (result left in partial[RED_BLOCKS + slot]).
void quad(ecpic2d_ctx *c, const double *x, int d1, int d2, int slot) {
    const int gC = std::min(grid_for(c->Nc), RED_BLOCKS);
    k2_mass<<<grid_for(c->Nc), BLOCK, 0, c->stream>>>(x, c->tmp, c->M1, c->M2, rows_of(c, d1, d2));
    k2_dot<<<gC, BLOCK, 0, c->stream>>>(x, c->tmp, c->Nc, c->partial);
    k2_sum<<<1, BLOCK, 0, c->stream>>>(c->partial, gC, c->partial + RED_BLOCKS + slot);
}

}  // namespace

extern "C" {

int ecpic2d_create(const ecpic2d_config *cfg, ecpic2d_ctx **out) {
    if (!cfg || !out) return ECPIC_EINVAL;
    *out = nullptr;
    const ecpic2d_config g = *cfg;
    auto pow2 = [](int m) { return m >= 8 && m <= MAXM && (m & (m - 1)) == 0; };
    const double dx1 = g.L1 / g.M1, dx2 = g.L2 / g.M2;
    if (!(g.L1 > 0) || !(g.L2 > 0) || !pow2(g.M1) || !pow2(g.M2) || g.degree < 2 || g.degree > 5 ||
        g.n_particles < 0 || g.n_particles > INT32_MAX || !(g.picard_tol > 0) || g.picard_max_iter < 0 ||
        g.picard_max_iter > MAXK || !(g.dt > 0) || !(g.dt < std::min(dx1, dx2)) || g.weight < 0 ||
        !std::isfinite(g.weight) || (g.spin != 0 && g.spin != 1) || !std::isfinite(g.hbar) ||
        (!g.spin && g.hbar != 0.0))
        return ECPIC_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || g.device < 0 || g.device >= ndev) return ECPIC_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g.device) != hipSuccess) return ECPIC_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return ECPIC_EDEVICE;
    if (hipSetDevice(g.device) != hipSuccess) return ECPIC_EDEVICE;
    ecpic2d_ctx *c = new ecpic2d_ctx();
    c->cfg = g;
    c->device = g.device;
    c->P = g.degree;
    c->M1 = g.M1;
    c->M2 = g.M2;
    c->Nc = g.M1 * g.M2;
    c->TW = std::min(TWMAX, g.M2);
    c->kmax = g.picard_max_iter ? g.picard_max_iter : 50;
    c->N = g.n_particles;
    c->dx1 = dx1;
    c->dx2 = dx2;
    c->w = g.weight > 0 ? g.weight : (c->N > 0 ? g.L1 * g.L2 / (double)c->N : 0.0);
    c->tol = g.picard_tol;
    c->spin = g.spin;
    c->hbar = g.hbar;
    c->m0row = mass_row2(c->P);
    c->m1row = mass_row2(c->P - 1);
    if (hipStreamCreate(&c->stream) != hipSuccess) { delete c; return ECPIC_EDEVICE; }
    const size_t N = (size_t)c->N, Nc = (size_t)c->Nc;
    int rc = 0;
    for (int b = 0; b < 2; ++b) {
        rc |= dalloc(c, &c->xi1[b], N) | dalloc(c, &c->xi2[b], N) | dalloc(c, &c->p1[b], N) |
              dalloc(c, &c->p2[b], N) | dalloc(c, &c->id[b], N) | dalloc(c, &c->d1[b], N) |
              dalloc(c, &c->d2[b], N);
    }
    rc |= dalloc(c, &c->pk1, N) | dalloc(c, &c->pk2, N) | dalloc(c, &c->azn, N) | dalloc(c, &c->gamn, N) |
          dalloc(c, &c->cell, N) | dalloc(c, &c->mig, N) |
          dalloc(c, &c->count, Nc) | dalloc(c, &c->start, Nc + 1) | dalloc(c, &c->bsum, Nc / SCAN_TILE + 2);
    c->ntiles = c->M1 * (c->M2 / c->TW);
    rc |= dalloc(c, &c->tstart[0], (size_t)c->ntiles + 1) | dalloc(c, &c->tstart[1], (size_t)c->ntiles + 1) |
          dalloc(c, &c->tstay, (size_t)c->ntiles) | dalloc(c, &c->tarr, (size_t)c->ntiles) |
          dalloc(c, &c->tcnt, (size_t)c->ntiles) | dalloc(c, &c->tcur, (size_t)c->ntiles);
    double **grids[] = {&c->e1, &c->e2, &c->bz, &c->ez, &c->az, &c->en1, &c->en2, &c->ek1, &c->ek2, &c->eb1,
                        &c->eb2, &c->J1, &c->J2, &c->g1a, &c->g2a, &c->ezn, &c->ezk, &c->S, &c->tmp};
    for (double **gp : grids) rc |= dalloc(c, gp, Nc);
    if (c->spin) {
        for (int b = 0; b < 2; ++b) rc |= dalloc(c, &c->sx[b], N) | dalloc(c, &c->sy[b], N) | dalloc(c, &c->sz[b], N);
        rc |= dalloc(c, &c->Dx, Nc) | dalloc(c, &c->Dy, Nc) | dalloc(c, &c->Dz, Nc) | dalloc(c, &c->ssrc, Nc);
    }
    rc |= dalloc(c, &c->Z, 4 * Nc) | dalloc(c, &c->R, Nc) | dalloc(c, &c->tw1, (size_t)c->M1 / 2) |
          dalloc(c, &c->tw2, (size_t)c->M2 / 2) | dalloc(c, &c->sym, 4 * (size_t)(c->M1 + c->M2)) |
          dalloc(c, &c->partial, RED_BLOCKS + 16) | dalloc(c, &c->res, 3 * MAXK + 4) | dalloc(c, &c->flags, 1) |
          dalloc(c, &c->gate, 1);
    if (rc || hipHostMalloc((void **)&c->hres, sizeof(double) * 6 * MAXK, hipHostMallocMapped) != hipSuccess) {
        ecpic2d_destroy(c);
        return ECPIC_ENOMEM;
    }
    if (hipHostGetDevicePointer((void **)&c->hres_dev, c->hres, 0) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev[1], hipEventDisableTiming) != hipSuccess) {
        ecpic2d_destroy(c);
        return ECPIC_EDEVICE;
    }
    // twiddles and 1D symbols (host, long double)
    const long double PI = 3.14159265358979323846264338327950288L;
    std::vector<double2> t1(c->M1 / 2), t2(c->M2 / 2);
    for (int j = 0; j < c->M1 / 2; ++j)
        t1[j] = make_double2((double)cosl(2 * PI * j / c->M1), (double)-sinl(2 * PI * j / c->M1));
    for (int j = 0; j < c->M2 / 2; ++j)
        t2[j] = make_double2((double)cosl(2 * PI * j / c->M2), (double)-sinl(2 * PI * j / c->M2));
    std::vector<double> sy(4 * (size_t)(c->M1 + c->M2));
    auto fill_dir = [&](int M, double dx, double *m0, double *m1, double *cr, double *ci) {
        const int p = c->P;
        for (int k = 0; k < M; ++k) {
            const long double th = 2 * PI * k / M;
            long double s0 = 0, s1 = 0;
            for (int q = -p; q <= p; ++q) s0 += (long double)c->m0row[q + p] * cosl(q * th);
            for (int q = -(p - 1); q <= p - 1; ++q) s1 += (long double)c->m1row[q + p - 1] * cosl(q * th);
            m0[k] = (double)(s0 * dx);
            m1[k] = (double)(s1 * dx);
            cr[k] = (double)((1 - cosl(th)) / dx);
            ci[k] = (double)(sinl(th) / dx);
        }
    };
    const int M1 = c->M1, M2 = c->M2;
    fill_dir(M1, dx1, &sy[0], &sy[M1], &sy[2 * M1], &sy[3 * M1]);
    fill_dir(M2, dx2, &sy[4 * M1], &sy[4 * M1 + M2], &sy[4 * M1 + 2 * M2], &sy[4 * M1 + 3 * M2]);
    bool ok = hipMemcpy(c->tw1, t1.data(), sizeof(double2) * t1.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->tw2, t2.data(), sizeof(double2) * t2.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->sym, sy.data(), sizeof(double) * sy.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) { ecpic2d_destroy(c); return ECPIC_EDEVICE; }
    for (double **gp : grids) k2_fill<<<grid_for(c->Nc), BLOCK, 0, c->stream>>>(*gp, c->Nc, 0.0);
    k2_fill_i32<<<grid_for(c->Nc), BLOCK, 0, c->stream>>>(c->count, c->Nc);
    // the commit accumulates arrivals per tile: every tile counter starts at zero
    for (int32_t *tp : {c->tstay, c->tarr, c->tcnt, c->tcur})
        k2_fill_i32<<<grid_for(c->ntiles), BLOCK, 0, c->stream>>>(tp, c->ntiles);
    k2_fill_i32<<<1, 1, 0, c->stream>>>(c->flags, 1);
    if (sync2(c)) { ecpic2d_destroy(c); return ECPIC_EDEVICE; }
    *out = c;
    return ECPIC_OK;
}

int ecpic2d_destroy(ecpic2d_ctx *c) {
    if (!c) return ECPIC_OK;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    for (auto &pe : c->prof.pending) { hipEventDestroy(pe.second.first); hipEventDestroy(pe.second.second); }
    for (void *p : c->allocs) hipFree(p);
    if (c->hres) hipHostFree(c->hres);
    for (hipEvent_t e : c->ev)
        if (e) hipEventDestroy(e);
    if (c->stream) hipStreamDestroy(c->stream);
    delete c;
    return ECPIC_OK;
}

int ecpic2d_set_particles(ecpic2d_ctx *c, const double *x1, const double *x2, const double *p1, const double *p2,
                          int64_t n) {
    if (!c || n != c->N || (n > 0 && (!x1 || !x2 || !p1 || !p2))) return ECPIC_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(x1[i]) || !std::isfinite(x2[i]) || !std::isfinite(p1[i]) || !std::isfinite(p2[i]))
            return ECPIC_EINVAL;
    hipSetDevice(c->device);
    const int B = 1 - c->cur, A = c->cur;
    const size_t bytes = sizeof(double) * (size_t)n;
    hipStream_t s = c->stream;
    // raw positions into the B buffers, momenta into A (scatter moves A -> B)
    if (n > 0) {
        if (hipMemcpyAsync(c->d1[0], x1, bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(c->d2[0], x2, bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(c->p1[A], p1, bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(c->p2[A], p2, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
            return ECPIC_EDEVICE;
    }
    (void)B;
    k2_fill_i32<<<1, 1, 0, s>>>(c->flags, 1);
    k2_fill_i32<<<grid_for(c->Nc), BLOCK, 0, s>>>(c->count, c->Nc);
    for (int32_t *tp : {c->tstay, c->tarr, c->tcnt, c->tcur})
        k2_fill_i32<<<grid_for(c->ntiles), BLOCK, 0, s>>>(tp, c->ntiles);
    k2_iota<<<grid_for(n), BLOCK, 0, s>>>(c->id[A], n);
    k2_bin_new<<<grid_for(n), BLOCK, 0, s>>>(c->d1[0], c->d2[0], c->xi1[A], c->xi2[A], c->cell, c->count, n,
                                             c->M1, c->M2, 1.0 / c->dx1, 1.0 / c->dx2, c->flags);
    sort_particles(c);
    if (c->spin)   // the spins start at zero; ecpic2d_set_spins gives them
        for (double *sp : {c->sx[c->cur], c->sy[c->cur], c->sz[c->cur]})
            k2_fill<<<grid_for(n), BLOCK, 0, s>>>(sp, n, 0.0);
    int rc = flags_status(c);
    if (rc) return rc == ECPIC_ENONFINITE ? ECPIC_EINVAL : rc;
    c->have_particles = true;
    return ECPIC_OK;
}

int ecpic2d_set_spins(ecpic2d_ctx *c, const double *sx, const double *sy, const double *sz, int64_t n) {
    if (!c || !c->spin || n != c->N || (n > 0 && (!sx || !sy || !sz))) return ECPIC_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(sx[i]) || !std::isfinite(sy[i]) || !std::isfinite(sz[i])) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    const int A = c->cur;
    const size_t bytes = sizeof(double) * (size_t)n;
    const double *in[3] = {sx, sy, sz};
    double *dst[3] = {c->sx[A], c->sy[A], c->sz[A]};
    for (int q = 0; q < 3 && n > 0; ++q) {
        // staging buffer: pk1 (free between substeps), in the caller's order
        if (hipMemcpyAsync(c->pk1, in[q], bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return ECPIC_EDEVICE;
        k2_gather_id<<<grid_for(n), BLOCK, 0, c->stream>>>(c->pk1, c->id[A], dst[q], n);
    }
    return sync2(c);
}

int ecpic2d_get_spins(ecpic2d_ctx *c, double *sx, double *sy, double *sz, int64_t n) {
    if (!c || !c->spin || n != c->N || (n > 0 && (!sx || !sy || !sz))) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    const int A = c->cur;
    const size_t bytes = sizeof(double) * (size_t)n;
    double *outs[3] = {sx, sy, sz};
    const double *srcs[3] = {c->sx[A], c->sy[A], c->sz[A]};
    for (int q = 0; q < 3 && n > 0; ++q) {
        k2_unsort<<<grid_for(n), BLOCK, 0, c->stream>>>(srcs[q], c->id[A], c->pk1, n, 1.0);
        if (hipMemcpyAsync(outs[q], c->pk1, bytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
            return ECPIC_EDEVICE;
        int rc = sync2(c);
        if (rc) return rc;
    }
    return sync2(c);
}

int ecpic2d_get_particles(ecpic2d_ctx *c, double *x1, double *x2, double *p1, double *p2, int64_t n) {
    if (!c || n != c->N || (n > 0 && (!x1 || !x2 || !p1 || !p2))) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    const int A = c->cur;
    const size_t bytes = sizeof(double) * (size_t)n;
    double *outs[4] = {x1, x2, p1, p2};
    const double *srcs[4] = {c->xi1[A], c->xi2[A], c->p1[A], c->p2[A]};
    const double scales[4] = {c->dx1, c->dx2, 1.0, 1.0};
    for (int q = 0; q < 4; ++q) {
        if (n == 0) break;
        k2_unsort<<<grid_for(n), BLOCK, 0, c->stream>>>(srcs[q], c->id[A], c->pk1, n, scales[q]);
        if (hipMemcpyAsync(outs[q], c->pk1, bytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
            return ECPIC_EDEVICE;
        int rc = sync2(c);
        if (rc) return rc;
    }
    return sync2(c);
}

int ecpic2d_set_fields(ecpic2d_ctx *c, const double *e1, const double *e2, const double *bz, const double *ez,
                       const double *az) {
    if (!c) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    const double *src[5] = {e1, e2, bz, ez, az};
    double *dst[5] = {c->e1, c->e2, c->bz, c->ez, c->az};
    for (int q = 0; q < 5; ++q) {
        if (src[q]) {
            if (hipMemcpyAsync(dst[q], src[q], sizeof(double) * c->Nc, hipMemcpyHostToDevice, c->stream) !=
                hipSuccess)
                return ECPIC_EDEVICE;
        } else {
            k2_fill<<<grid_for(c->Nc), BLOCK, 0, c->stream>>>(dst[q], c->Nc, 0.0);
        }
    }
    return sync2(c);
}

int ecpic2d_get_fields(ecpic2d_ctx *c, double *e1, double *e2, double *bz, double *ez, double *az) {
    if (!c) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    double *dst[5] = {e1, e2, bz, ez, az};
    const double *src[5] = {c->e1, c->e2, c->bz, c->ez, c->az};
    for (int q = 0; q < 5; ++q)
        if (dst[q] &&
            hipMemcpyAsync(dst[q], src[q], sizeof(double) * c->Nc, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
            return ECPIC_EDEVICE;
    return sync2(c);
}

int ecpic2d_solve_gauss(ecpic2d_ctx *c) {
    if (!c) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    deposit_rho(c, c->S);
    spectral<3>(c, "poisson", Ptrs<3>{{c->e1, c->e2, c->S}}, 4, OpPoisson{sym_of(c)},
                EpiStore<3>{Ptrs<3>{{c->e1, c->e2, c->S}}, nullptr});
    k2_fill<<<grid_for(c->Nc), BLOCK, 0, c->stream>>>(c->S, c->Nc, 0.0);
    return sync2(c);
}

int ecpic2d_substep_I(ecpic2d_ctx *c, double dt, ecpic2d_iter_stats *st) {
    if (!c || !(dt > 0) || !(dt < std::min(c->dx1, c->dx2))) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    return substep_I(c, dt, st);
}

int ecpic2d_substep_II(ecpic2d_ctx *c, double dt) {
    if (!c || !std::isfinite(dt)) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    substep_II(c, dt);
    return sync2(c);
}

int ecpic2d_substep_III(ecpic2d_ctx *c, double dt, ecpic2d_iter_stats *st) {
    if (!c || !(dt > 0) || !std::isfinite(dt)) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    int rc = substep_III(c, dt, st);
    if (rc) return rc;
    return sync2(c);
}

int ecpic2d_substep_IV(ecpic2d_ctx *c, double dt) {
    if (!c || !std::isfinite(dt)) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    substep_IV(c, dt);
    return sync2(c);
}

int ecpic2d_step(ecpic2d_ctx *c, int32_t nsteps, int32_t *sweeps_I, int32_t *iters_III) {
    if (!c || nsteps < 0) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    const double dt = c->cfg.dt;
    for (int s = 0; s < nsteps; ++s) {
        ecpic2d_iter_stats a{}, b{};
        int rc = substep_I(c, dt, &a);
        if (sweeps_I) sweeps_I[s] = a.sweeps;
        if (rc) return rc;
        substep_II(c, dt);
        rc = substep_III(c, dt, &b);
        if (iters_III) iters_III[s] = b.sweeps;
        if (rc) return rc;
        substep_IV(c, dt);
    }
    return sync2(c);
}

int ecpic2d_energy(ecpic2d_ctx *c, ecpic2d_energy_parts *out) {
    if (!c || !out) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    const int A = c->cur, P = c->P;
    hipStream_t s = c->stream;
    const int gN = std::min(grid_for(c->N), RED_BLOCKS);
    k2_fill<<<1, BLOCK, 0, s>>>(c->partial, RED_BLOCKS + 16, 0.0);
    LAUNCH_P(P, k2_kinetic<PP><<<gN, BLOCK, 0, s>>>(c->xi1[A], c->xi2[A], c->p1[A], c->p2[A], c->az, c->N, c->M1,
                                                     c->M2, c->w, c->partial));
    k2_sum<<<1, BLOCK, 0, s>>>(c->partial, gN, c->partial + RED_BLOCKS + 0);
    quad(c, c->e1, P - 1, P, 1);
    quad(c, c->e2, P, P - 1, 2);
    quad(c, c->bz, P - 1, P - 1, 3);
    quad(c, c->ez, P, P, 4);
    k2_grad<<<grid_for(c->Nc), BLOCK, 0, s>>>(c->az, c->g1a, c->g2a, c->M1, c->M2, 1.0 / c->dx1, 1.0 / c->dx2);
    quad(c, c->g1a, P - 1, P, 5);
    quad(c, c->g2a, P, P - 1, 6);
    if (c->spin) {
        k2_fill<<<1, BLOCK, 0, s>>>(c->partial, RED_BLOCKS, 0.0);
        LAUNCH_P(P, k2_zeeman<PP><<<gN, BLOCK, 0, s>>>(c->xi1[A], c->xi2[A], c->sx[A], c->sy[A], c->sz[A], c->g1a,
                                                        c->g2a, c->bz, c->N, c->M1, c->M2, c->w, c->partial));
        k2_sum<<<1, BLOCK, 0, s>>>(c->partial, gN, c->partial + RED_BLOCKS + 7);
    }
    double v[8];
    if (hipMemcpyAsync(v, c->partial + RED_BLOCKS, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess)
        return ECPIC_EDEVICE;
    int rc = sync2(c);
    if (rc) return rc;
    out->kinetic = v[0];
    out->e_xy = 0.5 * (v[1] + v[2]);
    out->b_z = 0.5 * v[3];
    out->e_z = 0.5 * v[4];
    out->a_z = 0.5 * (v[5] + v[6]);
    out->zeeman = c->spin ? c->hbar * v[7] : 0.0;
    out->total = out->kinetic + out->e_xy + out->b_z + out->e_z + out->a_z + out->zeeman;
    return ECPIC_OK;
}

int ecpic2d_deposit_charge(ecpic2d_ctx *c, double *rho) {
    if (!c || !rho) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    deposit_rho(c, c->S);
    if (hipMemcpyAsync(rho, c->S, sizeof(double) * c->Nc, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return ECPIC_EDEVICE;
    int rc = sync2(c);
    k2_fill<<<grid_for(c->Nc), BLOCK, 0, c->stream>>>(c->S, c->Nc, 0.0);
    return rc ? rc : sync2(c);
}

int ecpic2d_gauss_residual(ecpic2d_ctx *c, double *linf, double *vec) {
    if (!c || !linf) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    hipStream_t s = c->stream;
    const int P = c->P;
    deposit_rho(c, c->S);
    k2_mass<<<grid_for(c->Nc), BLOCK, 0, s>>>(c->e1, c->J1, c->M1, c->M2, rows_of(c, P - 1, P));
    k2_mass<<<grid_for(c->Nc), BLOCK, 0, s>>>(c->e2, c->J2, c->M1, c->M2, rows_of(c, P, P - 1));
    k2_fill_u64<<<1, 1, 0, s>>>(c->res + 3 * MAXK, 1);
    k2_gauss<<<std::min(grid_for(c->Nc), RED_BLOCKS), BLOCK, 0, s>>>(c->J1, c->J2, c->S, c->tmp, c->M1, c->M2,
                                                                     1.0 / c->dx1, 1.0 / c->dx2, c->dx1 * c->dx2,
                                                                     c->res + 3 * MAXK);
    int rc = 0;
    *linf = read_res(c, 3 * MAXK, &rc);
    if (!rc && vec &&
        hipMemcpyAsync(vec, c->tmp, sizeof(double) * c->Nc, hipMemcpyDeviceToHost, s) != hipSuccess)
        rc = ECPIC_EDEVICE;
    k2_fill<<<grid_for(c->Nc), BLOCK, 0, s>>>(c->S, c->Nc, 0.0);
    k2_fill<<<grid_for(c->Nc), BLOCK, 0, s>>>(c->J1, c->Nc, 0.0);
    k2_fill<<<grid_for(c->Nc), BLOCK, 0, s>>>(c->J2, c->Nc, 0.0);
    int rc2 = sync2(c);
    return rc ? rc : rc2;
}

int ecpic2d_profile_enable(ecpic2d_ctx *c, int32_t enable) {
    if (!c) return ECPIC_EINVAL;
    sync2(c);
    c->prof.on = enable != 0;
    if (c->prof.on) c->prof.acc.clear();
    return ECPIC_OK;
}

int ecpic2d_kernel_time(ecpic2d_ctx *c, const char *name, double *ms, int64_t *launches) {
    if (!c || !name || !ms || !launches) return ECPIC_EINVAL;
    sync2(c);
    auto it = c->prof.acc.find(name);
    *ms = it == c->prof.acc.end() ? 0.0 : it->second.first;
    *launches = it == c->prof.acc.end() ? 0 : it->second.second;
    return ECPIC_OK;
}

}  // extern "C"
