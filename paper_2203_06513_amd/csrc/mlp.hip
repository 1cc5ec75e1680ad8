// Learned warm start of Subsystem I (the initial Picard iterate, Section 4.2):
// a multilayer perceptron D -> 64 -> 64 -> 2 with the tanh form of GELU
// (Hendrycks and Gimpel, 2016).  Its input is a particle's local state
//   [t - 1/2, p, gamma0 - 1, a_y[c-P..c+P+1], a_z[c-P..c+P+1], e_x[c-P..c+P+1]]
// and its outputs the normalised targets
//   [(delta - dt p/gamma0)/dt^2, (p^{n+1} - p)/dt]
// of the converged step.  Training runs here in FP32 (forward, backward by the
// chain rule, Adam); inference runs per cell: all window features are constant
// on a cell and gamma0 is a function of (t, p) there, so the network is a
// function of (t, p) per cell.  It is evaluated with BF16 matrix cores on a
// WS_NT x WS_NP grid of nodes per cell, and each particle interpolates its
// cell's table (see the predictor pass in sub1.hip).
#include "sweep.hpp"

namespace ecpic {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int H = WS_H;

template <int D>
struct Lay {   // offsets in the flat parameter vector
    static constexpr int W1 = 0, B1 = H * D, W2 = B1 + H, B2 = W2 + H * H, W3 = B2 + H, B3 = W3 + 2 * H;
    static constexpr int N = B3 + 2;
};

__device__ __forceinline__ unsigned short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
    return (unsigned short)(u >> 16);
}

constexpr float GC = 0.7978845608028654f;   // sqrt(2/pi)
constexpr float GA = 0.044715f;

__device__ __forceinline__ float gelu_t(float z) { return 0.5f * z * (1.0f + tanhf(GC * (z + GA * z * z * z))); }

// The same function written as z sigma(2u) = z / (1 + exp(-2u)), u = sqrt(2/pi)(z + 0.044715 z^3),
// with the hardware exponential and reciprocal (inference tables).
__device__ __forceinline__ float gelu_fast(float z) {
    const float u2 = 2.0f * GC * fmaf(GA * z, z * z, z);
    return z * __builtin_amdgcn_rcpf(1.0f + __expf(-u2));
}

__device__ __forceinline__ float gelu_g(float z) {
    const float t = tanhf(GC * (z + GA * z * z * z));
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * GC * (1.0f + 3.0f * GA * z * z);
}

// splitmix64 (Steele, Lea and Flood, 2014): a counter-based generator.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace

// Glorot-uniform weights, zero biases.
template <int D>
__global__ void __launch_bounds__(256) k_ws_init(float *theta, uint64_t seed) {
    using L = Lay<D>;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= L::N) return;
    int fin = 0, fout = 0;
    if (q < L::B1) { fin = D; fout = H; }
    else if (q >= L::W2 && q < L::B2) { fin = H; fout = H; }
    else if (q >= L::W3 && q < L::B3) { fin = H; fout = 2; }
    if (!fin) { theta[q] = 0.0f; return; }
    const double u = (double)(mix64(seed ^ mix64((uint64_t)q)) >> 11) * (1.0 / 9007199254740992.0);
    theta[q] = (float)((2.0 * u - 1.0) * sqrt(6.0 / (fin + fout)));
}

// Mean and standard deviation of every feature (blocks 0..D-1) and target
// (blocks D, D+1) over the n records; block 1 (the momentum) also sets the
// momentum range of the table nodes, mean +- 4 standard deviations.
__global__ void __launch_bounds__(256) k_ws_stats(const float *feat, const float *targ, int64_t n, int D, float *mu,
                                                  float *sd, float *prange) {
    __shared__ double ls[MAX_WAVES], lq[MAX_WAVES];
    const int j = blockIdx.x;
    double s = 0.0, q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = j < D ? feat[i * D + j] : targ[i * 2 + (j - D)];
        s += v;
        q += v * v;
    }
    s = wave_sum(s);
    q = wave_sum(q);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    if (lane == 0) { ls[wid] = s; lq[wid] = q; }
    __syncthreads();
    if (threadIdx.x == 0) {
        s = 0.0; q = 0.0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) { s += ls[w]; q += lq[w]; }
        const double m = n > 0 ? s / n : 0.0;
        const double var = n > 0 ? fmax(q / n - m * m, 0.0) : 0.0;
        double d = sqrt(var);
        if (!(d > 1e-12 * fmax(1.0, fabs(m)))) d = 1.0;   // constant column
        mu[j] = (float)m;
        sd[j] = (float)d;
        if (j == 1) { prange[0] = (float)(m - 4.0 * d); prange[1] = (float)(m + 4.0 * d); }
    }
}

// Forward and backward pass of 32 samples per block (threads 0..31 one sample
// each), then the block's partial gradient of the mean squared error over the
// batch (all 64 threads, every parameter, samples in a fixed order).  The
// samples are drawn with a counter-based generator (step, position) or, with
// direct != 0, taken in order (samples past n count zero).
template <int D>
__global__ void __launch_bounds__(64) k_ws_fwd_bwd(const float *theta, const float *mu, const float *sd,
                                                   const float *feat, const float *targ, int64_t n, int direct,
                                                   uint64_t seed, int64_t step, int B, float *pgrad, float *ploss) {
    using L = Lay<D>;
    constexpr int S = 32, HP = H + 1;
    __shared__ float Xs[S * D];
    __shared__ float H1[S * HP], H2[S * HP], D1[S * HP], D2[S * HP];
    __shared__ float DY[S * 2], LS[S];
    const int tid = threadIdx.x;
    const int j = blockIdx.x * S + tid;
    if (tid < S) {
        const bool valid = direct ? j < n : j < B;
        int64_t idx = 0;
        if (valid) idx = direct ? j : (int64_t)(mix64(seed ^ mix64((uint64_t)step * (uint64_t)B + (uint64_t)j)) % (uint64_t)n);
        for (int i = 0; i < D; ++i) Xs[tid * D + i] = valid ? (feat[idx * D + i] - mu[i]) / sd[i] : 0.0f;
        const float t0 = valid ? (targ[idx * 2] - mu[D]) / sd[D] : 0.0f;
        const float t1 = valid ? (targ[idx * 2 + 1] - mu[D + 1]) / sd[D + 1] : 0.0f;
        for (int h = 0; h < H; ++h) {
            float z = theta[L::B1 + h];
            for (int i = 0; i < D; ++i) z = fmaf(theta[L::W1 + h * D + i], Xs[tid * D + i], z);
            H1[tid * HP + h] = gelu_t(z);
            D1[tid * HP + h] = gelu_g(z);
        }
        for (int h = 0; h < H; ++h) {
            float z = theta[L::B2 + h];
            for (int i = 0; i < H; ++i) z = fmaf(theta[L::W2 + h * H + i], H1[tid * HP + i], z);
            H2[tid * HP + h] = gelu_t(z);
            D2[tid * HP + h] = gelu_g(z);
        }
        float y0 = theta[L::B3], y1 = theta[L::B3 + 1];
        for (int i = 0; i < H; ++i) {
            y0 = fmaf(theta[L::W3 + i], H2[tid * HP + i], y0);
            y1 = fmaf(theta[L::W3 + H + i], H2[tid * HP + i], y1);
        }
        const float e0 = valid ? y0 - t0 : 0.0f, e1 = valid ? y1 - t1 : 0.0f;
        LS[tid] = e0 * e0 + e1 * e1;
        const float sc = 2.0f / (2.0f * (float)(direct ? n : B));   // d mean / d y
        const float dy0 = sc * e0, dy1 = sc * e1;
        DY[tid * 2] = dy0;
        DY[tid * 2 + 1] = dy1;
        for (int h = 0; h < H; ++h) D2[tid * HP + h] *= theta[L::W3 + h] * dy0 + theta[L::W3 + H + h] * dy1;
        for (int i = 0; i < H; ++i) {
            float g = 0.0f;
            for (int h = 0; h < H; ++h) g = fmaf(theta[L::W2 + h * H + i], D2[tid * HP + h], g);
            D1[tid * HP + i] *= g;
        }
    }
    __syncthreads();
    for (int q = tid; q < L::N; q += blockDim.x) {
        float g = 0.0f;
        if (q < L::B1) {
            const int h = q / D, i = q % D;
            for (int s = 0; s < S; ++s) g = fmaf(D1[s * HP + h], Xs[s * D + i], g);
        } else if (q < L::W2) {
            const int h = q - L::B1;
            for (int s = 0; s < S; ++s) g += D1[s * HP + h];
        } else if (q < L::B2) {
            const int h = (q - L::W2) / H, i = (q - L::W2) % H;
            for (int s = 0; s < S; ++s) g = fmaf(D2[s * HP + h], H1[s * HP + i], g);
        } else if (q < L::W3) {
            const int h = q - L::B2;
            for (int s = 0; s < S; ++s) g += D2[s * HP + h];
        } else if (q < L::B3) {
            const int o = (q - L::W3) / H, i = (q - L::W3) % H;
            for (int s = 0; s < S; ++s) g = fmaf(DY[s * 2 + o], H2[s * HP + i], g);
        } else {
            const int o = q - L::B3;
            for (int s = 0; s < S; ++s) g += DY[s * 2 + o];
        }
        pgrad[(size_t)blockIdx.x * L::N + q] = g;
    }
    if (tid == 0) {
        float l = 0.0f;
        for (int s = 0; s < S; ++s) l += LS[s];
        ploss[blockIdx.x] = l;
    }
}

// Sum of the block partials (fixed order), optional copy of the gradient, and
// one Adam step (Kingma and Ba, 2015) with bias correction at step t >= 1.
__global__ void __launch_bounds__(256) k_ws_adam(float *theta, float *m, float *v, const float *pgrad, int nblk, int np,
                                                 float lr, int t, int update, float *grad_out, const float *ploss,
                                                 float loss_scale, float *loss_out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < np) {
        float g = 0.0f;
        for (int b = 0; b < nblk; ++b) g += pgrad[(size_t)b * np + q];
        if (grad_out) grad_out[q] = g;
        if (update) {
            const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
            const float mq = b1 * m[q] + (1.0f - b1) * g;
            const float vq = b2 * v[q] + (1.0f - b2) * g * g;
            m[q] = mq;
            v[q] = vq;
            const float mh = mq / (1.0f - powf(b1, (float)t)), vh = vq / (1.0f - powf(b2, (float)t));
            theta[q] -= lr * mh / (sqrtf(vh) + eps);
        }
    }
    if (q == 0 && loss_out) {
        float l = 0.0f;
        for (int b = 0; b < nblk; ++b) l += ploss[b];
        *loss_out = l * loss_scale;
    }
}

// W2 in BF16 (row-major, rows padded to WS_H + 4) for the table kernel.
template <int D>
__global__ void __launch_bounds__(256) k_ws_w2_bf16(const float *theta, unsigned short *w2b) {
    using L = Lay<D>;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < H * H) w2b[(q / H) * (H + 4) + (q % H)] = to_bf16(theta[L::W2 + q]);
}

// The network's increment target (physical units) on the node grid of cell c,
// t_i = i / (WS_NT - 1), p_j = p_lo + j (p_hi - p_lo) / (WS_NP - 1), one node per
// lane (node l = i WS_NP + j).  Layer 1 splits into the cell's constant window
// part (once per cell) and the node part; layer 2, 64 x 64 x 64, runs on the
// matrix cores (v_mfma_f32_16x16x16_bf16: BF16 inputs, FP32 accumulation), and
// each lane folds its columns of GELU(Z2) into the output at once
// (y[m] = b3 + sum_n W3[0][n] GELU(Z2[m][n])); the 16 lanes of a row group sum
// their columns in a fixed order.  `nshare` waves (index `wshare`) split the
// hidden units of layer 1 and the column tiles of layer 2 between them and
// their partial outputs are summed in wave order.  Every thread of the block
// calls it (it holds block barriers).  W2b is the staged BF16 W2 (rows of
// WS_H + 4); h1, c1, xw and ys (nshare x 64) are the sharers' LDS scratch.
constexpr int WS_RS = WS_H + 4;

template <int P>
__device__ __forceinline__ float ws_cell_table(const WsNet &net, const unsigned short *W2b, unsigned short *h1,
                                               float *c1, float *xw, float *ys, int c, const double *coefA,
                                               const double *ay, const double *az, const double *ex, int M,
                                               int wshare, int nshare, int l) {
    constexpr int D = ws_d(P);
    using L = Lay<D>;
    const float *th = net.theta;
    if (wshare == 0) {
        for (int i = 3 + l; i < D; i += 64) {
            const int u = i - 3, f = u / (2 * (P + 1)), j = u % (2 * (P + 1)) - P;   // field f at cell c + j
            const double *src = f == 0 ? ay : (f == 1 ? az : ex);
            const double raw = src[imod(c + j, M) + HALO];
            xw[i] = ((float)raw - net.mu[i]) / net.sd[i];
        }
    }
    __syncthreads();
    if (wshare == 0) {
        float z = th[L::B1 + l];
        for (int i = 3; i < D; ++i) z = fmaf(th[L::W1 + l * D + i], xw[i], z);
        c1[l] = z;
    }
    const int it = l / WS_NP, ip = l % WS_NP;
    const double t = (double)it / (WS_NT - 1);
    const float plo = net.prange[0], phi = net.prange[1];
    const float p = plo + (phi - plo) * (float)ip / (float)(WS_NP - 1);
    const double *ra = coefA + (size_t)rec_index(c) * RecA<P>::N;
    double Ay = ra[P], Az = ra[2 * P + 1];
    for (int i = P - 1; i >= 0; --i) {
        Ay = fma(Ay, t, ra[i]);
        Az = fma(Az, t, ra[P + 1 + i]);
    }
    const double g0 = sqrt(1.0 + (double)p * p + Ay * Ay + Az * Az);
    const float x0 = ((float)(t - 0.5) - net.mu[0]) / net.sd[0];
    const float x1 = (p - net.mu[1]) / net.sd[1];
    const float x2 = ((float)(g0 - 1.0) - net.mu[2]) / net.sd[2];
    __syncthreads();
    {
        const int h0 = wshare * H / nshare, h1e = (wshare + 1) * H / nshare;
        for (int h = h0; h < h1e; ++h) {
            const float z = c1[h] + th[L::W1 + h * D] * x0 + th[L::W1 + h * D + 1] * x1 + th[L::W1 + h * D + 2] * x2;
            h1[l * WS_RS + h] = to_bf16(gelu_fast(z));
        }
    }
    __syncthreads();
    {
        const int r16 = l & 15, kq = (l >> 4) * 4;
        const int n0 = wshare * 4 / nshare, n1 = (wshare + 1) * 4 / nshare;
        float *yw = ys + wshare * 64;
        for (int mt = 0; mt < 4; ++mt) {
            float yp[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int nt = n0; nt < n1; ++nt) {
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const bf16x4 av = *reinterpret_cast<const bf16x4 *>(&h1[(mt * 16 + r16) * WS_RS + ks * 16 + kq]);
                    const bf16x4 bv = *reinterpret_cast<const bf16x4 *>(&W2b[(nt * 16 + r16) * WS_RS + ks * 16 + kq]);
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
                }
                const float bias = th[L::B2 + nt * 16 + r16], w3 = th[L::W3 + nt * 16 + r16];
#pragma unroll
                for (int i = 0; i < 4; ++i)   // acc[i] = Z2[mt*16 + kq + i][nt*16 + r16]
                    yp[i] = fmaf(w3, gelu_fast(acc[i] + bias), yp[i]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
#pragma unroll
                for (int off = 8; off >= 1; off >>= 1) yp[i] += __shfl_xor(yp[i], off, 16);
            }
            if (r16 == 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i) yw[mt * 16 + kq + i] = yp[i];
            }
        }
    }
    __syncthreads();
    float y = 0.0f;
    for (int w = 0; w < nshare; ++w) y += ys[w * 64 + l];
    return net.mu[D] + net.sd[D] * (th[L::B3] + y);
}

__device__ __forceinline__ void stage_w2b(const unsigned short *w2b, unsigned short *W2b) {
    const uint2 *src = reinterpret_cast<const uint2 *>(w2b);
    uint2 *dst = reinterpret_cast<uint2 *>(W2b);
    for (int q = threadIdx.x; q < H * WS_RS / 4; q += blockDim.x) dst[q] = src[q];
}

// Tables of all cells (four cells per block, one wave each), for inspection.
constexpr int WS_CELLS = 4;

template <int P>
__global__ void __launch_bounds__(64 * WS_CELLS) k_ws_table(WsNet net, const unsigned short *w2b,
                                                            const double *coefA, const double *ay, const double *az,
                                                            const double *ex, int M, float *table) {
    constexpr int D = ws_d(P);
    __shared__ __align__(16) unsigned short W2b[H * WS_RS];
    __shared__ __align__(16) unsigned short H1b[WS_CELLS][64 * WS_RS];
    __shared__ float ys[WS_CELLS][64], c1[WS_CELLS][H], xw[WS_CELLS][D];
    const int wv = threadIdx.x / 64, l = threadIdx.x & 63;
    const int c = blockIdx.x * WS_CELLS + wv;
    stage_w2b(w2b, W2b);
    const bool live = c < M;
    const float y = ws_cell_table<P>(net, W2b, H1b[wv], c1[wv], xw[wv], ys[wv], live ? c : M - 1, coefA, ay, az, ex,
                                     M, 0, 1, l);
    if (live) table[(size_t)c * (WS_NT * WS_NP) + l] = y;
}

// Predictor pass of the learned warm start, run as sweep 0: each particle's
// increment delta^(1) = dt p/gamma0 + dt^2 y, with y interpolated bilinearly in
// its cell's (t, p) table of network outputs (k_ws_table, same substep), and
// the current of that increment deposited like a sweep's, so that the field
// kernel after it makes e^(1) consistent with delta^(1).  The Picard sweeps
// start from both.  The increment is stored in the precision of the sweep that
// follows: single precision in the precision form (whose first FP64 sweep
// starts from the last single-precision one), else double.
constexpr int PRED_BATCH = 4;

template <int P>
__device__ __forceinline__ void ws_predict_item(const SweepIArgs &a, int item) {
    __shared__ float tab[WS_NT * WS_NP];
    DevStatus *st = a.st;
    // item count, status words and item description in one memory round trip
    const int n_items = *a.items.n_items;
    const int sgate = st->gate, sflags = st->flags, skconv = st->kconv;
    const int c = a.items.cell[item];
    const int beg = a.items.begin[item], end = a.items.begin[item + 1];
    asm volatile("" ::"s"(n_items), "s"(sgate), "s"(sflags), "s"(skconv), "s"(c), "s"(beg), "s"(end));
    if (item >= n_items) return;
    if (!sgate | sflags | (skconv >= 0)) return;
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
    int wb, we;
    wave_range(beg, end, wid, nw, wb, we);
    if (threadIdx.x < WS_NT * WS_NP) tab[threadIdx.x] = a.ws_table[(size_t)c * (WS_NT * WS_NP) + threadIdx.x];
    const double *ra = a.coefA + (size_t)rec_index(c) * RecA<P>::N;
    double cay[P + 1], caz[P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i) { cay[i] = ra[i]; caz[i] = ra[P + 1 + i]; }
    const float plo = a.ws.prange[0], phi = a.ws.prange[1];
    const float pscale = (float)(WS_NP - 1) / (phi - plo);
    const double dt2_dx = a.dt * a.dt * a.inv_dx;
    // rows in batches of PRED_BATCH, the next batch's loads issued before the
    // current one is computed (a row is short work next to a memory round trip)
    constexpr int B = PRED_BATCH;
    double xn[B], pn[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int il = min(wb + b * WAVE + lane, we - 1);
        xn[b] = wb < we ? a.xi[il] : 0.0;
        pn[b] = wb < we ? a.p[il] : 0.0;
    }
    __syncthreads();
    __builtin_amdgcn_s_waitcnt(0);
    Moments<P> mo{};
    int flags = 0;
    for (int row = wb; row < we; row += B * WAVE) {
        double xc[B], pc[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            xc[b] = xn[b];
            pc[b] = pn[b];
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int il = min(row + (B + b) * WAVE + lane, we - 1);
            xn[b] = a.xi[il];
            pn[b] = a.p[il];
        }
        __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the arithmetic
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int ia = row + b * WAVE + lane;
            const bool valid = ia < we;
            const double xi0 = xc[b], p0 = pc[b];
            double t0 = xi0 - (double)c;
            wave_flag(flags, !(t0 >= 0.0), FLAG_ORDER);
            wave_flag(flags, !(t0 < 1.0), FLAG_ORDER);
            t0 = fmin(fmax(t0, 0.0), 1.0);
            const double A0y = horner<P + 1>(cay, t0), A0z = horner<P + 1>(caz, t0);
            const double g00 = fsqrt(fma(p0, p0, 1.0) + A0y * A0y + A0z * A0z);
            const float ft = (float)t0 * (float)(WS_NT - 1);
            const int it = min((int)ft, WS_NT - 2);
            const float wt = ft - (float)it;
            const float fp = fminf(fmaxf(((float)p0 - plo) * pscale, 0.0f), (float)(WS_NP - 1));
            const int ip = min((int)fp, WS_NP - 2);
            const float wp = fp - (float)ip;
            const float *q = tab + it * WS_NP + ip;
            const float y = (1.0f - wt) * ((1.0f - wp) * q[0] + wp * q[1]) + wt * ((1.0f - wp) * q[WS_NP] + wp * q[WS_NP + 1]);
            const double d = a.dt_dx * p0 * frcp(g00) + dt2_dx * (double)y;
            double t1;
            int s;
            end_point(xi0, d, c, t1, s, flags);
            stage_deposit<P, double>(mo, __ballot(s != 0) != 0, t0, t1, s, valid ? 1.0 : 0.0);
            if (valid) {   // the sweep after it reads one of the two copies
                if (a.f1) a.f1[ia] = (float)d;
                else a.d1[ia] = d;
            }
        }
    }
    const double slot = moments_to_slots<P>(mo);
    const int fl = flags;   // wave-uniform (set through wave_flag)
    double *out = a.part + ((size_t)item * nw + wid) * UnitI<P>::N;
    double v = slot;
    v = lane == P + 2 ? 0.0 : v;
    v = lane == P + 3 ? (double)fl : v;
    if (lane < UnitI<P>::N) out[lane] = v;
}

// One block per work item; the grid may exceed the item count (the count of a
// step enqueued ahead is only known on the device) and the extra blocks exit.
template <int P>
__global__ void __launch_bounds__(MAX_BLOCK) k_ws_predict(SweepIArgs a) {
    ws_predict_item<P>(a, blockIdx.x);
}

// ---- launchers ------------------------------------------------------------
void launch_ws_init(int P, hipStream_t s, float *theta, uint64_t seed) {
    const int np = ws_nparams(ws_d(P));
#define ECPIC_WI(PP) case PP: launch_k((k_ws_init<ws_d(PP)>), dim3((np + 255) / 256), dim3(256), 0, s, theta, seed); break;
    switch (P) { ECPIC_WI(2) ECPIC_WI(3) ECPIC_WI(4) ECPIC_WI(5) }
#undef ECPIC_WI
}

void launch_ws_stats(hipStream_t s, const float *feat, const float *targ, int64_t n, int D, float *mu, float *sd,
                     float *prange) {
    launch_k(k_ws_stats, dim3(D + 2), dim3(256), 0, s, feat, targ, n, D, mu, sd, prange);
}

// One optimiser step (update != 0) or only the gradient (grad_out) of a batch.
void launch_ws_step(int P, hipStream_t s, float *theta, float *m, float *v, const float *mu, const float *sd,
                    const float *feat, const float *targ, int64_t n, int direct, uint64_t seed, int64_t step, int B,
                    float *pgrad, float *ploss, float lr, int update, float *grad_out, float *loss_out) {
    const int D = ws_d(P), np = ws_nparams(D);
    const int64_t cnt = direct ? n : B;
    const int nblk = (int)((cnt + 31) / 32);
#define ECPIC_WS(PP)                                                                                      \
    case PP:                                                                                              \
        launch_k((k_ws_fwd_bwd<ws_d(PP)>), dim3(nblk), dim3(64), 0, s, theta, mu, sd, feat, targ, \
                           n, direct, seed, step, B, pgrad, ploss);                                       \
        break;
    switch (P) { ECPIC_WS(2) ECPIC_WS(3) ECPIC_WS(4) ECPIC_WS(5) }
#undef ECPIC_WS
    launch_k(k_ws_adam, dim3((np + 255) / 256), dim3(256), 0, s, theta, m, v, pgrad, nblk, np, lr,
                       (int)(step + 1), update, grad_out, ploss, 1.0f / (2.0f * (float)cnt), loss_out);
}

void launch_ws_w2_bf16(int P, hipStream_t s, const float *theta, unsigned short *w2b) {
#define ECPIC_WB(PP) case PP: launch_k((k_ws_w2_bf16<ws_d(PP)>), dim3(H * H / 256), dim3(256), 0, s, theta, w2b); break;
    switch (P) { ECPIC_WB(2) ECPIC_WB(3) ECPIC_WB(4) ECPIC_WB(5) }
#undef ECPIC_WB
}

void launch_ws_predict(int P, int grid, int block, hipStream_t s, const SweepIArgs &a) {
#define ECPIC_WP(PP) case PP: launch_k((k_ws_predict<PP>), dim3(grid), dim3(block), 0, s, a); break;
    switch (P) { ECPIC_WP(2) ECPIC_WP(3) ECPIC_WP(4) ECPIC_WP(5) }
#undef ECPIC_WP
}

void launch_ws_table(int P, hipStream_t s, const WsNet &net, const unsigned short *w2b, const double *coefA,
                     const double *ay, const double *az, const double *ex, int M, float *table) {
    const int grid = (M + WS_CELLS - 1) / WS_CELLS;
#define ECPIC_WT(PP)                                                                                             \
    case PP:                                                                                                     \
        launch_k((k_ws_table<PP>), dim3(grid), dim3(64 * WS_CELLS), 0, s, net, w2b, coefA, ay, az, ex, \
                           M, table);                                                                            \
        break;
    switch (P) { ECPIC_WT(2) ECPIC_WT(3) ECPIC_WT(4) ECPIC_WT(5) }
#undef ECPIC_WT
}

}  // namespace ecpic
