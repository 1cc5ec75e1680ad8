// Diagnostics (discrete Hamiltonian, charge, Gauss-law residual), the initial
// discrete Poisson solve, the initial cell sort and the host <-> device
// conversions of the particle arrays.
#include "common.hpp"
#include "spline.hpp"

namespace ecpic {

// ---- discrete Hamiltonian (eq. discrete_H, spin term off) -----------------
// Kinetic part per item: sum_a (gamma_a - 1), with gamma - 1 written
// (p^2 + |A|^2)/(gamma + 1) to avoid the cancellation near gamma = 1.
template <int P>
__global__ void __launch_bounds__(MAX_BLOCK) k_energy_part(const double *xi, const double *p, ItemList items,
                                                           const double *ay, const double *az, double *part) {
    __shared__ double lds[MAX_WAVES];
    const int item = blockIdx.x;
    if (item >= *items.n_items) return;
    const int c = items.cell[item];
    const int beg = items.begin[item], end = items.begin[item + 1];
    double wy[P + 1], wz[P + 1];
    const int b0 = c - P + HALO;
#pragma unroll
    for (int q = 0; q <= P; ++q) { wy[q] = ay[b0 + q]; wz[q] = az[b0 + q]; }
    double acc[1] = {0.0};
    for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const double t0 = xi[i] - (double)c;
        double B[P + 1];
        basis_values<P>(t0, B);
        double Ay = 0.0, Az = 0.0;
#pragma unroll
        for (int m = 0; m <= P; ++m) { Ay += wy[P - m] * B[m]; Az += wz[P - m] * B[m]; }
        const double q = p[i] * p[i] + Ay * Ay + Az * Az;
        acc[0] += q / (sqrt(1.0 + q) + 1.0);
    }
    const double tot = block_sum_slot<1>(acc, lds);
    if (threadIdx.x == 0) part[item] = tot;
}

struct Rows {
    double m0[2 * MAX_DEG + 1];   // M0^ row, half width P
    double m1[2 * MAX_DEG + 1];   // M1^ row, half width P-1
    double kk[2 * MAX_DEG + 1];   // K^ row, half width P
    int P;
};

// out = {kinetic, e_long, e_trans, b_trans, total}; single block, fixed order.
__global__ void __launch_bounds__(1024) k_energy_final(const double *part, const int32_t *n_items, double w,
                                                      const double *ex, const double *ey, const double *ez,
                                                      const double *ay, const double *az, Rows rows, int M,
                                                      double dx, double *out) {
    __shared__ double lds[16 * 4];
    const int P = rows.P;
    const int ni = *n_items;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < ni; i += blockDim.x) v[0] += part[i];
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        double s1 = 0.0, sy = 0.0, sz = 0.0, ky = 0.0, kz = 0.0;
        for (int q = -(P - 1); q <= P - 1; ++q) s1 += rows.m1[q + P - 1] * ex[j + q + HALO];
        for (int q = -P; q <= P; ++q) {
            sy += rows.m0[q + P] * ey[j + q + HALO];
            sz += rows.m0[q + P] * ez[j + q + HALO];
            ky += rows.kk[q + P] * ay[j + q + HALO];
            kz += rows.kk[q + P] * az[j + q + HALO];
        }
        v[1] += ex[j + HALO] * s1;
        v[2] += ey[j + HALO] * sy + ez[j + HALO] * sz;
        v[3] += ay[j + HALO] * ky + az[j + HALO] * kz;
    }
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) lds[wid * 4 + q] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[4] = {0.0, 0.0, 0.0, 0.0};
        for (int wv = 0; wv < (int)blockDim.x / WAVE; ++wv)
            for (int q = 0; q < 4; ++q) t[q] += lds[wv * 4 + q];
        const double kin = w * t[0];
        const double el = 0.5 * dx * t[1];
        const double et = 0.5 * dx * t[2];
        const double bt = 0.5 / dx * t[3];
        out[0] = kin; out[1] = el; out[2] = et; out[3] = bt; out[4] = kin + el + et + bt;
    }
}

// ---- charge Lambda0(X)^T W 1 and Gauss residual (second remark, Section 4.2)
template <int P>
__global__ void __launch_bounds__(MAX_BLOCK) k_charge_part(const double *xi, ItemList items, double *part) {
    __shared__ double lds[MAX_WAVES * (P + 1)];
    const int item = blockIdx.x;
    if (item >= *items.n_items) return;
    const int c = items.cell[item];
    const int beg = items.begin[item], end = items.begin[item + 1];
    double acc[P + 1];
#pragma unroll
    for (int q = 0; q <= P; ++q) acc[q] = 0.0;
    for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
        double B[P + 1];
        basis_values<P>(xi[i] - (double)c, B);
#pragma unroll
        for (int m = 0; m <= P; ++m) acc[P - m] += B[m];
    }
    const double tot = block_sum_slot<P + 1>(acc, lds);
    if ((int)threadIdx.x <= P) part[(size_t)item * (P + 1) + threadIdx.x] = tot;
}

template <int P>
__global__ void __launch_bounds__(256) k_assemble_charge(ItemList items, const double *part, double w, int M,
                                                         double *rho) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    double s = 0.0;
#pragma unroll
    for (int r = 0; r <= P; ++r) {
        const int c = imod(j + r, M);
        const int slot = P - r;
        for (int i = items.cell_first[c]; i < items.cell_first[c + 1]; ++i) s += part[(size_t)i * (P + 1) + slot];
    }
    rho[j] = w * s;
}

// r_j = (G^T M1 e_x)_j + rho_j - dx, with (G^T M1 e)_j = sum_q m1_q (e_{j+q} - e_{j+1+q}).
__global__ void __launch_bounds__(256) k_gauss(const double *rho, const double *ex, Rows rows, int M, double dx,
                                               double *r, unsigned long long *maxbits) {
    __shared__ double ldsm[4];
    __shared__ int ldsf[4];
    const int P = rows.P;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0;
    if (j < M) {
        double s = 0.0;
        for (int q = -(P - 1); q <= P - 1; ++q)
            s += rows.m1[q + P - 1] * (ex[j + q + HALO] - ex[j + 1 + q + HALO]);
        const double v = s + rho[j] - dx;
        r[j] = v;
        a = fabs(v);
    }
    int f = 0;
    block_max_or(a, f, ldsm, ldsf);
    if (threadIdx.x == 0) atomicMax(maxbits, bitsd(a));
}

// Initial field of the discrete Poisson equation G^T M1 e = dx 1 - rho:
// u = M1 e solves G^T u = rhs, i.e. u_{j+1} = u_j - dx rhs_j; u is shifted to
// zero mean (zero-mean gauge), then e = M1^{-1} u by the convolution kernel.
__global__ void __launch_bounds__(1024) k_poisson_rhs(const double *rho, int M, double dx, double *u) {
    __shared__ double lds[32];
    const int per = (M + blockDim.x - 1) / blockDim.x;
    const int c0 = threadIdx.x * per;
    // mean of rhs
    double loc = 0.0;
    for (int c = c0; c < c0 + per && c < M; ++c) loc += dx - rho[c];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    double s = wave_sum(loc);
    if (lane == 0) lds[wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < nw; ++q) t += lds[q];
        lds[31] = t / M;
    }
    __syncthreads();
    const double mean = lds[31];
    __syncthreads();
    // inclusive prefix of -dx (rhs - mean) over cells, exclusive per chunk
    double chunk = 0.0;
    for (int c = c0; c < c0 + per && c < M; ++c) chunk += -dx * ((dx - rho[c]) - mean);
    // block exclusive scan of chunk sums (doubles)
    double x = chunk;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        double y = __shfl_up(x, o, WAVE);
        if (lane >= o) x += y;
    }
    if (lane == WAVE - 1) lds[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int q = 0; q < nw; ++q) { double t = lds[q]; lds[q] = acc; acc += t; }
    }
    __syncthreads();
    double run = lds[wid] + x - chunk;   // u at cell c0 (u_0 = 0)
    double usum = 0.0;
    for (int c = c0; c < c0 + per && c < M; ++c) {
        u[c] = run;
        usum += run;
        run += -dx * ((dx - rho[c]) - mean);
    }
    __syncthreads();
    double us = wave_sum(usum);
    if (lane == 0) lds[wid] = us;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < nw; ++q) t += lds[q];
        lds[31] = t / M;
    }
    __syncthreads();
    const double umean = lds[31];
    for (int c = c0; c < c0 + per && c < M; ++c) u[c] -= umean;
}

// Padded store of an unpadded vector times alpha.
__global__ void __launch_bounds__(256) k_pad(const double *in, double *out, double alpha, int M) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < M) store_padded(out, M, j, in ? alpha * in[j] : 0.0);
}

__global__ void __launch_bounds__(256) k_unpad(const double *in, double *out, int M) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < M) out[j] = in[j + HALO];
}

// ---- particles in and out -------------------------------------------------
// x any real -> xi = x/dx wrapped into [0, M); key = cell.
__global__ void __launch_bounds__(256) k_init_particles(const double *x, const double *p, int64_t n, double L,
                                                        double inv_dx, int M, double *xi, double *pp,
                                                        int32_t *key, int32_t *val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double xw = fmod(x[i], L);
    if (xw < 0.0) xw += L;
    double v = xw * inv_dx;
    if (v >= (double)M) v -= (double)M;
    if (!(v >= 0.0)) v = 0.0;
    if (v >= (double)M) v = 0.0;
    int c = (int)v;
    if (c >= M) c = M - 1;
    xi[i] = v;
    pp[i] = p[i];
    key[i] = c;
    val[i] = (int32_t)i;
}

// Stable LSD radix sort of (key, val) pairs, 4-bit digits.
constexpr int RADIX_CHUNK = 4096;

__global__ void __launch_bounds__(256) k_radix_hist(const int32_t *key, int64_t n, int shift, int32_t *hist,
                                                    int nblk) {
    __shared__ int h[16];
    if (threadIdx.x < 16) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * RADIX_CHUNK;
    const int64_t b1 = b0 + RADIX_CHUNK < n ? b0 + RADIX_CHUNK : n;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) atomicAdd(&h[(key[i] >> shift) & 15], 1);
    __syncthreads();
    if (threadIdx.x < 16) hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(1024) k_exscan_int(int32_t *a, int64_t n) {
    __shared__ int lds[40];
    const int64_t per = (n + blockDim.x - 1) / blockDim.x;
    const int64_t c0 = (int64_t)threadIdx.x * per;
    int local = 0;
    for (int64_t c = c0; c < c0 + per && c < n; ++c) local += a[c];
    int total;
    int off = block_exscan(local, lds, &total);
    for (int64_t c = c0; c < c0 + per && c < n; ++c) { const int t = a[c]; a[c] = off; off += t; }
}

__global__ void __launch_bounds__(256) k_radix_scatter(const int32_t *kin, const int32_t *vin, int32_t *kout,
                                                       int32_t *vout, int64_t n, int shift, const int32_t *offs,
                                                       int nblk) {
    __shared__ int run[16];
    __shared__ int wc[4][16];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    if (threadIdx.x < 16) run[threadIdx.x] = offs[threadIdx.x * nblk + blockIdx.x];
    const int64_t b0 = (int64_t)blockIdx.x * RADIX_CHUNK;
    const int64_t b1 = b0 + RADIX_CHUNK < n ? b0 + RADIX_CHUNK : n;
    __syncthreads();
    for (int64_t r0 = b0; r0 < b1; r0 += blockDim.x) {
        const int64_t i = r0 + threadIdx.x;
        const bool valid = i < b1;
        const int k = valid ? kin[i] : 0;
        const int v = valid ? vin[i] : 0;
        const int d = (k >> shift) & 15;
        unsigned long long m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const unsigned long long bb = __ballot((d >> b) & 1);
            m &= ((d >> b) & 1) ? bb : ~bb;
        }
        const int rank = __popcll(m & lt);
        if (threadIdx.x < 64) wc[threadIdx.x >> 4][threadIdx.x & 15] = 0;
        __syncthreads();
        if (valid && rank == 0) wc[wid][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            int pre = run[d] + rank;
            for (int q = 0; q < wid; ++q) pre += wc[q][d];
            kout[pre] = k;
            vout[pre] = v;
        }
        __syncthreads();
        if (threadIdx.x < 16) run[threadIdx.x] += wc[0][threadIdx.x] + wc[1][threadIdx.x] + wc[2][threadIdx.x] +
                                                  wc[3][threadIdx.x];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_gather_sorted(const int32_t *val, const double *xi_t, const double *p_t,
                                                       int64_t n, double *xi, double *p, int32_t *id) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = val[i];
    xi[i] = xi_t[v];
    p[i] = p_t[v];
    id[i] = v;
}

// Particles per cell of a cell-grouped order (each cell's particles contiguous,
// cells ascending), from the ends of the runs: the first particle of cell c's run
// adds -i and the last adds i + 1, two atomics per occupied cell whatever its
// count (one atomic per particle serialised on the cell's address: 69 ms for
// 1.28e8 particles in 16384 cells).  count must be zero on entry.
template <class CellOf>
__device__ __forceinline__ void count_runs(CellOf cell_of, int64_t n, int32_t *count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell_of(i);
    const bool first = i == 0 || cell_of(i - 1) != c;
    const bool last = i == n - 1 || cell_of(i + 1) != c;
    const int add = (first ? -(int)i : 0) + (last ? (int)(i + 1) : 0);
    if (first || last) atomicAdd(&count[c], add);
}

__global__ void __launch_bounds__(256) k_count_cells(const int32_t *key, int64_t n, int32_t *count) {
    count_runs([=](int64_t j) { return key[j]; }, n, count);
}

// The same from the particles' positions (xi in [0, M), cell-grouped), for an
// item list rebuilt from the particles alone.
__global__ void __launch_bounds__(256) k_count_cells_xi(const double *xi, int64_t n, int M, int32_t *count) {
    count_runs(
        [=](int64_t j) {
            const double v = xi[j];
            return v >= 0.0 && v < (double)M ? (int)v : 0;
        },
        n, count);
}

__global__ void __launch_bounds__(1024) k_items_from_counts(const int32_t *count, int32_t *start, int M, int chunk,
                                                            int64_t N, ItemList out) {
    __shared__ int lds[40];
    scan_cells(count, start, M, lds);
    __syncthreads();
    build_items(count, start, M, chunk, N, out, lds);
}

__global__ void __launch_bounds__(256) k_unpermute(const double *xi, const double *p, const int32_t *id, int64_t n,
                                                   double dx, double *x_out, double *p_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t d = id[i];
    x_out[d] = xi[i] * dx;
    p_out[d] = p[i];
}

// Current of arbitrary straight segments (a checking entry point built from
// the same segment formulas as the sweep): J_j += w dx int Lambda1_j dxi, by
// floating-point atomics.
template <int P>
__global__ void __launch_bounds__(256) k_deposit_segments(const double *x0, const double *x1, int64_t n,
                                                          double inv_dx, double dx, double w, int M,
                                                          double *J, int *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi0 = x0[i] * inv_dx;
    const double cf = floor(xi0);
    const int c = (int)cf;
    const double t0 = xi0 - cf;
    const double t1 = x1[i] * inv_dx - cf;
    if (!(t1 > -1.0 && t1 < 2.0)) { atomicOr(flags, FLAG_CFL); return; }
    const int s = t1 >= 1.0 ? 1 : (t1 < 0.0 ? -1 : 0);
    double I[P + 2];
    segment_integrals<P>(t0, t1, s, I);
#pragma unroll
    for (int q = 0; q < P + 2; ++q) atomicAdd(&J[imod(c - P + q, M)], w * dx * I[q]);
}

// Plain streaming copy of n doubles (16-byte accesses): the calibration kernel
// for bandwidth and for the fetch/write counters.
__global__ void __launch_bounds__(256) k_copy(const double2 *in, double2 *out, int64_t n2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // one 16-byte element per thread
    if (i < n2) out[i] = in[i];
}

// ---- launchers ------------------------------------------------------------
void launch_energy(int P, int grid, int block, hipStream_t s, const double *xi, const double *p, ItemList items,
                   const double *ay, const double *az, double *part) {
#define CALL(PP) launch_k((k_energy_part<PP>), dim3(grid), dim3(block), 0, s, xi, p, items, ay, az, part)
    ECPIC_DISPATCH(P, CALL)
#undef CALL
}

void launch_energy_final(hipStream_t s, const double *part, const int32_t *n_items, double w, const double *ex,
                         const double *ey, const double *ez, const double *ay, const double *az,
                         const double *m0, const double *m1, const double *kr, int P, int M, double dx,
                         double *out) {
    Rows r{};
    r.P = P;
    for (int q = 0; q <= 2 * P; ++q) { r.m0[q] = m0[q]; r.kk[q] = kr[q]; }
    for (int q = 0; q <= 2 * P - 2; ++q) r.m1[q] = m1[q];
    launch_k(k_energy_final, dim3(1), dim3(1024), 0, s, part, n_items, w, ex, ey, ez, ay, az, r, M, dx,
                       out);
}

void launch_charge(int P, int grid, int block, hipStream_t s, const double *xi, ItemList items, double *part,
                   double w, int M, double *rho) {
#define CALL(PP) launch_k((k_charge_part<PP>), dim3(grid), dim3(block), 0, s, xi, items, part)
    ECPIC_DISPATCH(P, CALL)
#undef CALL
#define CALL(PP) \
    launch_k((k_assemble_charge<PP>), dim3((M + 255) / 256), dim3(256), 0, s, items, part, w, M, rho)
    ECPIC_DISPATCH(P, CALL)
#undef CALL
}

void launch_gauss(hipStream_t s, const double *rho, const double *ex, const double *m1, int P, int M, double dx,
                  double *r, unsigned long long *maxbits) {
    Rows rows{};
    rows.P = P;
    for (int q = 0; q <= 2 * P - 2; ++q) rows.m1[q] = m1[q];
    launch_k(k_gauss, dim3((M + 255) / 256), dim3(256), 0, s, rho, ex, rows, M, dx, r, maxbits);
}

void launch_poisson_rhs(hipStream_t s, const double *rho, int M, double dx, double *u) {
    launch_k(k_poisson_rhs, dim3(1), dim3(1024), 0, s, rho, M, dx, u);
}

void launch_pad(hipStream_t s, const double *in, double *out, double alpha, int M) {
    launch_k(k_pad, dim3((M + 255) / 256), dim3(256), 0, s, in, out, alpha, M);
}

void launch_unpad(hipStream_t s, const double *in, double *out, int M) {
    launch_k(k_unpad, dim3((M + 255) / 256), dim3(256), 0, s, in, out, M);
}

void launch_init_particles(hipStream_t s, const double *x, const double *p, int64_t n, double L, double inv_dx,
                           int M, double *xi, double *pp, int32_t *key, int32_t *val) {
    launch_k(k_init_particles, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, p, n, L, inv_dx, M,
                       xi, pp, key, val);
}

// Sort (key, val) by key, stably; returns through kout/vout (ping-pong buffers).
void radix_sort(hipStream_t s, int32_t *k0, int32_t *v0, int32_t *k1, int32_t *v1, int64_t n, int key_bits,
                int32_t *hist, int32_t **kres, int32_t **vres) {
    const int nblk = (int)((n + RADIX_CHUNK - 1) / RADIX_CHUNK);
    int32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
    for (int shift = 0; shift < key_bits; shift += 4) {
        launch_k(k_radix_hist, dim3(nblk), dim3(256), 0, s, ki, n, shift, hist, nblk);
        launch_k(k_exscan_int, dim3(1), dim3(1024), 0, s, hist, (int64_t)16 * nblk);
        launch_k(k_radix_scatter, dim3(nblk), dim3(256), 0, s, ki, vi, ko, vo, n, shift, hist, nblk);
        int32_t *t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    *kres = ki;
    *vres = vi;
}

void launch_gather_sorted(hipStream_t s, const int32_t *val, const double *xi_t, const double *p_t, int64_t n,
                          double *xi, double *p, int32_t *id) {
    launch_k(k_gather_sorted, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, val, xi_t, p_t, n, xi,
                       p, id);
}

void launch_count_cells(hipStream_t s, const int32_t *key, int64_t n, int32_t *count) {
    if (n > 0)
        launch_k(k_count_cells, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, key, n, count);
}

void launch_count_cells_xi(hipStream_t s, const double *xi, int64_t n, int M, int32_t *count) {
    if (n > 0)
        launch_k(k_count_cells_xi, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xi, n, M, count);
}

void launch_items_from_counts(hipStream_t s, const int32_t *count, int32_t *start, int M, int chunk, int64_t N,
                              ItemList out) {
    launch_k(k_items_from_counts, dim3(1), dim3(1024), 0, s, count, start, M, chunk, N, out);
}

void launch_unpermute(hipStream_t s, const double *xi, const double *p, const int32_t *id, int64_t n, double dx,
                      double *x_out, double *p_out) {
    if (n > 0)
        launch_k(k_unpermute, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xi, p, id, n, dx, x_out,
                           p_out);
}

void launch_copy(hipStream_t s, const double *in, double *out, int64_t n) {
    const int64_t n2 = n / 2;
    launch_k(k_copy, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, (const double2 *)in, (double2 *)out, n2);
}

void launch_deposit_segments(int P, hipStream_t s, const double *x0, const double *x1, int64_t n, double inv_dx,
                             double dx, double w, int M, double *J, int *flags) {
    const unsigned grid = (unsigned)((n + 255) / 256);
#define CALL(PP) \
    launch_k((k_deposit_segments<PP>), dim3(grid), dim3(256), 0, s, x0, x1, n, inv_dx, dx, w, M, J, flags)
    if (n > 0) ECPIC_DISPATCH(P, CALL)
#undef CALL
}

}  // namespace ecpic
