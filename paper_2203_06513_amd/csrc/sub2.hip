// Subsystem II of the Poisson splitting (Section 4.2): update of
// (e_y, e_z, a_y, a_z) with the particles frozen.  The scheme is
//   (M0 + dt^2 K/4) e^{n+1} = (M0 - dt^2 K/4) e^n + dt K a^n + dt b,
//   b = sum_a w (A^{n+1}(x_a) + A^n(x_a)) Lambda0(x_a) / (gamma^n_a + gamma^{n+1}_a),
//   a^{n+1} = a^n - dt/2 (e^n + e^{n+1}),
// solved by fixed-point iteration on e^{n+1} with the particle term b lagged
// and the matrix inverted exactly (its inverse applied as a convolution with
// the first row of the circulant inverse).  With M0 = dx M0^, K = K^/dx and
// r = dt/(2 dx):  e^{n+1} = A^-1 [(M0^ - r^2 K^) e^n + (dt/dx^2) K^ a^n]
//                         + (dt w / dx) A^-1 b^,   A = M0^ + r^2 K^,
// where b^ is the deposit without the weight.
#include "common.hpp"
#include "spline.hpp"

namespace ecpic {

template <int P>
__global__ void __launch_bounds__(MAX_BLOCK) k_sweep_II(SweepIIArgs a) {
    __shared__ double lds[MAX_WAVES * 2 * (P + 1)];
    const DevStatus *st = a.st;
    const int item = blockIdx.x;
    if (item >= *a.items.n_items) return;
    if (!st->gate | st->converged | st->flags) return;
    const int k = st->k;
    const double *eyk = k == 0 ? a.eyn : ((k & 1) ? a.ey1 : a.ey0);
    const double *ezk = k == 0 ? a.ezn : ((k & 1) ? a.ez1 : a.ez0);
    const int c = a.items.cell[item];
    const int beg = a.items.begin[item], end = a.items.begin[item + 1];
    // V0 window, slot q <-> index c - P + q
    double any[P + 1], anz[P + 1], aky[P + 1], akz[P + 1];
    const int b0 = c - P + HALO;
#pragma unroll
    for (int q = 0; q <= P; ++q) {
        any[q] = a.ayn[b0 + q];
        anz[q] = a.azn[b0 + q];
        aky[q] = any[q] - a.half_dt * (a.eyn[b0 + q] + eyk[b0 + q]);
        akz[q] = anz[q] - a.half_dt * (a.ezn[b0 + q] + ezk[b0 + q]);
    }
    double acc[2 * (P + 1)];
#pragma unroll
    for (int q = 0; q < 2 * (P + 1); ++q) acc[q] = 0.0;
    int flags = 0;
    for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const double xi0 = a.xi[i];
        const double p0 = a.p[i];
        double t0 = xi0 - (double)c;
        if (!(t0 >= 0.0 && t0 < 1.0)) { flags |= FLAG_ORDER; t0 = 0.5; }
        double B[P + 1];
        basis_values<P>(t0, B);
        double Any = 0.0, Anz = 0.0, Aky = 0.0, Akz = 0.0;
#pragma unroll
        for (int m = 0; m <= P; ++m) {
            Any += any[P - m] * B[m];
            Anz += anz[P - m] * B[m];
            Aky += aky[P - m] * B[m];
            Akz += akz[P - m] * B[m];
        }
        const double pp = 1.0 + p0 * p0;
        const double gn = sqrt(pp + Any * Any + Anz * Anz);
        const double gk = sqrt(pp + Aky * Aky + Akz * Akz);
        const double inv = 1.0 / (gn + gk);
        const double cy = (Aky + Any) * inv, cz = (Akz + Anz) * inv;
#pragma unroll
        for (int m = 0; m <= P; ++m) {
            acc[P - m] += cy * B[m];
            acc[P + 1 + P - m] += cz * B[m];
        }
    }
    const double tot = block_sum_slot<2 * (P + 1)>(acc, lds);
    if ((int)threadIdx.x < 2 * (P + 1)) a.part[(size_t)item * 2 * (P + 1) + threadIdx.x] = tot;
    flags = wave_or(flags);
    if ((threadIdx.x & (WAVE - 1)) == 0 && flags) atomicOr(&a.st->flags, flags);
}

template <int P>
__device__ __forceinline__ void assemble_v0(const ItemList &it, const double *part, int j, int M, double &sy,
                                            double &sz) {
    sy = 0.0;
    sz = 0.0;
#pragma unroll
    for (int r = 0; r <= P; ++r) {
        const int c = imod(j + r, M);
        const int slot = P - r;   // V0 index c - P + slot == j (unwrapped)
        const int i0 = it.cell_first[c], i1 = it.cell_first[c + 1];
        for (int i = i0; i < i1; ++i) {
            sy += part[(size_t)i * 2 * (P + 1) + slot];
            sz += part[(size_t)i * 2 * (P + 1) + P + 1 + slot];
        }
    }
}

template <int P>
__global__ void __launch_bounds__(256) k_field_II(FieldIIArgs a) {
    extern __shared__ double S[];   // [2][256 + ntaps]
    __shared__ double ldsm[MAX_WAVES];
    __shared__ int ldsf[MAX_WAVES];
    __shared__ int last;
    DevStatus *st = a.st;
    if (!st->gate | st->converged | st->flags) return;
    const int k = st->k;
    const int M = a.M;
    const int j0 = blockIdx.x * 256;
    const int mhi = a.mlo + a.ntaps - 1;
    const int len = 256 + a.ntaps - 1;
    double *Sy = S, *Sz = S + len;
    for (int idx = threadIdx.x; idx < len; idx += blockDim.x) {
        const int j = imod(j0 - mhi + idx, M);
        assemble_v0<P>(a.items, a.part, j, M, Sy[idx], Sz[idx]);
    }
    __syncthreads();
    const double *eyk = k == 0 ? a.eyn : ((k & 1) ? a.ey1 : a.ey0);
    const double *ezk = k == 0 ? a.ezn : ((k & 1) ? a.ez1 : a.ez0);
    double *eyo = (k & 1) ? a.ey0 : a.ey1;
    double *ezo = (k & 1) ? a.ez0 : a.ez1;
    double re = 0.0;
    int flags = 0;
    const int j = j0 + threadIdx.x;
    if (j < M) {
        double cy = 0.0, cz = 0.0;
        for (int i = 0; i < a.ntaps; ++i) {
            const int q = threadIdx.x + mhi - (a.mlo + i);
            cy += a.taps[i] * Sy[q];
            cz += a.taps[i] * Sz[q];
        }
        const double ny = a.E0y[j] + a.coef * cy;
        const double nz = a.E0z[j] + a.coef * cz;
        store_padded(eyo, M, j, ny);
        store_padded(ezo, M, j, nz);
        re = fmax(fabs(ny - eyk[j + HALO]), fabs(nz - ezk[j + HALO]));
        if (!(fabs(ny) < 1.0e300) || !(fabs(nz) < 1.0e300)) flags |= FLAG_NONFINITE;
    }
    block_max_or(re, flags, ldsm, ldsf);
    if (threadIdx.x == 0) {
        atomicMax(&st->re_bits, bitsd(re));
        if (flags) atomicOr(&st->flags, flags);
        __threadfence();
        const unsigned ticket = atomicAdd(&st->counter, 1u);
        last = (ticket == gridDim.x - 1);
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        const double r = dbits(atomicAdd(&st->re_bits, 0ull));
        st->res = r;
        if (k < MAX_HIST) st->res_hist[k] = r;
        if (r <= a.tol && st->flags == 0) {
            st->converged = 1;
            st->kconv = k;
        }
        st->re_bits = 0ull;
        st->counter = 0u;
        __threadfence();
        st->k = k + 1;
    }
}

struct Stencil {
    double v[2 * MAX_DEG + 1];
    int half;
};

// Constant right-hand side: (M0^ - r^2 K^) e^n + (dt/dx^2) K^ a^n, per component.
__global__ void __launch_bounds__(256) k_rhs_II(const DevStatus *st, const double *eyn, const double *ezn,
                                                const double *ayn, const double *azn, Stencil m0,
                                                Stencil kk, double r2, double ck, int M, double *ry,
                                                double *rz) {
    if (!st->gate) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    double sy = 0.0, sz = 0.0;
    for (int q = -m0.half; q <= m0.half; ++q) {
        const double cm = m0.v[q + m0.half] - r2 * kk.v[q + kk.half];
        sy += cm * eyn[j + q + HALO] + ck * kk.v[q + kk.half] * ayn[j + q + HALO];
        sz += cm * ezn[j + q + HALO] + ck * kk.v[q + kk.half] * azn[j + q + HALO];
    }
    ry[j] = sy;
    rz[j] = sz;
}

// out_j = alpha * sum_i taps[i] in[(j - mlo - i) mod M]  (in, out unpadded)
__global__ void __launch_bounds__(256) k_conv(const DevStatus *st, const double *in, double *out,
                                              const double *taps, int ntaps, int mlo, double alpha, int M) {
    if (st && !st->gate) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    double s = 0.0;
    for (int i = 0; i < ntaps; ++i) s += taps[i] * in[imod(j - mlo - i, M)];
    out[j] = alpha * s;
}

__global__ void __launch_bounds__(256) k_commit_II(DevStatus *st, const double *eyn, const double *ezn,
                                                   const double *ayn, const double *azn, const double *ey0,
                                                   const double *ey1, const double *ez0, const double *ez1,
                                                   double *ey_next, double *ez_next, double *ay_next,
                                                   double *az_next, double half_dt, int M) {
    if (!(st->gate && st->converged && !st->committed && st->flags == 0)) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int kc = st->kconv;
    const double *eya = ((kc + 1) & 1) ? ey1 : ey0;
    const double *eza = ((kc + 1) & 1) ? ez1 : ez0;
    const double ny = eya[j + HALO], nz = eza[j + HALO];
    store_padded(ey_next, M, j, ny);
    store_padded(ez_next, M, j, nz);
    store_padded(ay_next, M, j, ayn[j + HALO] - half_dt * (eyn[j + HALO] + ny));
    store_padded(az_next, M, j, azn[j + HALO] - half_dt * (ezn[j + HALO] + nz));
}

void launch_sweep_II(int P, int grid, int block, hipStream_t s, const SweepIIArgs &a) {
#define ECPIC_S2(PP) case PP: hipLaunchKernelGGL((k_sweep_II<PP>), dim3(grid), dim3(block), 0, s, a); break;
    switch (P) { ECPIC_S2(2) ECPIC_S2(3) ECPIC_S2(4) ECPIC_S2(5) }
#undef ECPIC_S2
}

void launch_field_II(int P, int grid, hipStream_t s, const FieldIIArgs &a) {
    const size_t lds = sizeof(double) * 2 * (256 + a.ntaps);
#define ECPIC_F2(PP) case PP: hipLaunchKernelGGL((k_field_II<PP>), dim3(grid), dim3(256), lds, s, a); break;
    switch (P) { ECPIC_F2(2) ECPIC_F2(3) ECPIC_F2(4) ECPIC_F2(5) }
#undef ECPIC_F2
}

void launch_rhs_II(int grid, hipStream_t s, const DevStatus *st, const double *eyn, const double *ezn,
                   const double *ayn, const double *azn, const double *m0, const double *kr, int P,
                   double r2, double ck, int M, double *ry, double *rz) {
    Stencil a{}, b{};
    a.half = P; b.half = P;
    for (int q = 0; q <= 2 * P; ++q) { a.v[q] = m0[q]; b.v[q] = kr[q]; }
    hipLaunchKernelGGL(k_rhs_II, dim3(grid), dim3(256), 0, s, st, eyn, ezn, ayn, azn, a, b, r2, ck, M, ry, rz);
}

void launch_conv(int grid, hipStream_t s, const DevStatus *st, const double *in, double *out, const double *taps,
                 int ntaps, int mlo, double alpha, int M) {
    hipLaunchKernelGGL(k_conv, dim3(grid), dim3(256), 0, s, st, in, out, taps, ntaps, mlo, alpha, M);
}

void launch_commit_II(int grid, hipStream_t s, DevStatus *st, const double *eyn, const double *ezn,
                      const double *ayn, const double *azn, const double *ey0, const double *ey1,
                      const double *ez0, const double *ez1, double *ey_next, double *ez_next,
                      double *ay_next, double *az_next, double half_dt, int M) {
    hipLaunchKernelGGL(k_commit_II, dim3(grid), dim3(256), 0, s, st, eyn, ezn, ayn, azn, ey0, ey1, ez0, ez1,
                       ey_next, ez_next, ay_next, az_next, half_dt, M);
}

}  // namespace ecpic
