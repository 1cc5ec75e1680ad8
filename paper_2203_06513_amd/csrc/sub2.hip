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
// where b^ is the deposit without the weight.  The particle kernel evaluates
// A^n and A^(k) as per-cell polynomials (coef.hpp) and accumulates the deposit
// as moments sum_a c_a t_a^i, turned into the P+1 V0 coefficients once per
// block.
#include "coef.hpp"

namespace ecpic {

__device__ __forceinline__ bool prev_converged2(DevStatus *st, int k, double tol, bool writer) {
    if (k <= 0) return false;
    const double r = dbits(st->re_bits[(k - 1) & 1]);
    if (writer && k - 1 < MAX_HIST) st->res_hist[k - 1] = r;
    if (r <= tol) {
        if (writer) { st->kconv = k - 1; st->res = r; }
        return true;
    }
    return false;
}

// One particle of a Subsystem II iteration: the deposit coefficients
// c = (A^(k) + A^n)/(gamma^n + gamma^(k)) and its local coordinate.
template <int P>
__device__ __forceinline__ void sub2_coef(const double *cn, const double *ck, double t0, double p0, double &cy,
                                          double &cz) {
    const double Any = horner<P + 1>(cn, t0), Anz = horner<P + 1>(cn + P + 1, t0);
    const double Aky = horner<P + 1>(ck, t0), Akz = horner<P + 1>(ck + P + 1, t0);
    const double q = fma(p0, p0, 1.0);
    const double gn = fsqrt(q + Any * Any + Anz * Anz);
    const double gk = fsqrt(q + Aky * Aky + Akz * Akz);
    const double inv = frcp(gn + gk);
    cy = (Aky + Any) * inv;
    cz = (Akz + Anz) * inv;
}

template <int P>
__global__ void __launch_bounds__(MAX_BLOCK) k_sweep_II(SweepIIArgs a) {
    __shared__ double lds[MAX_WAVES * 2 * (P + 1)];
    constexpr int NA = RecA<P>::N;
    DevStatus *st = a.st;
    const int item = blockIdx.x;
    if (item >= *a.items.n_items) return;
    if (!st->gate | st->flags | (st->kconv >= 0)) return;
    const int k = a.k;
    if (prev_converged2(st, k, a.tol, threadIdx.x == 0)) return;
    const int c = a.items.cell[item];
    const int beg = a.items.begin[item], end = a.items.begin[item + 1];
    const double *rn = a.coefAn + (size_t)rec_index(c) * NA;
    const double *rk = ((k & 1) ? a.coefAk1 : a.coefAk0) + (size_t)rec_index(c) * NA;
    double cn[NA], ck[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) { cn[i] = rn[i]; ck[i] = rk[i]; }
    double my[P + 1], mz[P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i) { my[i] = 0.0; mz[i] = 0.0; }
    int flags = 0;
    const int B = blockDim.x;
    for (int ia = beg + threadIdx.x; ia < end; ia += 2 * B) {
        const int ib = ia + B;
        const bool vb = ib < end;
        const int ibs = vb ? ib : ia;
        const double xa = a.xi[ia], xb = a.xi[ibs];
        const double pa = a.p[ia], pb = a.p[ibs];
        double ta = xa - (double)c, tb = xb - (double)c;
        if (!(ta >= 0.0 && ta < 1.0)) { flags |= FLAG_ORDER; ta = 0.5; }
        if (!(tb >= 0.0 && tb < 1.0)) { flags |= FLAG_ORDER; tb = 0.5; }
        double cya, cza, cyb, czb;
        sub2_coef<P>(cn, ck, ta, pa, cya, cza);
        sub2_coef<P>(cn, ck, tb, pb, cyb, czb);
        const double wb = vb ? 1.0 : 0.0;
        cyb *= wb;
        czb *= wb;
        double sa = 1.0, sb = 1.0;
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            my[j] = fma(cya, sa, fma(cyb, sb, my[j]));
            mz[j] = fma(cza, sa, fma(czb, sb, mz[j]));
            sa *= ta;
            sb *= tb;
        }
    }
    // block sums of the moments, then V0 slot q <-> index c - P + q
    double v[2 * (P + 1)];
#pragma unroll
    for (int j = 0; j <= P; ++j) { v[j] = my[j]; v[P + 1 + j] = mz[j]; }
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
#pragma unroll 1
    for (int j = 0; j < 2 * (P + 1); ++j) {
        const double s = wave_sum(v[j]);
        if (lane == 0) lds[wid * 2 * (P + 1) + j] = s;
    }
    __syncthreads();
    const int q = threadIdx.x;
    if (q < 2 * (P + 1)) {
        constexpr Pieces<P> Bp{};
        const int comp = q / (P + 1), slot = q % (P + 1), m = P - slot;
        double out = 0.0;
        for (int j = 0; j <= P; ++j) {
            double t = 0.0;
            for (int w = 0; w < nw; ++w) t += lds[w * 2 * (P + 1) + comp * (P + 1) + j];
            out += Bp.c[m][j] * t;
        }
        a.part[(size_t)item * 2 * (P + 1) + q] = out;
    }
    flags = wave_or(flags);
    if (lane == 0 && flags) atomicOr(&st->flags, flags);
}

// sum_i taps[i] S[ntaps - 1 - i] for two interleaved vectors, split accumulators.
__device__ __forceinline__ void conv2x2(const double *taps, int ntaps, const double *Sy, const double *Sz,
                                       double &cy, double &cz) {
    double y0 = 0.0, y1 = 0.0, z0 = 0.0, z1 = 0.0;
    int i = 0;
    for (; i + 1 < ntaps; i += 2) {
        y0 = fma(taps[i], Sy[ntaps - 1 - i], y0);
        z0 = fma(taps[i], Sz[ntaps - 1 - i], z0);
        y1 = fma(taps[i + 1], Sy[ntaps - 2 - i], y1);
        z1 = fma(taps[i + 1], Sz[ntaps - 2 - i], z1);
    }
    if (i < ntaps) {
        y0 = fma(taps[i], Sy[ntaps - 1 - i], y0);
        z0 = fma(taps[i], Sz[ntaps - 1 - i], z0);
    }
    cy = y0 + y1;
    cz = z0 + z1;
}

// New e_perp iterate, A-records of the next a^(k+1).  Block b computes e on
// cells [256 b - P, 256 b + 256) (the first P only for records).
template <int P>
__global__ void __launch_bounds__(256) k_field_II(FieldIIArgs a) {
    extern __shared__ double smem[];
    __shared__ double ldsm[MAX_WAVES];
    __shared__ int ldsf[MAX_WAVES];
    constexpr int NA = RecA<P>::N, NS = 2 * (P + 1);
    DevStatus *st = a.st;
    if (!st->gate | st->flags | (st->kconv >= 0)) return;
    const int k = a.k;
    const int M = a.M;
    const int j0 = blockIdx.x * 256 - P;
    const int nout = 256 + P;
    const int mhi = a.mlo + a.ntaps - 1;
    const int slen = nout + a.ntaps - 1;   // b on cells [j0 - mhi, j0 - mhi + slen)
    const int clo = j0 - mhi;              // b_j needs the partials of cells j .. j+P
    const int clen = slen + P;
    double *cp = smem;
    double *Sy = cp + (size_t)clen * NS;
    double *Sz = Sy + slen;
    double *eyl = Sz + slen;
    double *ezl = eyl + nout;
    for (int t = threadIdx.x; t < clen; t += blockDim.x) {
        const int c = imod(clo + t, M);
#pragma unroll
        for (int q = 0; q < NS; ++q) cp[t * NS + q] = 0.0;
        for (int i = a.items.cell_first[c]; i < a.items.cell_first[c + 1]; ++i) {
#pragma unroll
            for (int q = 0; q < NS; ++q) cp[t * NS + q] += a.part[(size_t)i * NS + q];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < slen; t += blockDim.x) {
        double sy = 0.0, sz = 0.0;
#pragma unroll
        for (int r = 0; r <= P; ++r) {   // cell j + r: slot P - r
            sy += cp[(t + r) * NS + (P - r)];
            sz += cp[(t + r) * NS + P + 1 + (P - r)];
        }
        Sy[t] = sy;
        Sz[t] = sz;
    }
    __syncthreads();
    const double *eyk = k == 0 ? a.eyn : ((k & 1) ? a.ey1 : a.ey0);
    const double *ezk = k == 0 ? a.ezn : ((k & 1) ? a.ez1 : a.ez0);
    double *eyo = (k & 1) ? a.ey0 : a.ey1;
    double *ezo = (k & 1) ? a.ez0 : a.ez1;
    double *Aout = ((k + 1) & 1) ? a.coefAk1 : a.coefAk0;
    double re = 0.0;
    int flags = 0;
    for (int q = threadIdx.x; q < nout; q += blockDim.x) {
        const int jj = j0 + q;
        const int j = imod(jj, M);
        double cy, cz;
        conv2x2(a.taps, a.ntaps, Sy + q, Sz + q, cy, cz);
        const double ny = a.E0y[j] + a.coef * cy;
        const double nz = a.E0z[j] + a.coef * cz;
        eyl[q] = ny;
        ezl[q] = nz;
        if (q >= P && jj < M) {
            store_padded(eyo, M, j, ny);
            store_padded(ezo, M, j, nz);
            re = fmax(re, fmax(fabs(ny - eyk[j + HALO]), fabs(nz - ezk[j + HALO])));
            if (!(fabs(ny) < 1.0e300) || !(fabs(nz) < 1.0e300)) flags |= FLAG_NONFINITE;
        }
    }
    __syncthreads();
    {
        const int q = threadIdx.x + P;
        const int j = j0 + q;
        if (j < M) {
            constexpr Pieces<P> B{};
            for (int i = 0; i <= P; ++i) {
                double sy = 0.0, sz = 0.0;
                for (int m = 0; m <= P; ++m) {
                    const int jj = j - m, jm = imod(jj, M);
                    const double ay = a.ayn[jm + HALO] - a.half_dt * (a.eyn[jm + HALO] + eyl[jj - j0]);
                    const double az = a.azn[jm + HALO] - a.half_dt * (a.ezn[jm + HALO] + ezl[jj - j0]);
                    sy += ay * B.c[m][i];
                    sz += az * B.c[m][i];
                }
                store_record(Aout, M, j, NA, i, sy);
                store_record(Aout, M, j, NA, P + 1 + i, sz);
            }
        }
    }
    block_max_or(re, flags, ldsm, ldsf);
    if (threadIdx.x == 0) {
        atomicMax(&st->re_bits[k & 1], bitsd(re));
        if (flags) atomicOr(&st->flags, flags);
        if (blockIdx.x == 0) st->re_bits[(k + 1) & 1] = 0ull;
    }
}

struct Stencil {
    double v[2 * MAX_DEG + 1];
    int half;
};

// Start of Subsystem II: A-records of a^n and of a^(0) = a^n - dt e^n.
template <int P>
__global__ void __launch_bounds__(256) k_prep_II(const DevStatus *st, const double *ayn, const double *azn,
                                                 const double *eyn, const double *ezn, double dt, double *coefAn,
                                                 double *coefAk0, int M) {
    if (!st->gate) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= M) return;
    constexpr Pieces<P> B{};
    constexpr int NA = RecA<P>::N;
    for (int i = 0; i <= P; ++i) {
        double ny = 0.0, nz = 0.0, ky = 0.0, kz = 0.0;
        for (int m = 0; m <= P; ++m) {
            const int j = c - m + HALO;
            ny += ayn[j] * B.c[m][i];
            nz += azn[j] * B.c[m][i];
            ky += (ayn[j] - dt * eyn[j]) * B.c[m][i];
            kz += (azn[j] - dt * ezn[j]) * B.c[m][i];
        }
        store_record(coefAn, M, c, NA, i, ny);
        store_record(coefAn, M, c, NA, P + 1 + i, nz);
        store_record(coefAk0, M, c, NA, i, ky);
        store_record(coefAk0, M, c, NA, P + 1 + i, kz);
    }
}

// E0 = A^{-1} [(M0^ - r^2 K^) e^n + (dt/dx^2) K^ a^n] for both components: the
// right-hand side is formed on the block's input window in LDS and convolved
// with the first row of A^{-1}.
__global__ void __launch_bounds__(256) k_E0_II(const DevStatus *st, const double *eyn, const double *ezn,
                                               const double *ayn, const double *azn, Stencil m0, Stencil kk,
                                               double r2, double ck, const double *taps, int ntaps, int mlo, int M,
                                               double *E0y, double *E0z) {
    extern __shared__ double R[];   // [2][256 + ntaps]
    if (!st->gate) return;
    const int j0 = blockIdx.x * 256;
    const int mhi = mlo + ntaps - 1;
    const int len = 256 + ntaps - 1;
    double *Ry = R, *Rz = R + len;
    for (int idx = threadIdx.x; idx < len; idx += blockDim.x) {
        const int j = imod(j0 - mhi + idx, M);
        double sy = 0.0, sz = 0.0;
        for (int q = -m0.half; q <= m0.half; ++q) {
            const double cm = m0.v[q + m0.half] - r2 * kk.v[q + kk.half];
            const double ka = ck * kk.v[q + kk.half];
            sy += cm * eyn[j + q + HALO] + ka * ayn[j + q + HALO];
            sz += cm * ezn[j + q + HALO] + ka * azn[j + q + HALO];
        }
        Ry[idx] = sy;
        Rz[idx] = sz;
    }
    __syncthreads();
    const int j = j0 + threadIdx.x;
    if (j >= M) return;
    double cy = 0.0, cz = 0.0;
    for (int i = 0; i < ntaps; ++i) {
        const int o = threadIdx.x + mhi - (mlo + i);
        cy = fma(taps[i], Ry[o], cy);
        cz = fma(taps[i], Rz[o], cz);
    }
    E0y[j] = cy;
    E0z[j] = cz;
}

// out_j = alpha * sum_i taps[i] in[(j - mlo - i) mod M]  (in, out unpadded)
__global__ void __launch_bounds__(256) k_conv(const double *in, double *out, const double *taps, int ntaps, int mlo,
                                              double alpha, int M) {
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
                                                   double *az_next, double half_dt, int M, int nsweeps,
                                                   double tol) {
    if (!st->gate || st->flags || st->committed) return;
    int kc = st->kconv;
    if (kc < 0) {
        if (!prev_converged2(st, nsweeps, tol, blockIdx.x == 0 && threadIdx.x == 0)) return;
        kc = nsweeps - 1;
    }
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
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
    const int slen = 256 + P + a.ntaps - 1;
    const size_t lds = sizeof(double) * ((size_t)(slen + P) * 2 * (P + 1) + 2 * slen + 2 * (256 + P));
#define ECPIC_F2(PP) case PP: hipLaunchKernelGGL((k_field_II<PP>), dim3(grid), dim3(256), lds, s, a); break;
    switch (P) { ECPIC_F2(2) ECPIC_F2(3) ECPIC_F2(4) ECPIC_F2(5) }
#undef ECPIC_F2
}

void launch_prep_II(int P, hipStream_t s, const DevStatus *st, const double *ayn, const double *azn,
                    const double *eyn, const double *ezn, double dt, double *coefAn, double *coefAk0, int M) {
    const int grid = (M + 255) / 256;
#define ECPIC_P2(PP)                                                                                       \
    case PP:                                                                                               \
        hipLaunchKernelGGL((k_prep_II<PP>), dim3(grid), dim3(256), 0, s, st, ayn, azn, eyn, ezn, dt, coefAn, \
                           coefAk0, M);                                                                    \
        break;
    switch (P) { ECPIC_P2(2) ECPIC_P2(3) ECPIC_P2(4) ECPIC_P2(5) }
#undef ECPIC_P2
}

void launch_E0_II(hipStream_t s, const DevStatus *st, const double *eyn, const double *ezn, const double *ayn,
                  const double *azn, const double *m0, const double *kr, int P, double r2, double ck,
                  const double *taps, int ntaps, int mlo, int M, double *E0y, double *E0z) {
    Stencil a{}, b{};
    a.half = P; b.half = P;
    for (int q = 0; q <= 2 * P; ++q) { a.v[q] = m0[q]; b.v[q] = kr[q]; }
    const size_t lds = sizeof(double) * 2 * (256 + ntaps);
    hipLaunchKernelGGL(k_E0_II, dim3((M + 255) / 256), dim3(256), lds, s, st, eyn, ezn, ayn, azn, a, b, r2, ck, taps,
                       ntaps, mlo, M, E0y, E0z);
}

void launch_conv(int grid, hipStream_t s, const double *in, double *out, const double *taps, int ntaps, int mlo,
                 double alpha, int M) {
    hipLaunchKernelGGL(k_conv, dim3(grid), dim3(256), 0, s, in, out, taps, ntaps, mlo, alpha, M);
}

void launch_commit_II(int grid, hipStream_t s, DevStatus *st, const double *eyn, const double *ezn,
                      const double *ayn, const double *azn, const double *ey0, const double *ey1,
                      const double *ez0, const double *ez1, double *ey_next, double *ez_next,
                      double *ay_next, double *az_next, double half_dt, int M, int nsweeps, double tol) {
    hipLaunchKernelGGL(k_commit_II, dim3(grid), dim3(256), 0, s, st, eyn, ezn, ayn, azn, ey0, ey1, ez0, ez1,
                       ey_next, ez_next, ay_next, az_next, half_dt, M, nsweeps, tol);
}

}  // namespace ecpic
