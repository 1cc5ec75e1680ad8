// Subsystem I of the Poisson splitting (Section 4.2): implicit discrete-gradient
// update of (x, p, e_x) with a_perp frozen, solved by Picard sweeps.
//
// One sweep k, for every particle a (cell-local coordinates, d = delta/dx):
//   A0 = A_perp(x_a), A1 = A_perp(x_a + delta^(k))          V0 gathers
//   g00 = gamma(p_a, A0), g01 = gamma(p_a, A1)
//   lbar = time-averaged Lambda1 along x_a -> x_a + delta^(k) (line mean)
//   F = lbar.ebar - (A0 + A1).(lbar.G a) / (dx (g00 + g01))
//   p1 = p_a + dt F,  g11 = gamma(p1, A1),  delta^(k+1) = dt (p_a + p1)/(g01 + g11)
//   S += (x1 - x0)/dx * lbar   (current of the step, Jacobi: delta^(k); Seidel: delta^(k+1))
// then e^(k+1) = e_x^n - w M1^-1 (dx S) (field kernel), with the divided
// difference (A1 - A0)/(x1 - x0) taken as lbar.(G a), the 0/0-free identity.
#include "common.hpp"
#include "spline.hpp"

namespace ecpic {

template <int P>
struct Window1 {
    double ay[P + 3], az[P + 3];   // V0 coefficients of cells c-P-1 .. c+1
    double gy[P + 2], gz[P + 2];   // (G a) * dx on V1 indices c-P .. c+1
    double eb[P + 2];              // ebar on V1 indices c-P .. c+1
};

template <int P>
__device__ __forceinline__ void load_window1(Window1<P> &w, int c, const double *ay, const double *az,
                                             const double *en, const double *ek) {
    const int b0 = c - P - 1 + HALO;
#pragma unroll
    for (int k = 0; k < P + 3; ++k) { w.ay[k] = ay[b0 + k]; w.az[k] = az[b0 + k]; }
#pragma unroll
    for (int k = 0; k < P + 2; ++k) {
        w.gy[k] = w.ay[k + 1] - w.ay[k];
        w.gz[k] = w.az[k + 1] - w.az[k];
        w.eb[k] = 0.5 * (en[b0 + 1 + k] + ek[b0 + 1 + k]);
    }
}

// Position bookkeeping: xi0 in [c, c+1); the end point is the rounded
// xi0 + d, so that deposit and committed position describe the same segment.
__device__ __forceinline__ void end_point(double xi0, double d, int c, double &t1, int &s, int &flags) {
    double xi1 = xi0 + d;
    t1 = xi1 - (double)c;
    if (!(t1 > -1.0 && t1 < 2.0)) {   // |d| >= 1 cell, or NaN
        flags |= FLAG_CFL;
        t1 = t1 >= 2.0 ? 1.5 : (t1 <= -1.0 ? -0.5 : 0.5);
    }
    s = t1 >= 1.0 ? 1 : (t1 < 0.0 ? -1 : 0);
}

template <int P>
__device__ __forceinline__ void particle_map(const Window1<P> &w, double t0, double p0, double d,
                                             bool explicit_start, int c, double xi0, double dt,
                                             double dt_dx, double inv_dx, double &dn, double &p1,
                                             double &d_used, double (&lb)[P + 2], double &dr,
                                             int &flags) {
    double B0[P + 1];
    basis_values<P>(t0, B0);
    double A0y = 0.0, A0z = 0.0;
#pragma unroll
    for (int m = 0; m <= P; ++m) {
        A0y += w.ay[P + 1 - m] * B0[m];
        A0z += w.az[P + 1 - m] * B0[m];
    }
    const double pp = p0 * p0;
    const double g00 = sqrt(1.0 + pp + A0y * A0y + A0z * A0z);
    if (explicit_start) d = dt_dx * p0 / g00;
    d_used = d;
    double t1;
    int s;
    end_point(xi0, d, c, t1, s, flags);
    dr = t1 - t0;
    double B1[P + 1];
    basis_values<P>(t1 - (double)s, B1);
    double y0 = 0.0, yR = 0.0, yL = 0.0, z0 = 0.0, zR = 0.0, zL = 0.0;
#pragma unroll
    for (int m = 0; m <= P; ++m) {
        y0 += w.ay[P + 1 - m] * B1[m]; yR += w.ay[P + 2 - m] * B1[m]; yL += w.ay[P - m] * B1[m];
        z0 += w.az[P + 1 - m] * B1[m]; zR += w.az[P + 2 - m] * B1[m]; zL += w.az[P - m] * B1[m];
    }
    const double A1y = s > 0 ? yR : (s < 0 ? yL : y0);
    const double A1z = s > 0 ? zR : (s < 0 ? zL : z0);
    const double qa1 = A1y * A1y + A1z * A1z;
    const double g01 = sqrt(1.0 + pp + qa1);
    line_mean_v1<P>(t0, t1, s, lb);
    double LE = 0.0, LGy = 0.0, LGz = 0.0;
#pragma unroll
    for (int k = 0; k < P + 2; ++k) {
        LE += lb[k] * w.eb[k];
        LGy += lb[k] * w.gy[k];
        LGz += lb[k] * w.gz[k];
    }
    const double F = LE - ((A0y + A1y) * LGy + (A0z + A1z) * LGz) * inv_dx / (g00 + g01);
    p1 = p0 + dt * F;
    const double g11 = sqrt(1.0 + p1 * p1 + qa1);
    dn = dt_dx * (p0 + p1) / (g01 + g11);
    if (!(fabs(dn) < 1.0e300) || !(fabs(p1) < 1.0e300)) flags |= FLAG_NONFINITE;
}

template <int P, bool SEIDEL>
__global__ void __launch_bounds__(MAX_BLOCK) k_sweep_I(SweepIArgs a) {
    __shared__ double lds[MAX_WAVES * (P + 2)];
    __shared__ double ldsm[MAX_WAVES];
    __shared__ int ldsf[MAX_WAVES];
    const DevStatus *st = a.st;
    const int item = blockIdx.x;
    if (item >= *a.items.n_items) return;
    if (!st->gate | st->converged | st->flags) return;
    const int k = st->k;
    const double *din = (k & 1) ? a.d1 : a.d0;
    double *dout = (k & 1) ? a.d0 : a.d1;
    const double *ek = k == 0 ? a.en : ((k & 1) ? a.ek1 : a.ek0);
    const bool explicit_start = (k == 0) && a.explicit_start;
    const int c = a.items.cell[item];
    const int beg = a.items.begin[item], end = a.items.begin[item + 1];

    Window1<P> w;
    load_window1<P>(w, c, a.ay, a.az, a.en, ek);

    double acc[P + 2];
#pragma unroll
    for (int q = 0; q < P + 2; ++q) acc[q] = 0.0;
    double rmax = 0.0;
    int flags = 0;
    for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const double xi0 = a.xi[i];
        const double p0 = a.p[i];
        const double dprev = explicit_start ? 0.0 : din[i];
        double t0 = xi0 - (double)c;
        if (!(t0 >= 0.0 && t0 < 1.0)) { flags |= FLAG_ORDER; t0 = 0.5; }
        double dn, p1, dused, dr, lb[P + 2];
        particle_map<P>(w, t0, p0, dprev, explicit_start, c, xi0, a.dt, a.dt_dx, a.inv_dx, dn, p1, dused,
                        lb, dr, flags);
        if (!SEIDEL && explicit_start) a.d0[i] = dused;   // keep d^(0) for a Jacobi commit
        dout[i] = dn;
        rmax = fmax(rmax, fabs(dn - dused));
        if (SEIDEL) {
            double t1;
            int s;
            end_point(xi0, dn, c, t1, s, flags);
            line_mean_v1<P>(t0, t1, s, lb);
            dr = t1 - t0;
        }
#pragma unroll
        for (int q = 0; q < P + 2; ++q) acc[q] += dr * lb[q];
    }
    const double tot = block_sum_slot<P + 2>(acc, lds);
    if ((int)threadIdx.x < P + 2) a.part[(size_t)item * (P + 2) + threadIdx.x] = tot;
    block_max_or(rmax, flags, ldsm, ldsf);
    if (threadIdx.x == 0) {
        atomicMax(&a.st->rx_bits, bitsd(rmax));
        if (flags) atomicOr(&a.st->flags, flags);
    }
}

// Assemble the current of V1 index j from the item partials (fixed order:
// cells j-1 .. j+P ascending, items of a cell ascending).
template <int P>
__device__ __forceinline__ double assemble_current(const ItemList &it, const double *part, int j, int M) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < P + 2; ++r) {
        const int c = imod(j - 1 + r, M);
        const int slot = P + 1 - r;   // V1 index c - P + slot == j (unwrapped)
        const int i0 = it.cell_first[c], i1 = it.cell_first[c + 1];
        for (int i = i0; i < i1; ++i) s += part[(size_t)i * (P + 2) + slot];
    }
    return s;
}

// Field update of one sweep and the convergence test.  Block b produces
// e^(k+1) on cells [256 b, 256 b + 256); the last block to finish decides.
template <int P>
__global__ void __launch_bounds__(256) k_field_I(FieldIArgs a) {
    extern __shared__ double S[];
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
    for (int idx = threadIdx.x; idx < len; idx += blockDim.x) {
        const int j = imod(j0 - mhi + idx, M);
        S[idx] = assemble_current<P>(a.items, a.part, j, M);
    }
    __syncthreads();
    const double *ek = k == 0 ? a.en : ((k & 1) ? a.ek1 : a.ek0);
    double *eout = (k & 1) ? a.ek0 : a.ek1;
    double re = 0.0;
    int flags = 0;
    const int j = j0 + threadIdx.x;
    if (j < M) {
        double conv = 0.0;
        for (int i = 0; i < a.ntaps; ++i) conv += a.taps[i] * S[threadIdx.x + mhi - (a.mlo + i)];
        const double enew = a.en[j + HALO] - a.w * conv;
        store_padded(eout, M, j, enew);
        re = fabs(enew - ek[j + HALO]);
        if (!(fabs(enew) < 1.0e300)) flags |= FLAG_NONFINITE;
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
        const double rx = dbits(atomicAdd(&st->rx_bits, 0ull)) * a.dx;
        const double rf = dbits(atomicAdd(&st->re_bits, 0ull));
        const double r = fmax(rx, rf);
        st->res = r;
        if (k < MAX_HIST) st->res_hist[k] = r;
        if (r <= a.tol && st->flags == 0) {
            st->converged = 1;
            st->kconv = k;
        }
        st->rx_bits = 0ull;
        st->re_bits = 0ull;
        st->counter = 0u;
        __threadfence();
        st->k = k + 1;
    }
}

// ---- commit: re-evaluate the committed momentum, move the particles and
// keep them cell-sorted.  A particle moves at most one cell per step, so the
// new order of cell c' is [right-movers of c'-1][stayers of c'][left-movers of
// c'+1], each group in the old order (a stable three-way merge).

struct CommitPick {
    const double *d;     // increment to commit
    const double *ek;    // e iterate used in ebar for the momentum
    const double *enew;  // e_x^{n+1}
};

__device__ __forceinline__ CommitPick commit_pick(const CommitIArgs &a) {
    const int kc = a.st->kconv;
    CommitPick r;
    const double *e_after = ((kc + 1) & 1) ? a.ek1 : a.ek0;   // e^(kc+1)
    r.enew = e_after;
    if (a.seidel) {
        r.d = ((kc + 1) & 1) ? a.d1 : a.d0;    // delta^(kc+1)
        r.ek = e_after;
    } else {
        r.d = (kc & 1) ? a.d1 : a.d0;          // delta^(kc)
        r.ek = kc == 0 ? a.en : ((kc & 1) ? a.ek1 : a.ek0);
    }
    return r;
}

__device__ __forceinline__ bool commit_enabled(const DevStatus *st) {
    return st->gate && st->converged && !st->committed && st->flags == 0;
}

__device__ __forceinline__ int mover_type(double xi0, double d, int c) {
    const double t1 = (xi0 + d) - (double)c;
    return t1 >= 1.0 ? 2 : (t1 < 0.0 ? 0 : 1);   // 0 left, 1 stay, 2 right
}

__global__ void __launch_bounds__(MAX_BLOCK) k_commit_count(CommitIArgs a) {
    __shared__ int lds[MAX_WAVES * 3];
    const int item = blockIdx.x;
    if (item >= *a.items.n_items || !commit_enabled(a.st)) return;
    const CommitPick pk = commit_pick(a);
    const int c = a.items.cell[item];
    const int beg = a.items.begin[item], end = a.items.begin[item + 1];
    int n0 = 0, n1 = 0, n2 = 0;
    for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const int t = mover_type(a.cur.xi[i], pk.d[i], c);
        n0 += t == 0; n1 += t == 1; n2 += t == 2;
    }
    n0 = wave_isum(n0); n1 = wave_isum(n1); n2 = wave_isum(n2);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    if (lane == 0) { lds[wid * 3] = n0; lds[wid * 3 + 1] = n1; lds[wid * 3 + 2] = n2; }
    __syncthreads();
    if (threadIdx.x < 3) {
        int s = 0;
        for (int w = 0; w < (int)(blockDim.x + WAVE - 1) / WAVE; ++w) s += lds[w * 3 + threadIdx.x];
        a.cnt[item * 3 + threadIdx.x] = s;
    }
}

__global__ void __launch_bounds__(1024) k_commit_scan(CommitIArgs a) {
    __shared__ int lds[40];
    if (!commit_enabled(a.st)) return;
    const int M = a.M;
    const ItemList &it = a.items;
    // totals per old cell and exclusive prefix of each item within its cell
    for (int c = threadIdx.x; c < M; c += blockDim.x) {
        int r0 = 0, r1 = 0, r2 = 0;
        for (int i = it.cell_first[c]; i < it.cell_first[c + 1]; ++i) {
            a.base[i * 3 + 0] = r0; a.base[i * 3 + 1] = r1; a.base[i * 3 + 2] = r2;
            r0 += a.cnt[i * 3 + 0]; r1 += a.cnt[i * 3 + 1]; r2 += a.cnt[i * 3 + 2];
        }
        a.tot[c * 3 + 0] = r0; a.tot[c * 3 + 1] = r1; a.tot[c * 3 + 2] = r2;
    }
    __syncthreads();
    // new counts: right-movers of c-1, stayers of c, left-movers of c+1
    int32_t *ncount = a.nstart + (M + 1);   // scratch of M ints after nstart
    for (int c = threadIdx.x; c < M; c += blockDim.x)
        ncount[c] = a.tot[imod(c - 1, M) * 3 + 2] + a.tot[c * 3 + 1] + a.tot[imod(c + 1, M) * 3 + 0];
    __syncthreads();
    scan_cells(ncount, a.nstart, M, lds);
    __syncthreads();
    // destination bases of each old item's three groups
    for (int c = threadIdx.x; c < M; c += blockDim.x) {
        const int cm = imod(c - 1, M), cp = imod(c + 1, M), cmm = imod(c - 2, M);
        const int bL = a.nstart[cm] + a.tot[cmm * 3 + 2] + a.tot[cm * 3 + 1];
        const int bS = a.nstart[c] + a.tot[cm * 3 + 2];
        const int bR = a.nstart[cp];
        for (int i = it.cell_first[c]; i < it.cell_first[c + 1]; ++i) {
            a.base[i * 3 + 0] += bL;
            a.base[i * 3 + 1] += bS;
            a.base[i * 3 + 2] += bR;
        }
    }
    __syncthreads();
    build_items(ncount, a.nstart, M, a.chunk, a.N, a.items_next, lds);
    __syncthreads();
    // e_x^{n+1}
    const CommitPick pk = commit_pick(a);
    for (int idx = threadIdx.x; idx < M + 2 * HALO; idx += blockDim.x) a.ex_next[idx] = pk.enew[idx];
}

template <int P>
__global__ void __launch_bounds__(MAX_BLOCK) k_commit_scatter(CommitIArgs a) {
    __shared__ int wc[MAX_WAVES][3];
    const int item = blockIdx.x;
    if (item >= *a.items.n_items || !commit_enabled(a.st)) return;
    const CommitPick pk = commit_pick(a);
    const int c = a.items.cell[item];
    const int beg = a.items.begin[item], end = a.items.begin[item + 1];
    const int M = a.M;
    Window1<P> w;
    load_window1<P>(w, c, a.ay, a.az, a.en, pk.ek);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    int run0 = a.base[item * 3 + 0], run1 = a.base[item * 3 + 1], run2 = a.base[item * 3 + 2];
    int flags = 0;
    for (int r0 = beg; r0 < end; r0 += blockDim.x) {
        const int i = r0 + threadIdx.x;
        const bool valid = i < end;
        int t = -1;
        double xin = 0.0, p1 = 0.0;
        int32_t pid = 0;
        if (valid) {
            const double xi0 = a.cur.xi[i];
            const double p0 = a.cur.p[i];
            const double d = pk.d[i];
            pid = a.cur.id[i];
            double t0 = xi0 - (double)c;
            if (!(t0 >= 0.0 && t0 < 1.0)) { flags |= FLAG_ORDER; t0 = 0.5; }
            double dn, dused, dr, lb[P + 2];
            particle_map<P>(w, t0, p0, d, false, c, xi0, a.dt, a.dt_dx, a.inv_dx, dn, p1, dused, lb, dr, flags);
            t = mover_type(xi0, d, c);
            xin = xi0 + d;
            if (xin >= (double)M) xin -= (double)M;
            else if (xin < 0.0) {
                xin += (double)M;
                if (xin >= (double)M) xin = __longlong_as_double(__double_as_longlong((double)M) - 1);
            }
        }
        const unsigned long long b0 = __ballot(t == 0), b1 = __ballot(t == 1), b2 = __ballot(t == 2);
        if (lane == 0) { wc[wid][0] = __popcll(b0); wc[wid][1] = __popcll(b1); wc[wid][2] = __popcll(b2); }
        __syncthreads();
        int pre0 = 0, pre1 = 0, pre2 = 0, s0 = 0, s1 = 0, s2 = 0;
        for (int q = 0; q < nw; ++q) {
            if (q < wid) { pre0 += wc[q][0]; pre1 += wc[q][1]; pre2 += wc[q][2]; }
            s0 += wc[q][0]; s1 += wc[q][1]; s2 += wc[q][2];
        }
        if (valid) {
            int dest;
            if (t == 0) dest = run0 + pre0 + __popcll(b0 & lt);
            else if (t == 1) dest = run1 + pre1 + __popcll(b1 & lt);
            else dest = run2 + pre2 + __popcll(b2 & lt);
            a.nxt.xi[dest] = xin;
            a.nxt.p[dest] = p1;
            a.nxt.id[dest] = pid;
        }
        run0 += s0; run1 += s1; run2 += s2;
        __syncthreads();
    }
    flags = wave_or(flags);
    if (lane == 0 && flags) atomicOr(&a.st->flags, flags);
}

__global__ void k_mark_committed(DevStatus *st) {
    if (st->converged && !st->committed && st->flags == 0 && st->gate) st->committed = 1;
}

__global__ void k_begin(DevStatus *st, const DevStatus *gate) {
    st->rx_bits = 0ull;
    st->re_bits = 0ull;
    st->k = 0;
    st->converged = 0;
    st->kconv = -1;
    st->committed = 0;
    st->flags = 0;
    st->counter = 0u;
    st->fp32_sweeps = 0;
    st->res = 0.0;
    st->gate = gate ? gate->committed : 1;   // 0: every kernel of the substep skips
}

// ---- launchers ------------------------------------------------------------
void launch_sweep_I(int P, bool seidel, int grid, int block, hipStream_t s, const SweepIArgs &a) {
#define ECPIC_SW(PP)                                                                              \
    case PP:                                                                                      \
        if (seidel) hipLaunchKernelGGL((k_sweep_I<PP, true>), dim3(grid), dim3(block), 0, s, a);  \
        else hipLaunchKernelGGL((k_sweep_I<PP, false>), dim3(grid), dim3(block), 0, s, a);        \
        break;
    switch (P) { ECPIC_SW(2) ECPIC_SW(3) ECPIC_SW(4) ECPIC_SW(5) }
#undef ECPIC_SW
}

void launch_field_I(int P, int grid, hipStream_t s, const FieldIArgs &a) {
    const size_t lds = sizeof(double) * (256 + a.ntaps);
#define ECPIC_F(PP) case PP: hipLaunchKernelGGL((k_field_I<PP>), dim3(grid), dim3(256), lds, s, a); break;
    switch (P) { ECPIC_F(2) ECPIC_F(3) ECPIC_F(4) ECPIC_F(5) }
#undef ECPIC_F
}

void launch_commit_I(int P, int grid, int block, hipStream_t s, const CommitIArgs &a) {
    hipLaunchKernelGGL(k_commit_count, dim3(grid), dim3(block), 0, s, a);
    hipLaunchKernelGGL(k_commit_scan, dim3(1), dim3(1024), 0, s, a);
#define ECPIC_C(PP) case PP: hipLaunchKernelGGL((k_commit_scatter<PP>), dim3(grid), dim3(block), 0, s, a); break;
    switch (P) { ECPIC_C(2) ECPIC_C(3) ECPIC_C(4) ECPIC_C(5) }
#undef ECPIC_C
    hipLaunchKernelGGL(k_mark_committed, dim3(1), dim3(1), 0, s, a.st);
}

void launch_begin(DevStatus *st, const DevStatus *gate, hipStream_t s) {
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(1), 0, s, st, gate);
}

void launch_mark(DevStatus *st, hipStream_t s) { hipLaunchKernelGGL(k_mark_committed, dim3(1), dim3(1), 0, s, st); }

}  // namespace ecpic
