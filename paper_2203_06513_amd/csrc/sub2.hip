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
// block.  Within a full step the deposit of iterate 0 is formed by the
// Subsystem I commit (sub1.hip), which holds the new positions and momenta,
// and the first field kernel reads it (WIDE); the particle kernel then runs
// from iterate 1 on.
#include <cstddef>

#include "coef.hpp"

namespace ecpic {

__device__ __forceinline__ bool prev_converged2(DevStatus *st, int k, double tol, bool writer,
                                                unsigned long long reb) {
    if (k <= 0) return false;
    const double r = dbits(reb);
    if (writer && k - 1 < MAX_HIST) st->res_hist[k - 1] = r;
    if (r <= tol) {
        if (writer) { st->kconv = k - 1; st->res = r; }
        return true;
    }
    return false;
}

constexpr int SUB2_BATCH = 4;

// The particle pass.  Each wave takes every nw-th row of 64 particles of the
// item and keeps the loads of its next two rows in flight while it computes
// the current one (a row here is short work, shorter than a memory round
// trip); it writes its own 2 (P+1) partial slots (V0 slot q <-> index
// c - P + q, y then z).
template <int P>
__device__ __forceinline__ void sweep_II_item(const SweepIIArgs &a, int item) {
    constexpr int NA = RecA<P>::N;
    DevStatus *st = a.st;
    const int k = a.k;
    // item count, status words and item description in one memory round trip
    const int n_items = *a.items.n_items;
    const int sgate = st->gate, sflags = st->flags, skconv = st->kconv;
    const unsigned long long reb = st->re_bits[(k - 1) & 1];
    const int c = a.items.cell[item];
    const int beg = a.items.begin[item], end = a.items.begin[item + 1];
    asm volatile("" ::"s"(n_items), "s"(sgate), "s"(sflags), "s"(skconv), "s"(reb), "s"(c), "s"(beg), "s"(end));
    if (item >= n_items) return;
    if (!sgate | sflags | (skconv >= 0)) return;
    if (prev_converged2(st, k, a.tol, threadIdx.x == 0, reb)) return;
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
    const int stride = nw * WAVE;
    const int last = end - 1;   // items are never empty; loads past the run re-read it
    const int first = beg + wid * WAVE;
    // rows are taken in batches of SUB2_BATCH: the loads of the next batch are
    // issued before the current one is computed, so every memory round trip
    // has a whole batch of arithmetic to hide behind
    double xn[SUB2_BATCH], pn[SUB2_BATCH];
#pragma unroll
    for (int b = 0; b < SUB2_BATCH; ++b) {
        const int il = min(first + b * stride + lane, last);
        xn[b] = a.xi[il];
        pn[b] = a.p[il];
    }
    const double *rn = a.coefAn + (size_t)rec_index(c) * NA;
    const double *rk = ((k & 1) ? a.coefAk1 : a.coefAk0) + (size_t)rec_index(c) * NA;
    double cn[NA], ck[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) { cn[i] = rn[i]; ck[i] = rk[i]; }
    double my[P + 1], mz[P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i) { my[i] = 0.0; mz[i] = 0.0; }
    int flags = 0;
    // everything loaded so far completes here, so the loop's waits only
    // concern its own loads
    __builtin_amdgcn_s_waitcnt(0);
    for (int row = first; row < end; row += SUB2_BATCH * stride) {
        double xc[SUB2_BATCH], pc[SUB2_BATCH];
#pragma unroll
        for (int b = 0; b < SUB2_BATCH; ++b) {
            xc[b] = xn[b];
            pc[b] = pn[b];
        }
#pragma unroll
        for (int b = 0; b < SUB2_BATCH; ++b) {
            const int il = min(row + (SUB2_BATCH + b) * stride + lane, last);
            xn[b] = a.xi[il];
            pn[b] = a.p[il];
        }
        __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the arithmetic
#pragma unroll
        for (int b = 0; b < SUB2_BATCH; ++b) {
            const bool valid = row + b * stride + lane < end;
            double t = xc[b] - (double)c;
            wave_flag(flags, !(t >= 0.0), FLAG_ORDER);
            wave_flag(flags, !(t < 1.0), FLAG_ORDER);
            t = fmin(fmax(t, 0.0), 1.0);
            double cy, cz;
            sub2_coef<P>(cn, cn + P + 1, ck, ck + P + 1, t, pc[b], cy, cz);
            const double wv = valid ? 1.0 : 0.0;
            cy *= wv;
            cz *= wv;
            double tp = 1.0;
#pragma unroll
            for (int j = 0; j <= P; ++j) {
                my[j] = fma(cy, tp, my[j]);
                mz[j] = fma(cz, tp, mz[j]);
                tp *= t;
            }
        }
    }
    // wave sums of the moments, then lane q < 2 (P+1) forms slot q
    double ty[P + 1], tz[P + 1];
#pragma unroll
    for (int j = 0; j <= P; ++j) {
        ty[j] = wave_sum_dpp(my[j]);
        tz[j] = wave_sum_dpp(mz[j]);
    }
    constexpr Pieces<P> Bp{};
    const int comp = lane / (P + 1), slot = lane % (P + 1), m = P - slot;
    double out = 0.0;
#pragma unroll
    for (int j = 0; j <= P; ++j) out += Bp.c[m < 0 ? 0 : m][j] * (comp == 0 ? ty[j] : tz[j]);
    if (lane < 2 * (P + 1)) a.part[((size_t)item * nw + wid) * 2 * (P + 1) + lane] = out;
    if (flags && lane == 0) atomicOr(&st->flags, flags);   // flags is wave-uniform (wave_flag)
}

// One block per work item; the grid may exceed the item count (the count of a
// step enqueued ahead is only known on the device) and the extra blocks exit.
template <int P>
__global__ void __launch_bounds__(MAX_BLOCK) k_sweep_II(SweepIIArgs a) {
    sweep_II_item<P>(a, blockIdx.x);
}

// Field iterate k+1 of Subsystem II and the A-records of a^(k+1).  Block b
// computes e^(k+1) on the FIELD2_OUT cells from b * TILE - P (the first P only
// to form the records of cells b * TILE .. b * TILE + TILE - 1).  The item
// partials are summed per cell into LDS, the two deposits assembled, and the
// inverse of (M0^ + r^2 K^) applied as a convolution by four lanes per output
// (every fourth tap each, combined in a fixed order).  WIDE: iterate 0 from
// the partials the Subsystem I commit formed (items of the order before the
// commit; a cell's partial spans V0 indices c-P-1 .. c+1, P+3 per component).
constexpr int FIELD2_OUT = 64;

// Sum over the WPI wave partials of cell c when item c is cell c, all loads
// issued before any is used.
template <int NS, int WPI>
__device__ __forceinline__ void cell_partials_one2(const double *part, int c, double (&v)[NS]) {
    double u[WPI][NS];
#pragma unroll
    for (int w = 0; w < WPI; ++w)
#pragma unroll
        for (int q = 0; q < NS; ++q) u[w][q] = part[((size_t)c * WPI + w) * NS + q];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        v[q] = 0.0;
#pragma unroll
        for (int w = 0; w < WPI; ++w) v[q] += u[w][q];
    }
}

template <int NS>
__device__ __forceinline__ void cell_partials_one2(const double *part, int c, int wpi, double (&v)[NS]) {
    switch (wpi) {
        case 1: cell_partials_one2<NS, 1>(part, c, v); break;
        case 2: cell_partials_one2<NS, 2>(part, c, v); break;
        case 3: cell_partials_one2<NS, 3>(part, c, v); break;
        default: cell_partials_one2<NS, 4>(part, c, v); break;
    }
}

template <int P, bool WIDE>
__global__ void __launch_bounds__(256) k_field_II(FieldIIArgs a) {
    extern __shared__ double smem[];
    __shared__ double ldsm[MAX_WAVES];
    __shared__ int ldsf[MAX_WAVES];
    constexpr int RL = WIDE ? 1 : 0;           // cells a partial reaches to the right of its V0 range
    constexpr int NC = P + 1 + 2 * RL;         // slots per component
    constexpr int NA = RecA<P>::N, NS = 2 * NC;
    constexpr int TILE = FIELD2_OUT - P;
    DevStatus *st = a.st;
    // the status is tested once the loads that do not depend on it are issued
    const int sgate = st->gate, sflags = st->flags, skconv = st->kconv;
    const bool one_each = a.items.n_items[1] != 0;   // item c is cell c
    const int k = a.k;
    const int M = a.M;
    const int j0 = blockIdx.x * TILE - P;
    const int mhi = a.mlo + a.ntaps - 1;
    const int slen = FIELD2_OUT + a.ntaps - 1;   // b on cells [j0 - mhi, j0 - mhi + slen)
    const int clo = j0 - mhi - RL;               // b_j needs the partials of cells j-RL .. j+P+RL
    const int clen = slen + P + 2 * RL;
    double *cp = smem;
    double *Sy = cp + (size_t)clen * NS;
    double *Sz = Sy + slen;
    double *tp = Sz + slen;
    double *eyl = tp + a.ntaps;
    double *ezl = eyl + FIELD2_OUT;
    double *bay = ezl + FIELD2_OUT;   // a^n - dt/2 e^n on the block's cells (the part of a^(k+1) known now)
    double *baz = bay + FIELD2_OUT;
    const double *eyk = k == 0 ? a.eyn : ((k & 1) ? a.ey1 : a.ey0);
    const double *ezk = k == 0 ? a.ezn : ((k & 1) ? a.ez1 : a.ez0);
    // One memory round trip before the status test: this quad's output cell,
    // the first taps, a^n and e^n on the block's cells and the first round of
    // partials, loaded as if item c were cell c (in bounds whatever the list
    // holds) and kept if it is (a list with several items per cell is followed
    // only after the test).  The empty asm keeps the loads above the branch.
    const int quad = threadIdx.x >> 2, ql = threadIdx.x & 3;
    const int jq = j0 + quad, jqm = imod(jq, M);
    const int t0 = threadIdx.x;
    const double E0y_q = a.E0y[jqm], E0z_q = a.E0z[jqm];
    const double eyk_q = eyk[jqm + HALO], ezk_q = ezk[jqm + HALO];
    const double tap0 = a.taps[min(t0, a.ntaps - 1)];
    const int jm0 = imod(j0 + min(t0, FIELD2_OUT - 1), M) + HALO;
    const double ay0 = a.ayn[jm0], ey0 = a.eyn[jm0], az0 = a.azn[jm0], ez0 = a.ezn[jm0];
    double v0[NS];
    cell_partials_one2<NS>(a.part, imod(clo + min(t0, clen - 1), M), a.wpi, v0);
    asm volatile("" ::"v"(E0y_q), "v"(E0z_q), "v"(eyk_q), "v"(ezk_q), "v"(tap0));
    asm volatile("" ::"v"(ay0), "v"(ey0), "v"(az0), "v"(ez0));
#pragma unroll
    for (int q = 0; q < NS; ++q) asm volatile("" ::"v"(v0[q]));
    if (!sgate | sflags | (skconv >= 0)) return;
    if (t0 < a.ntaps) tp[t0] = tap0;
    for (int t = t0 + blockDim.x; t < a.ntaps; t += blockDim.x) tp[t] = a.taps[t];
    if (t0 < FIELD2_OUT) {
        bay[t0] = ay0 - a.half_dt * ey0;
        baz[t0] = az0 - a.half_dt * ez0;
    }
    for (int t = threadIdx.x; t < clen; t += blockDim.x) {
        const int c = imod(clo + t, M);
        double v[NS];
        if (one_each && t == t0) {
#pragma unroll
            for (int q = 0; q < NS; ++q) cp[q * clen + t] = v0[q];
            continue;
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) v[q] = 0.0;
        const int u0 = (one_each ? c : a.items.cell_first[c]) * a.wpi;
        const int u1 = one_each ? u0 + a.wpi : a.items.cell_first[c + 1] * a.wpi;
        for (int u = u0; u < u1; ++u) {   // the wave partials of the cell's items
#pragma unroll
            for (int q = 0; q < NS; ++q) v[q] += a.part[(size_t)u * NS + q];
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) cp[q * clen + t] = v[q];   // slot-major: consecutive cells, banks
    }
    __syncthreads();
    for (int t = threadIdx.x; t < slen; t += blockDim.x) {
        double sy = 0.0, sz = 0.0;
#pragma unroll
        for (int r = 0; r <= P + 2 * RL; ++r) {   // cell j - RL + r: slot P + 2 RL - r
            sy += cp[(P + 2 * RL - r) * clen + t + r];
            sz += cp[(NC + P + 2 * RL - r) * clen + t + r];
        }
        Sy[t] = sy;
        Sz[t] = sz;
    }
    __syncthreads();
    double *eyo = (k & 1) ? a.ey0 : a.ey1;
    double *ezo = (k & 1) ? a.ez0 : a.ez1;
    double *Aout = ((k + 1) & 1) ? a.coefAk1 : a.coefAk0;
    double re = 0.0;
    int flags = 0;
    {
        const double *Syq = Sy + quad + a.ntaps - 1, *Szq = Sz + quad + a.ntaps - 1;
        double cy = 0.0, cz = 0.0, cy1 = 0.0, cz1 = 0.0, cy2 = 0.0, cz2 = 0.0, cy3 = 0.0, cz3 = 0.0;
        int i = ql;
        for (; i + 12 < a.ntaps; i += 16) {   // four chains per component
            cy = fma(tp[i], Syq[-i], cy);
            cz = fma(tp[i], Szq[-i], cz);
            cy1 = fma(tp[i + 4], Syq[-i - 4], cy1);
            cz1 = fma(tp[i + 4], Szq[-i - 4], cz1);
            cy2 = fma(tp[i + 8], Syq[-i - 8], cy2);
            cz2 = fma(tp[i + 8], Szq[-i - 8], cz2);
            cy3 = fma(tp[i + 12], Syq[-i - 12], cy3);
            cz3 = fma(tp[i + 12], Szq[-i - 12], cz3);
        }
        for (; i < a.ntaps; i += 4) {
            cy = fma(tp[i], Syq[-i], cy);
            cz = fma(tp[i], Szq[-i], cz);
        }
        cy = (cy + cy1) + (cy2 + cy3);
        cz = (cz + cz1) + (cz2 + cz3);
        cy += dpp_d<0xB1>(cy);
        cz += dpp_d<0xB1>(cz);
        cy += dpp_d<0x4E>(cy);
        cz += dpp_d<0x4E>(cz);
        const double ny = E0y_q + a.coef * cy;
        const double nz = E0z_q + a.coef * cz;
        if (ql == 0) {
            eyl[quad] = ny;
            ezl[quad] = nz;
            if (quad >= P && jq < M) {
                store_padded(eyo, M, jqm, ny);
                store_padded(ezo, M, jqm, nz);
                re = fmax(fabs(ny - eyk_q), fabs(nz - ezk_q));
                if (!(fabs(ny) < 1.0e300) || !(fabs(nz) < 1.0e300)) flags |= FLAG_NONFINITE;
            }
        }
    }
    __syncthreads();
    {
        const int q = threadIdx.x + P;
        const int j = j0 + q;
        if (q < FIELD2_OUT && j < M) {
            constexpr Pieces<P> B{};
            for (int i = 0; i <= P; ++i) {
                double sy = 0.0, sz = 0.0;
                for (int m = 0; m <= P; ++m) {
                    const int u = j - m - j0;
                    const double ay = bay[u] - a.half_dt * eyl[u];
                    const double az = baz[u] - a.half_dt * ezl[u];
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

// The step-start work of one block from its window in LDS (a^n, e^n on cells
// wlo .., e_x^n on cells j0 - P ..): the A-records of a^n and of
// a^(0) = a^n - dt e^n, the E-records of e_x^n, and with do_II the stencil
// R = (M0 - r^2 K) e^n + ck K a^n and E0 = (M0 + r^2 K)^{-1} R on the block's
// cells.  Every thread of the block calls it.
struct StepStart {
    double *coefA, *coefE0, *coefAk0, *E0y, *E0z;
    Stencil m0, kk;
    double dt, r2, ck;
    int do_II, ntaps, mlo, M;
};

template <int P>
__device__ __forceinline__ void step_start_body(const StepStart &a, int j0, int wlo, int len, const double *Way,
                                                const double *Waz, const double *Wey, const double *Wez,
                                                const double *Wex, const double *tp, double *Ry, double *Rz) {
    const int t = threadIdx.x, M = a.M, ntaps = a.ntaps;
    if (a.do_II) {
        for (int idx = t; idx < len; idx += blockDim.x) {
            double sy = 0.0, sz = 0.0;
#pragma unroll
            for (int q = -P; q <= P; ++q) {
                const double cm = a.m0.v[q + P] - a.r2 * a.kk.v[q + P];
                const double ka = a.ck * a.kk.v[q + P];
                const int u = idx + P + q;
                sy += cm * Wey[u] + ka * Way[u];
                sz += cm * Wez[u] + ka * Waz[u];
            }
            Ry[idx] = sy;
            Rz[idx] = sz;
        }
    }
    {
        const int c = j0 + t;
        if (t < FIELD2_OUT && c < M) {
            constexpr Pieces<P> B{};
            constexpr int NA = RecA<P>::N;
            const int u0 = c - wlo;   // window index of cell c
#pragma unroll
            for (int i = 0; i <= P; ++i) {
                double ny = 0.0, nz = 0.0, ky = 0.0, kz = 0.0;
#pragma unroll
                for (int m = 0; m <= P; ++m) {
                    const int u = u0 - m;
                    ny += Way[u] * B.c[m][i];
                    nz += Waz[u] * B.c[m][i];
                    ky += (Way[u] - a.dt * Wey[u]) * B.c[m][i];
                    kz += (Waz[u] - a.dt * Wez[u]) * B.c[m][i];
                }
                store_record(a.coefA, M, c, NA, i, ny);
                store_record(a.coefA, M, c, NA, P + 1 + i, nz);
                if (a.do_II) {
                    store_record(a.coefAk0, M, c, NA, i, ky);
                    store_record(a.coefAk0, M, c, NA, P + 1 + i, kz);
                }
            }
            if (a.coefE0) {
                double r[P];
                make_recE<P>([&](int jj) { return Wex[jj - (j0 - P)]; }, c, r);
                for (int i = 0; i < P; ++i) store_record(a.coefE0, M, c, RecE<P>::N, i, r[i]);
            }
        }
    }
    if (!a.do_II) return;
    __syncthreads();
    const int quad = t >> 2, ql = t & 3;
    const double *Ryq = Ry + quad + ntaps - 1, *Rzq = Rz + quad + ntaps - 1;
    double cy = 0.0, cz = 0.0, cy1 = 0.0, cz1 = 0.0;
    int i = ql;
    for (; i + 4 < ntaps; i += 8) {   // two chains per component
        cy = fma(tp[i], Ryq[-i], cy);
        cz = fma(tp[i], Rzq[-i], cz);
        cy1 = fma(tp[i + 4], Ryq[-i - 4], cy1);
        cz1 = fma(tp[i + 4], Rzq[-i - 4], cz1);
    }
    if (i < ntaps) {
        cy = fma(tp[i], Ryq[-i], cy);
        cz = fma(tp[i], Rzq[-i], cz);
    }
    cy += cy1;
    cz += cz1;
    cy += dpp_d<0xB1>(cy);
    cz += dpp_d<0xB1>(cz);
    cy += dpp_d<0x4E>(cy);
    cz += dpp_d<0x4E>(cz);
    const int j = j0 + quad;
    if (ql == 0 && j < M) {
        a.E0y[j] = cy;
        a.E0z[j] = cz;
    }
}

// LDS of a step start: Ry, Rz [len], taps [ntaps], the window of a_y, a_z,
// e_y, e_z [len + 2 P] each and e_x on cells j0 - P .. j0 + FIELD2_OUT - 1.
__host__ __device__ constexpr size_t step_start_lds(int P, int ntaps) {
    return sizeof(double) * (2 * (size_t)(FIELD2_OUT + ntaps - 1) + (size_t)ntaps +
                             4 * (size_t)(FIELD2_OUT + ntaps - 1 + 2 * P) + FIELD2_OUT + P);
}

// Start of a step (or of one substep).  Block 0 resets the statuses it is
// given (stI for Subsystem I, gated on gate_src, the Subsystem II status of the
// step before when it was enqueued ahead; stII for a Subsystem II run on its
// own; in a full step the Subsystem I commit resets stII).  A gated-off step
// writes nothing else.  Block b, on cells
// b * FIELD2_OUT .. + FIELD2_OUT - 1, writes the A-records of a^n (shared by
// both substeps, Subsystem I leaves a_perp alone), with do_I the E-records of
// e_x^n, and with do_II the A-records of a^(0) = a^n - dt e^n (the iterate for
// e^(0) = e^n) and the constant part of every Subsystem II iterate,
//   E0 = A^-1 [(M0^ - r^2 K^) e^n + (dt/dx^2) K^ a^n],   A = M0^ + r^2 K^,
// with the stencils applied on a window in LDS and A^-1 as a convolution by
// four lanes per output.
template <int P>
__global__ void __launch_bounds__(256) k_begin_step(DevStatus *stI, const DevStatus *gate_src, DevStatus *stII,
                                                    const double *ayn, const double *azn, const double *eyn,
                                                    const double *ezn, const double *exn, const double *taps,
                                                    StepStart a) {
    extern __shared__ double R[];
    // a step enqueued behind another runs only if that one committed
    const bool go = gate_src ? (gate_src->committed && gate_src->flags == 0) : true;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (stI) init_status(stI, gate_src);
        if (stII) init_status(stII, nullptr);
    }
    const int M = a.M, ntaps = a.ntaps;
    const int j0 = blockIdx.x * FIELD2_OUT;
    const int mhi = a.mlo + ntaps - 1;
    const int len = FIELD2_OUT + ntaps - 1;   // R on cells j0 - mhi .. j0 - mhi + len - 1
    const int wlo = j0 - mhi - P;             // the window: every cell the stencil and the records read
    const int wlen = len + 2 * P;
    constexpr int XL = FIELD2_OUT + P;
    double *Ry = R, *Rz = R + len, *tp = Rz + len;
    double *Way = tp + ntaps, *Waz = Way + wlen, *Wey = Waz + wlen, *Wez = Wey + wlen, *Wex = Wez + wlen;
    // one memory round trip: the first round of the window, taps and e_x (none
    // of it depends on the gate; nothing is written before it)
    const int t = threadIdx.x;
    const int jw = imod(wlo + min(t, wlen - 1), M) + HALO;
    const double w_ay = ayn[jw], w_az = azn[jw], w_ey = eyn[jw], w_ez = ezn[jw];
    const double w_tp = ntaps > 0 ? taps[min(t, ntaps - 1)] : 0.0;
    const double w_ex = exn ? exn[imod(j0 - P + min(t, XL - 1), M) + HALO] : 0.0;
    asm volatile("" ::"v"(w_ay), "v"(w_az), "v"(w_ey), "v"(w_ez), "v"(w_tp), "v"(w_ex));
    if (!go) return;
    if (t < wlen) { Way[t] = w_ay; Waz[t] = w_az; Wey[t] = w_ey; Wez[t] = w_ez; }
    for (int idx = t + blockDim.x; idx < wlen; idx += blockDim.x) {
        const int j = imod(wlo + idx, M) + HALO;
        Way[idx] = ayn[j]; Waz[idx] = azn[j]; Wey[idx] = eyn[j]; Wez[idx] = ezn[j];
    }
    if (t < ntaps) tp[t] = w_tp;
    for (int idx = t + blockDim.x; idx < ntaps; idx += blockDim.x) tp[idx] = taps[idx];
    if (t < XL) Wex[t] = w_ex;
    __syncthreads();
    step_start_body<P>(a, j0, wlo, len, Way, Waz, Wey, Wez, Wex, tp, Ry, Rz);
}

// The Subsystem II commit of one step joined to the start of the next (steps
// enqueued back to back).  Every block settles the convergence test of step n
// on its own (same answer); block 0 records it, mirrors both statuses of step
// n to the host and resets the Subsystem I status of step n+1, gated on the
// commit.  Each block forms the committed e_perp^{n+1} = e^(kc+1) and
// a^{n+1} = a^n - dt/2 (e^n + e^{n+1}) on its whole window from the iterates
// (one memory round trip, both parity candidates loaded), writes them on its
// own cells, and does the step-start work of step n+1 from that window.
struct JoinArgs {
    DevStatus *st;                         // Subsystem II status of step n
    const DevStatus *stI;                  // Subsystem I status of step n (mirrored)
    DevStatus *mirror;                     // host mirror of step n's statuses, or null
    DevStatus *stI_next;                   // Subsystem I status of step n+1
    const double *eyn, *ezn, *ayn, *azn;   // fields of step n
    const double *ey0, *ey1, *ez0, *ez1;   // Subsystem II iterates, by parity
    double *ey_next, *ez_next, *ay_next, *az_next;
    const double *exn;                     // e_x^{n+1} (Subsystem I commit of step n)
    const double *taps;
    double half_dt, tol;
    int nsweeps;
};

template <int P>
__global__ void __launch_bounds__(256) k_step_join(JoinArgs g, StepStart a) {
    extern __shared__ double R[];
    DevStatus *st = g.st;
    const int sgate = st->gate, sflags = st->flags, skconv = st->kconv;
    const unsigned long long reb = st->re_bits[(g.nsweeps - 1) & 1];
    asm volatile("" ::"s"(sgate), "s"(sflags), "s"(skconv), "s"(reb));
    const int M = a.M, ntaps = a.ntaps;
    const int j0 = blockIdx.x * FIELD2_OUT;
    const int mhi = a.mlo + ntaps - 1;
    const int len = FIELD2_OUT + ntaps - 1;
    const int wlo = j0 - mhi - P;
    const int wlen = len + 2 * P;
    constexpr int XL = FIELD2_OUT + P;
    double *Ry = R, *Rz = R + len, *tp = Rz + len;
    double *Way = tp + ntaps, *Waz = Way + wlen, *Wey = Waz + wlen, *Wez = Wey + wlen, *Wex = Wez + wlen;
    const int t = threadIdx.x;
    const int jw = imod(wlo + min(t, wlen - 1), M) + HALO;
    const double w_ay = g.ayn[jw], w_az = g.azn[jw], w_ey = g.eyn[jw], w_ez = g.ezn[jw];
    const double w_y0 = g.ey0[jw], w_y1 = g.ey1[jw], w_z0 = g.ez0[jw], w_z1 = g.ez1[jw];
    const double w_tp = ntaps > 0 ? g.taps[min(t, ntaps - 1)] : 0.0;
    const double w_ex = g.exn[imod(j0 - P + min(t, XL - 1), M) + HALO];
    asm volatile("" ::"v"(w_ay), "v"(w_az), "v"(w_ey), "v"(w_ez), "v"(w_tp), "v"(w_ex));
    asm volatile("" ::"v"(w_y0), "v"(w_y1), "v"(w_z0), "v"(w_z1));
    int kc = -1;
    if (sgate && !sflags) {
        kc = skconv;
        if (kc < 0 && prev_converged2(st, g.nsweeps, g.tol, blockIdx.x == 0 && t == 0, reb)) kc = g.nsweeps - 1;
    }
    if (blockIdx.x == 0) {
        if (t == 0 && kc >= 0) st->committed = 1;
        if (g.mirror) {   // the words before the residual history of both statuses
            __syncthreads();
            constexpr int W = (int)(offsetof(DevStatus, res_hist) / sizeof(int32_t));
            if (t < 2 * W) {
                const int32_t *src = reinterpret_cast<const int32_t *>(t < W ? g.stI : st);
                int32_t *dst = reinterpret_cast<int32_t *>(g.mirror + (t < W ? 0 : 1));
                dst[t % W] = src[t % W];
            }
        }
        if (t == 0) init_status(g.stI_next, st);
    }
    if (kc < 0) return;
    const bool odd = ((kc + 1) & 1) != 0;
    auto commit_cell = [&](int idx, double ay, double az, double ey, double ez, double y0, double y1, double z0,
                           double z1) {
        const double ny = odd ? y1 : y0, nz = odd ? z1 : z0;
        const double na_y = fma(-g.half_dt, ey + ny, ay), na_z = fma(-g.half_dt, ez + nz, az);
        Way[idx] = na_y; Waz[idx] = na_z; Wey[idx] = ny; Wez[idx] = nz;
        const int q = idx - (mhi + P);   // own cell j0 + q
        if (q >= 0 && q < FIELD2_OUT && j0 + q < M) {
            store_padded(g.ey_next, M, j0 + q, ny);
            store_padded(g.ez_next, M, j0 + q, nz);
            store_padded(g.ay_next, M, j0 + q, na_y);
            store_padded(g.az_next, M, j0 + q, na_z);
        }
    };
    if (t < wlen) commit_cell(t, w_ay, w_az, w_ey, w_ez, w_y0, w_y1, w_z0, w_z1);
    for (int idx = t + blockDim.x; idx < wlen; idx += blockDim.x) {
        const int j = imod(wlo + idx, M) + HALO;
        commit_cell(idx, g.ayn[j], g.azn[j], g.eyn[j], g.ezn[j], g.ey0[j], g.ey1[j], g.ez0[j], g.ez1[j]);
    }
    if (t < ntaps) tp[t] = w_tp;
    for (int idx = t + blockDim.x; idx < ntaps; idx += blockDim.x) tp[idx] = g.taps[idx];
    if (t < XL) Wex[t] = w_ex;
    __syncthreads();
    step_start_body<P>(a, j0, wlo, len, Way, Waz, Wey, Wez, Wex, tp, Ry, Rz);
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

// Commit of Subsystem II: e_perp^{n+1} = e^(kc+1), a^{n+1} = a^n - dt/2 (e^n + e^{n+1}).
// Every block settles the convergence test on its own (same answer); block 0
// records the commit.  Running it again is harmless (same writes).
__global__ void __launch_bounds__(256) k_commit_II(DevStatus *st, const DevStatus *stI, DevStatus *mirror,
                                                   const double *eyn, const double *ezn, const double *ayn,
                                                   const double *azn, const double *ey0, const double *ey1,
                                                   const double *ez0, const double *ez1, double *ey_next,
                                                   double *ez_next, double *ay_next, double *az_next, double half_dt,
                                                   int M, int nsweeps, double tol) {
    // one memory round trip: the status words, the last residual and this
    // cell's fields, with both candidates for e^(kc+1) (which one depends only
    // on the parity of kc)
    const int sgate = st->gate, sflags = st->flags, skconv = st->kconv;
    const unsigned long long reb = st->re_bits[(nsweeps - 1) & 1];
    asm volatile("" ::"s"(sgate), "s"(sflags), "s"(skconv), "s"(reb));
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int jj = min(j, M - 1) + HALO;
    const double y0 = ey0[jj], y1 = ey1[jj], z0 = ez0[jj], z1 = ez1[jj];
    const double ay = ayn[jj], az = azn[jj], ey = eyn[jj], ez = ezn[jj];
    int kc = -1;
    if (sgate && !sflags) {
        kc = skconv;
        if (kc < 0 && prev_converged2(st, nsweeps, tol, blockIdx.x == 0 && threadIdx.x == 0, reb)) kc = nsweeps - 1;
    }
    if (kc >= 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->committed = 1;
        if (j < M) {
            const bool odd = ((kc + 1) & 1) != 0;
            const double ny = odd ? y1 : y0, nz = odd ? z1 : z0;
            store_padded(ey_next, M, j, ny);
            store_padded(ez_next, M, j, nz);
            store_padded(ay_next, M, j, fma(-half_dt, ey + ny, ay));
            store_padded(az_next, M, j, fma(-half_dt, ez + nz, az));
        }
    }
    if (mirror && blockIdx.x == 0) {
        // the host's copy of both statuses (the words before the residual
        // history), written straight into its pinned mirror
        __syncthreads();
        constexpr int W = (int)(offsetof(DevStatus, res_hist) / sizeof(int32_t));
        const int t = threadIdx.x;
        if (t < 2 * W) {
            const int32_t *src = reinterpret_cast<const int32_t *>(t < W ? stI : st);
            int32_t *dst = reinterpret_cast<int32_t *>(mirror + (t < W ? 0 : 1));
            dst[t % W] = src[t % W];
        }
    }
}

void launch_sweep_II(int P, int grid, int block, hipStream_t s, const SweepIIArgs &a) {
#define ECPIC_S2(PP) case PP: launch_k((k_sweep_II<PP>), dim3(grid), dim3(block), 0, s, a); break;
    switch (P) { ECPIC_S2(2) ECPIC_S2(3) ECPIC_S2(4) ECPIC_S2(5) }
#undef ECPIC_S2
}

void launch_field_II(int P, int M, hipStream_t s, const FieldIIArgs &a) {
    const int grid = (M + FIELD2_OUT - P - 1) / (FIELD2_OUT - P);
    const int slen = FIELD2_OUT + a.ntaps - 1;
    const int rl = a.wide ? 1 : 0;
    const size_t lds =
        sizeof(double) * ((size_t)(slen + P + 2 * rl) * 2 * (P + 1 + 2 * rl) + 2 * slen + a.ntaps + 4 * FIELD2_OUT);
#define ECPIC_F2(PP)                                                                          \
    case PP:                                                                                  \
        if (a.wide) launch_k((k_field_II<PP, true>), dim3(grid), dim3(256), lds, s, a);       \
        else launch_k((k_field_II<PP, false>), dim3(grid), dim3(256), lds, s, a);             \
        break;
    switch (P) { ECPIC_F2(2) ECPIC_F2(3) ECPIC_F2(4) ECPIC_F2(5) }
#undef ECPIC_F2
}

void launch_begin_step(int P, hipStream_t s, DevStatus *stI, const DevStatus *gate_src, DevStatus *stII,
                       const double *ayn, const double *azn,
                       const double *eyn, const double *ezn, const double *exn, double dt, double *coefA,
                       double *coefE0, double *coefAk0, int do_II, const double *m0, const double *kr, double r2,
                       double ck, const double *taps, int ntaps, int mlo, int M, double *E0y, double *E0z) {
    StepStart a{};
    a.coefA = coefA; a.coefE0 = coefE0; a.coefAk0 = coefAk0; a.E0y = E0y; a.E0z = E0z;
    a.m0.half = P; a.kk.half = P;
    for (int q = 0; q <= 2 * P; ++q) { a.m0.v[q] = m0[q]; a.kk.v[q] = kr[q]; }
    a.dt = dt; a.r2 = r2; a.ck = ck; a.do_II = do_II; a.ntaps = ntaps; a.mlo = mlo; a.M = M;
    const int grid = (M + FIELD2_OUT - 1) / FIELD2_OUT;
    const size_t lds = step_start_lds(P, ntaps);
#define ECPIC_B2(PP)                                                                                          \
    case PP:                                                                                                  \
        launch_k((k_begin_step<PP>), dim3(grid), dim3(256), lds, s, stI, gate_src, stII, ayn, azn, eyn, ezn, \
                 exn, taps, a);                                                                               \
        break;
    switch (P) { ECPIC_B2(2) ECPIC_B2(3) ECPIC_B2(4) ECPIC_B2(5) }
#undef ECPIC_B2
}

void launch_step_join(int P, hipStream_t s, DevStatus *st, const DevStatus *stI, DevStatus *mirror,
                      DevStatus *stI_next, const double *eyn, const double *ezn, const double *ayn, const double *azn,
                      const double *ey0, const double *ey1, const double *ez0, const double *ez1, double *ey_next,
                      double *ez_next, double *ay_next, double *az_next, int nsweeps, double tol,
                      const double *exn_next, double dt, double *coefA, double *coefE0, double *coefAk0,
                      const double *m0, const double *kr, double r2, double ck, const double *taps, int ntaps,
                      int mlo, int M, double *E0y, double *E0z) {
    JoinArgs g{st, stI, mirror, stI_next, eyn, ezn, ayn, azn, ey0, ey1, ez0, ez1, ey_next, ez_next, ay_next,
               az_next, exn_next, taps, 0.5 * dt, tol, nsweeps};
    StepStart a{};
    a.coefA = coefA; a.coefE0 = coefE0; a.coefAk0 = coefAk0; a.E0y = E0y; a.E0z = E0z;
    a.m0.half = P; a.kk.half = P;
    for (int q = 0; q <= 2 * P; ++q) { a.m0.v[q] = m0[q]; a.kk.v[q] = kr[q]; }
    a.dt = dt; a.r2 = r2; a.ck = ck; a.do_II = 1; a.ntaps = ntaps; a.mlo = mlo; a.M = M;
    const int grid = (M + FIELD2_OUT - 1) / FIELD2_OUT;
    const size_t lds = step_start_lds(P, ntaps);
#define ECPIC_J(PP) case PP: launch_k((k_step_join<PP>), dim3(grid), dim3(256), lds, s, g, a); break;
    switch (P) { ECPIC_J(2) ECPIC_J(3) ECPIC_J(4) ECPIC_J(5) }
#undef ECPIC_J
}

void launch_conv(int grid, hipStream_t s, const double *in, double *out, const double *taps, int ntaps, int mlo,
                 double alpha, int M) {
    launch_k(k_conv, dim3(grid), dim3(256), 0, s, in, out, taps, ntaps, mlo, alpha, M);
}

void launch_commit_II(int grid, hipStream_t s, DevStatus *st, const DevStatus *stI, DevStatus *mirror,
                      const double *eyn, const double *ezn, const double *ayn, const double *azn, const double *ey0,
                      const double *ey1, const double *ez0, const double *ez1, double *ey_next, double *ez_next,
                      double *ay_next, double *az_next, double half_dt, int M, int nsweeps, double tol) {
    launch_k(k_commit_II, dim3(grid), dim3(256), 0, s, st, stI, mirror, eyn, ezn, ayn, azn, ey0, ey1, ez0,
                       ez1, ey_next, ez_next, ay_next, az_next, half_dt, M, nsweeps, tol);
}

}  // namespace ecpic
