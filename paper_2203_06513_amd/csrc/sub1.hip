// Subsystem I of the Poisson splitting (Section 4.2): implicit discrete-gradient
// update of (x, p, e_x) with a_perp frozen, solved by Picard sweeps.
//
// One sweep k, for every particle (cell-local coordinate t, d = delta/dx):
//   A0 = A(t0), A1 = A(t1), t1 = t0 + d^(k)          (V0 gathers)
//   g00 = gamma(p, A0), g01 = gamma(p, A1)
//   lbar = mean of Lambda1 along the step; DA = (A1 - A0)/(t1 - t0) = lbar.(G a) dx
//   F = lbar.ebar - (A0 + A1).DA / (dx (g00 + g01))
//   p1 = p + dt F,  g11 = gamma(p1, A1),  d^(k+1) = (dt/dx) (p + p1)/(g01 + g11)
//   current += int Lambda1 along the step (Jacobi: of d^(k); Seidel: of d^(k+1))
// and then e^(k+1) = e_x^n - w M1^-1 (dx S) (field kernel).  A block owns one
// cell, so A, the divided differences and the line means are polynomials of
// the particle's local coordinates whose coefficients (coef.hpp) the block
// loads once; the current is accumulated as the moments sum (signed length) *
// h_i of its pieces and turned into the per-cell deposit once per block.  A
// step that enters a neighbour cell (at most one, since |d| < 1) adds a second
// piece; waves with no such step skip that code.
#include "coef.hpp"

namespace ecpic {

template <int P>
struct Coef1 {
    double ay[3][P + 1], az[3][P + 1];   // A on cells c-1, c, c+1
    double eb[3][P];                     // ebar piece-mean weights on cells c-1, c, c+1
};

template <int P>
__device__ __forceinline__ void load_coef1(Coef1<P> &k, int c, const double *coefA, const double *coefE) {
    constexpr int NA = RecA<P>::N, NE = RecE<P>::N;
    const double *a = coefA + (size_t)(rec_index(c) - 1) * NA;
    const double *e = coefE + (size_t)(rec_index(c) - 1) * NE;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int i = 0; i <= P; ++i) {
            k.ay[r][i] = a[r * NA + i];
            k.az[r][i] = a[r * NA + P + 1 + i];
        }
#pragma unroll
        for (int i = 0; i < P; ++i) k.eb[r][i] = e[r * NE + i];
    }
}

template <int P>
struct Moments {
    double A[P], R[P], L[P];   // sum over particles of (signed piece length) h_i(piece)
};

// End point of a step: xi0 in [c, c+1), t1 = (xi0 + d) - c is exact in floating
// point, so the committed position and the deposited segment agree.
__device__ __forceinline__ void end_point(double xi0, double d, int c, double &t1, int &s, int &flags) {
    t1 = (xi0 + d) - (double)c;
    if (!(t1 > -1.0 && t1 < 2.0)) {   // |d| >= 1 cell, or NaN
        flags |= FLAG_CFL;
        t1 = t1 >= 2.0 ? 1.5 : (t1 <= -1.0 ? -0.5 : 0.5);
    }
    s = t1 >= 1.0 ? 1 : (t1 < 0.0 ? -1 : 0);
}

template <int P>
__device__ __forceinline__ void deposit(Moments<P> &mo, double t0, double t1, int s) {
    const Seg<double> g = make_seg(t0, t1, s);
    double h[P];
    homog<P - 1>(g.aA, g.bA, h);
#pragma unroll
    for (int i = 0; i < P; ++i) mo.A[i] = fma(g.sA, h[i], mo.A[i]);
    if (__ballot(s != 0)) {
        homog<P - 1>(g.aB, g.bB, h);
        const double sr = s > 0 ? g.sB : 0.0, sl = s < 0 ? g.sB : 0.0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            mo.R[i] = fma(sr, h[i], mo.R[i]);
            mo.L[i] = fma(sl, h[i], mo.L[i]);
        }
    }
}

__device__ __forceinline__ double dt_dx_times(double dt_dx, double p) { return dt_dx * p; }

struct MapOut {
    double dn, p1, dused, t1;
    int s;
};

// The particle map of one sweep (see the file header).
template <int P>
__device__ __forceinline__ MapOut particle_map(const Coef1<P> &k, double xi0, int c, double p0, double d,
                                               bool explicit_start, double dt, double dt_dx, double inv_dx,
                                               int &flags) {
    MapOut o;
    double t0 = xi0 - (double)c;
    if (!(t0 >= 0.0 && t0 < 1.0)) { flags |= FLAG_ORDER; t0 = 0.5; }
    const double A0y = horner<P + 1>(k.ay[1], t0), A0z = horner<P + 1>(k.az[1], t0);
    const double q0 = fma(p0, p0, 1.0);
    const double g00 = fsqrt(q0 + A0y * A0y + A0z * A0z);
    if (explicit_start) d = dt_dx * p0 * frcp(g00);
    o.dused = d;
    double t1;
    int s;
    end_point(xi0, d, c, t1, s, flags);
    o.t1 = t1;
    o.s = s;
    const Seg<double> g = make_seg(t0, t1, s);
    double hA[P];
    homog<P - 1>(g.aA, g.bA, hA);
    double LE = pmean<P>(k.eb[1], hA);
    double DAy = divdiff<P>(k.ay[1], hA), DAz = divdiff<P>(k.az[1], hA);
    double A1y, A1z;
    if (__ballot(s != 0)) {
        const double tl = t1 - (double)s;
        const double yc = horner<P + 1>(k.ay[1], tl), yr = horner<P + 1>(k.ay[2], tl), yl = horner<P + 1>(k.ay[0], tl);
        const double zc = horner<P + 1>(k.az[1], tl), zr = horner<P + 1>(k.az[2], tl), zl = horner<P + 1>(k.az[0], tl);
        A1y = s > 0 ? yr : (s < 0 ? yl : yc);
        A1z = s > 0 ? zr : (s < 0 ? zl : zc);
        double hB[P];
        homog<P - 1>(g.aB, g.bB, hB);
        const double EB = s > 0 ? pmean<P>(k.eb[2], hB) : pmean<P>(k.eb[0], hB);
        const double DyB = s > 0 ? divdiff<P>(k.ay[2], hB) : divdiff<P>(k.ay[0], hB);
        const double DzB = s > 0 ? divdiff<P>(k.az[2], hB) : divdiff<P>(k.az[0], hB);
        if (s != 0) {
            const double inv = frcp(g.sA + g.sB);
            LE = (g.sA * LE + g.sB * EB) * inv;
            DAy = (g.sA * DAy + g.sB * DyB) * inv;
            DAz = (g.sA * DAz + g.sB * DzB) * inv;
        }
    } else {
        A1y = horner<P + 1>(k.ay[1], t1);
        A1z = horner<P + 1>(k.az[1], t1);
    }
    const double qa1 = A1y * A1y + A1z * A1z;
    const double g01 = fsqrt(q0 + qa1);
    const double F = LE - ((A0y + A1y) * DAy + (A0z + A1z) * DAz) * inv_dx * frcp(g00 + g01);
    o.p1 = fma(dt, F, p0);
    const double g11 = fsqrt(fma(o.p1, o.p1, 1.0) + qa1);
    o.dn = dt_dx * (p0 + o.p1) * frcp(g01 + g11);
    if (!(fabs(o.dn) < 1.0e300) || !(fabs(o.p1) < 1.0e300)) flags |= FLAG_NONFINITE;
    return o;
}

// Wave sum of the moments and conversion to the P+2 V1 slots of the wave's
// particles (slot q <-> V1 index c - P + q); lane q < P+2 returns slot q.
template <int P>
__device__ __forceinline__ double moments_to_slots(const Moments<P> &mo) {
    constexpr Pieces<P - 1> Q{};
    double t[3 * P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        t[i] = wave_sum_dpp(mo.A[i]);
        t[P + i] = wave_sum_dpp(mo.R[i]);
        t[2 * P + i] = wave_sum_dpp(mo.L[i]);
    }
    const int q = threadIdx.x & (WAVE - 1);
    double out = 0.0;
#pragma unroll
    for (int i = 0; i < 3 * P; ++i) {
        const int grp = i / P, ii = i % P;   // 0: cell c, 1: c+1, 2: c-1
        const int m = (grp == 0 ? P : (grp == 1 ? P + 1 : P - 1)) - q;   // index c + shift - m == c - P + q
        out += (m >= 0 && m < P) ? Q.q[m < 0 ? 0 : (m >= P ? P - 1 : m)][ii] * t[i] : 0.0;
    }
    return out;
}

// The sweep.  The block's own-cell coefficients stay in registers; the three
// cells' records are also staged in LDS, where the rare steps that enter a
// neighbour cell read them with a per-lane (position-dependent) address.  The
// waves of a block share only that staging: each wave takes every nw-th row of
// 64 particles of the item, loads the next row while it computes the current
// one, and writes its own partial slots (P+2 current sums, its residual max and
// its error flags), which the field kernel assembles per cell.
template <int P>
struct Own {
    double ay[P + 1], az[P + 1], eb[P];
};

template <int P>
struct LdsRec {   // one cell's coefficients in LDS
    double ay[P + 1], az[P + 1], eb[P];
};

struct Lane {
    double xi0, p0, d, t0, t1, q0, A0y, A0z, g00;
    int s;
};

template <int P>
__device__ __forceinline__ void stage_gather(const Own<P> &o, Lane &L, int c, bool explicit_start, double dt_dx,
                                             int &flags) {
    L.t0 = L.xi0 - (double)c;
    if (!(L.t0 >= 0.0 && L.t0 < 1.0)) { flags |= FLAG_ORDER; L.t0 = 0.5; }
    L.A0y = horner<P + 1>(o.ay, L.t0);
    L.A0z = horner<P + 1>(o.az, L.t0);
    L.q0 = fma(L.p0, L.p0, 1.0);
    L.g00 = fsqrt(L.q0 + L.A0y * L.A0y + L.A0z * L.A0z);
    if (explicit_start) L.d = dt_dx * L.p0 * frcp(L.g00);
    end_point(L.xi0, L.d, c, L.t1, L.s, flags);
}

// Momentum update and next increment; anycross is wave-uniform.
template <int P>
__device__ __forceinline__ void stage_push(const Own<P> &o, const LdsRec<P> *rec, bool anycross, const Lane &L,
                                           double dt, double dt_dx, double inv_dx, double &p1, double &dn,
                                           int &flags) {
    const double t1c = fmin(fmax(L.t1, 0.0), 1.0);
    double h[P];
    homog<P - 1>(fmin(L.t0, t1c), fmax(L.t0, t1c), h);
    double LE = pmean<P>(o.eb, h);
    double DAy = divdiff<P>(o.ay, h), DAz = divdiff<P>(o.az, h);
    double A1y, A1z;
    if (anycross) {
        // record of the cell holding t1, indexed arithmetically (t1 in (-1, 2))
        const int r = (int)floor(L.t1) + 1;
        const LdsRec<P> &nb = rec[r];
        const double tl = L.t1 - (double)(r - 1);
        A1y = horner<P + 1>(nb.ay, tl);
        A1z = horner<P + 1>(nb.az, tl);
        if (L.s != 0) {
            // piece inside cell c + s: [0, t1 - 1] or [t1 + 1, 1]
            double hb[P];
            homog<P - 1>(L.s > 0 ? 0.0 : tl, L.s > 0 ? tl : 1.0, hb);
            const double sA = t1c - L.t0, sB = L.t1 - t1c;
            const double inv = frcp(L.t1 - L.t0);
            LE = (sA * LE + sB * pmean<P>(nb.eb, hb)) * inv;
            DAy = (sA * DAy + sB * divdiff<P>(nb.ay, hb)) * inv;
            DAz = (sA * DAz + sB * divdiff<P>(nb.az, hb)) * inv;
        }
    } else {
        A1y = horner<P + 1>(o.ay, L.t1);
        A1z = horner<P + 1>(o.az, L.t1);
    }
    const double qa1 = A1y * A1y + A1z * A1z;
    const double g01 = fsqrt(L.q0 + qa1);
    const double F = LE - ((L.A0y + A1y) * DAy + (L.A0z + A1z) * DAz) * inv_dx * frcp(L.g00 + g01);
    p1 = fma(dt, F, L.p0);
    const double g11 = fsqrt(fma(p1, p1, 1.0) + qa1);
    dn = dt_dx * (L.p0 + p1) * frcp(g01 + g11);
    if (!(fabs(dn) < 1.0e300) || !(fabs(p1) < 1.0e300)) flags |= FLAG_NONFINITE;
}

// Moments of a step from t0 to t1 (end in cell c + s); scale 0 drops it.
template <int P>
__device__ __forceinline__ void stage_deposit(Moments<P> &mo, bool anycross, double t0, double t1, int s,
                                              double scale) {
    const double t1c = fmin(fmax(t1, 0.0), 1.0);
    double h[P];
    homog<P - 1>(fmin(t0, t1c), fmax(t0, t1c), h);
    const double sA = scale * (t1c - t0);
#pragma unroll
    for (int i = 0; i < P; ++i) mo.A[i] = fma(sA, h[i], mo.A[i]);
    if (anycross) {
        const double tl = t1 - (double)s;
        homog<P - 1>(s > 0 ? 0.0 : (s < 0 ? tl : 0.0), s > 0 ? tl : (s < 0 ? 1.0 : 0.0), h);
        const double sB = scale * (t1 - t1c);
        const double sr = s > 0 ? sB : 0.0, sl = s < 0 ? sB : 0.0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            mo.R[i] = fma(sr, h[i], mo.R[i]);
            mo.L[i] = fma(sl, h[i], mo.L[i]);
        }
    }
}

// Has sweep k-1 met the tolerance?  Records kconv if so.
__device__ __forceinline__ bool prev_converged(DevStatus *st, int k, double dx, double tol, bool writer) {
    if (k <= 0) return false;
    const double r = fmax(dbits(st->rx_bits[(k - 1) & 1]) * dx, dbits(st->re_bits[(k - 1) & 1]));
    if (writer && k - 1 < MAX_HIST) st->res_hist[k - 1] = r;
    if (r <= tol) {
        if (writer) { st->kconv = k - 1; st->res = r; }
        return true;
    }
    return false;
}

template <int P, bool SEIDEL>
__global__ void __launch_bounds__(MAX_BLOCK) k_sweep_I(SweepIArgs a) {
    __shared__ LdsRec<P> rec[3];   // cells c-1, c, c+1
    DevStatus *st = a.st;
    const int item = blockIdx.x;
    if (item >= *a.items.n_items) return;
    if (!st->gate | st->flags | (st->kconv >= 0)) return;
    const int k = a.k;
    if (prev_converged(st, k, a.dx, a.tol, threadIdx.x == 0)) return;
    const double *din = (k & 1) ? a.d1 : a.d0;
    double *dout = (k & 1) ? a.d0 : a.d1;
    const double *coefE = (k & 1) ? a.coefE1 : a.coefE0;
    const bool explicit_start = (k == 0) && a.explicit_start;
    const int c = a.items.cell[item];
    const int beg = a.items.begin[item], end = a.items.begin[item + 1];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
    // first row of this wave (clamped index: lanes past the end recompute the
    // item's last particle and discard it)
    int ia = beg + wid * WAVE + lane;
    double nx, np, nd;
    {
        const int il = min(ia, end - 1);
        nx = a.xi[il];
        np = a.p[il];
        nd = explicit_start ? 0.0 : din[il];
    }
    {
        constexpr int NA = RecA<P>::N, NE = RecE<P>::N;
        const double *ra = a.coefA + (size_t)(rec_index(c) - 1) * NA;
        const double *re = coefE + (size_t)(rec_index(c) - 1) * NE;
        const int t = threadIdx.x;
        if (t < 3 * NA) {
            const int r = t / NA, i = t % NA;
            if (i <= P) rec[r].ay[i] = ra[t];
            else rec[r].az[i - P - 1] = ra[t];
        } else if (t < 3 * NA + 3 * NE) {
            const int u = t - 3 * NA, r = u / NE, i = u % NE;
            rec[r].eb[i] = re[u];
        }
    }
    Own<P> o1;
    {
        const double *ra = a.coefA + (size_t)rec_index(c) * RecA<P>::N;
        const double *re = coefE + (size_t)rec_index(c) * RecE<P>::N;
#pragma unroll
        for (int i = 0; i <= P; ++i) { o1.ay[i] = ra[i]; o1.az[i] = ra[P + 1 + i]; }
#pragma unroll
        for (int i = 0; i < P; ++i) o1.eb[i] = re[i];
    }
    __syncthreads();
    Moments<P> mo;
#pragma unroll
    for (int i = 0; i < P; ++i) { mo.A[i] = 0.0; mo.R[i] = 0.0; mo.L[i] = 0.0; }
    double rmax = 0.0;
    int flags = 0;
    const int stride = nw * WAVE;
    for (int row = beg + wid * WAVE; row < end; row += stride, ia += stride) {
        Lane La;
        La.xi0 = nx;
        La.p0 = np;
        La.d = nd;
        const bool valid = ia < end;
        if (row + stride < end) {   // prefetch the next row
            const int il = min(ia + stride, end - 1);
            nx = a.xi[il];
            np = a.p[il];
            nd = explicit_start ? 0.0 : din[il];
        }
        stage_gather<P>(o1, La, c, explicit_start, a.dt_dx, flags);
        const bool cross1 = __ballot(La.s != 0) != 0;
        double pa, dna;
        stage_push<P>(o1, rec, cross1, La, a.dt, a.dt_dx, a.inv_dx, pa, dna, flags);
        if (valid) {
            if (!SEIDEL && explicit_start) a.d0[ia] = La.d;   // keep d^(0) for a Jacobi commit
            dout[ia] = dna;
            rmax = fmax(rmax, fabs(dna - La.d));
        }
        const double w = valid ? 1.0 : 0.0;
        if (SEIDEL) {
            double ta;
            int sa;
            end_point(La.xi0, dna, c, ta, sa, flags);
            stage_deposit<P>(mo, __ballot(sa != 0) != 0, La.t0, ta, sa, w);
        } else {
            stage_deposit<P>(mo, cross1, La.t0, La.t1, La.s, w);
        }
    }
    const double slot = moments_to_slots<P>(mo);
    rmax = wave_max_dpp(rmax);
    const int fl = __ballot(flags != 0) ? wave_or(flags) : 0;
    double *out = a.part + ((size_t)item * nw + wid) * (P + 4);
    if (lane < P + 2) out[lane] = slot;
    else if (lane == P + 2) out[lane] = rmax;
    else if (lane == P + 3) out[lane] = (double)fl;
}

// Partial sums of the items of cell c (usually one item), slot by slot.
template <int NS>
__device__ __forceinline__ void cell_partials(const ItemList &it, const double *part, int c, double (&v)[NS]) {
#pragma unroll
    for (int q = 0; q < NS; ++q) v[q] = 0.0;
    const int i0 = it.cell_first[c], i1 = it.cell_first[c + 1];
    for (int i = i0; i < i1; ++i) {
#pragma unroll
        for (int q = 0; q < NS; ++q) v[q] += part[(size_t)i * NS + q];
    }
}

// Sum of the wave partials of cell c (its items times wpi waves each): the P+2
// current slots, the max of the residuals and the OR of the flags.
template <int P>
__device__ __forceinline__ void cell_partials_I(const ItemList &it, const double *part, int c, int wpi,
                                                double (&v)[P + 2], double &rx, int &flags) {
#pragma unroll
    for (int q = 0; q < P + 2; ++q) v[q] = 0.0;
    const int u0 = it.cell_first[c] * wpi, u1 = it.cell_first[c + 1] * wpi;
    for (int u = u0; u < u1; ++u) {
        const double *w = part + (size_t)u * (P + 4);
#pragma unroll
        for (int q = 0; q < P + 2; ++q) v[q] += w[q];
        rx = fmax(rx, w[P + 2]);
        flags |= (int)w[P + 3];
    }
}

// Field update of sweep k and the E-records of the next ebar.  Block b
// computes e^(k+1) on the FIELD_OUT cells starting at b * TILE - (P - 1) (the
// first P - 1 only to form the records of cells b * TILE .. b * TILE + TILE - 1).
// The wave partials are summed per cell into LDS, the current S assembled from
// them, and the M1 inverse applied as a convolution: four lanes share an output,
// each taking every fourth tap, and their sums are combined in a fixed order.
constexpr int FIELD_OUT = 64;

template <int P>
__global__ void __launch_bounds__(256) k_field_I(FieldIArgs a) {
    extern __shared__ double smem[];
    __shared__ double ldsm[MAX_WAVES], ldsx[MAX_WAVES];
    __shared__ int ldsf[MAX_WAVES];
    constexpr int NS = P + 2;
    constexpr int TILE = FIELD_OUT - (P - 1);
    DevStatus *st = a.st;
    if (!st->gate | st->flags | (st->kconv >= 0)) return;
    const int k = a.k;
    const int M = a.M;
    const int j0 = blockIdx.x * TILE - (P - 1);   // first cell computed
    const int mhi = a.mlo + a.ntaps - 1;
    const int slen = FIELD_OUT + a.ntaps - 1;     // S on cells [j0 - mhi, j0 - mhi + slen)
    const int clo = j0 - mhi - 1;                 // S_j needs the partials of cells j-1 .. j+P
    const int clen = slen + P + 1;
    double *cp = smem;
    double *S = cp + (size_t)clen * NS;
    double *tp = S + slen;
    double *enl = tp + a.ntaps;
    const double *ek = k == 0 ? a.en : ((k & 1) ? a.ek1 : a.ek0);
    // loads that do not depend on the partials: this quad's output cell
    const int quad = threadIdx.x >> 2, ql = threadIdx.x & 3;
    const int jq = j0 + quad, jqm = imod(jq, M);
    const double en_q = a.en[jqm + HALO];
    const double ek_q = ek[jqm + HALO];
    for (int t = threadIdx.x; t < a.ntaps; t += blockDim.x) tp[t] = a.taps[t];
    double rx = 0.0;
    int flags = 0;
    for (int t = threadIdx.x; t < clen; t += blockDim.x) {
        double v[NS];
        cell_partials_I<P>(a.items, a.part, imod(clo + t, M), a.wpi, v, rx, flags);
#pragma unroll
        for (int q = 0; q < NS; ++q) cp[t * NS + q] = v[q];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < slen; t += blockDim.x) {
        double sum = 0.0;
#pragma unroll
        for (int r = 0; r < NS; ++r) sum += cp[(t + r) * NS + (P + 1 - r)];   // cell (j-1+r): slot P+1-r
        S[t] = sum;
    }
    __syncthreads();
    double *eout = (k & 1) ? a.ek0 : a.ek1;
    double *Eout = ((k + 1) & 1) ? a.coefE1 : a.coefE0;
    double re = 0.0;
    {
        // S_{j - m} for m = mlo + i sits at S[quad + mhi - m] = S[quad + ntaps - 1 - i]
        const double *Sq = S + quad + a.ntaps - 1;
        double acc0 = 0.0, acc1 = 0.0;
        int i = ql;
        for (; i + 4 < a.ntaps; i += 8) {
            acc0 = fma(tp[i], Sq[-i], acc0);
            acc1 = fma(tp[i + 4], Sq[-i - 4], acc1);
        }
        if (i < a.ntaps) acc0 = fma(tp[i], Sq[-i], acc0);
        double conv = acc0 + acc1;
        conv += dpp_d<0xB1>(conv);   // quad_perm [1,0,3,2]
        conv += dpp_d<0x4E>(conv);   // quad_perm [2,3,0,1]
        const double enew = en_q - a.w * conv;
        if (ql == 0) {
            enl[quad] = enew;
            if (quad >= P - 1 && jq < M) {
                store_padded(eout, M, jqm, enew);
                re = fabs(enew - ek_q);
                if (!(fabs(enew) < 1.0e300)) flags |= FLAG_NONFINITE;
            }
        }
    }
    __syncthreads();
    {
        const int q = threadIdx.x + P - 1;
        const int j = j0 + q;
        if (q < FIELD_OUT && j < M) {
            double r[P];
            make_recE<P>([&](int jj) { return 0.5 * (a.en[imod(jj, M) + HALO] + enl[jj - j0]); }, j, r);
            for (int i = 0; i < P; ++i) store_record(Eout, M, j, RecE<P>::N, i, r[i]);
        }
    }
    re = wave_max(re);
    rx = wave_max(rx);
    flags = wave_or(flags);
    {
        const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
        if (lane == 0) { ldsm[wid] = re; ldsx[wid] = rx; ldsf[wid] = flags; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / WAVE); ++w) {
            re = fmax(re, ldsm[w]);
            rx = fmax(rx, ldsx[w]);
            flags |= ldsf[w];
        }
        atomicMax(&st->re_bits[k & 1], bitsd(re));
        atomicMax(&st->rx_bits[k & 1], bitsd(rx));
        if (flags) atomicOr(&st->flags, flags);
        if (blockIdx.x == 0) {   // clear the slots field kernel k+1 accumulates into
            st->rx_bits[(k + 1) & 1] = 0ull;
            st->re_bits[(k + 1) & 1] = 0ull;
        }
    }
}

// Records of a substep start: A-records of a_perp and E-records of e.
template <int P>
__global__ void __launch_bounds__(256) k_prep_records(const DevStatus *st, const double *ay, const double *az,
                                                      const double *e, double *coefA, double *coefE, int M) {
    if (st && !st->gate) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= M) return;
    double ry[P + 1], rz[P + 1];
    make_recA<P>(ay, az, c, ry, rz);
    for (int i = 0; i <= P; ++i) {
        store_record(coefA, M, c, RecA<P>::N, i, ry[i]);
        store_record(coefA, M, c, RecA<P>::N, P + 1 + i, rz[i]);
    }
    if (coefE) {
        double r[P];
        make_recE<P>([&](int jj) { return e[jj + HALO]; }, c, r);
        for (int i = 0; i < P; ++i) store_record(coefE, M, c, RecE<P>::N, i, r[i]);
    }
}

// ---- commit: re-evaluate the committed momentum, move the particles and
// keep them cell-sorted.  A particle moves at most one cell per step, so the
// new order of cell c' is [right-movers of c'-1][stayers of c'][left-movers of
// c'+1], each group in the old order (a stable three-way merge).

struct CommitPick {
    const double *d;       // increment to commit
    const double *coefE;   // ebar records for the committed momentum
    const double *enew;    // e_x^{n+1}
};

__device__ __forceinline__ CommitPick commit_pick(const CommitIArgs &a, int kc) {
    CommitPick r;
    r.enew = ((kc + 1) & 1) ? a.ek1 : a.ek0;   // e^(kc+1)
    if (a.seidel) {
        r.d = ((kc + 1) & 1) ? a.d1 : a.d0;     // delta^(kc+1)
        r.coefE = ((kc + 1) & 1) ? a.coefE1 : a.coefE0;
    } else {
        r.d = (kc & 1) ? a.d1 : a.d0;           // delta^(kc)
        r.coefE = (kc & 1) ? a.coefE1 : a.coefE0;
    }
    return r;
}

__device__ __forceinline__ bool commit_enabled(const DevStatus *st) {
    return st->gate && st->kconv >= 0 && !st->committed && st->flags == 0;
}

// Converged sweep index for the commit, making the test of the last enqueued
// sweep if no later sweep made it; -1 if the commit must not run.
__device__ __forceinline__ int settle_last(DevStatus *st, int nsweeps, double dx, double tol, bool writer) {
    if (!st->gate || st->flags || st->committed) return -1;
    if (st->kconv >= 0) return st->kconv;
    return prev_converged(st, nsweeps, dx, tol, writer) ? nsweeps - 1 : -1;
}

__device__ __forceinline__ int mover_type(double xi0, double d, int c) {
    const double t1 = (xi0 + d) - (double)c;
    return t1 >= 1.0 ? 2 : (t1 < 0.0 ? 0 : 1);   // 0 left, 1 stay, 2 right
}

__global__ void __launch_bounds__(MAX_BLOCK) k_commit_count(CommitIArgs a) {
    __shared__ int lds[MAX_WAVES * 3];
    const int item = blockIdx.x;
    const int kc = settle_last(a.st, a.nsweeps, a.dx, a.tol, item == 0 && threadIdx.x == 0);
    if (kc < 0) return;
    if (item >= *a.items.n_items) return;
    const CommitPick pk = commit_pick(a, kc);
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
    const CommitPick pk = commit_pick(a, a.st->kconv);
    for (int idx = threadIdx.x; idx < M + 2 * HALO; idx += blockDim.x) a.ex_next[idx] = pk.enew[idx];
}

template <int P>
__global__ void __launch_bounds__(MAX_BLOCK) k_commit_scatter(CommitIArgs a) {
    __shared__ int wc[MAX_WAVES][3];
    const int item = blockIdx.x;
    if (item >= *a.items.n_items || !commit_enabled(a.st)) return;
    const CommitPick pk = commit_pick(a, a.st->kconv);
    const int c = a.items.cell[item];
    const int beg = a.items.begin[item], end = a.items.begin[item + 1];
    const int M = a.M;
    Coef1<P> kc;
    load_coef1<P>(kc, c, a.coefA, pk.coefE);
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
            const MapOut o = particle_map<P>(kc, xi0, c, p0, d, false, a.dt, a.dt_dx, a.inv_dx, flags);
            p1 = o.p1;
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
    if (st->kconv >= 0 && !st->committed && st->flags == 0 && st->gate) st->committed = 1;
}

__global__ void k_begin(DevStatus *st, const DevStatus *gate) {
    st->rx_bits[0] = 0ull;
    st->rx_bits[1] = 0ull;
    st->re_bits[0] = 0ull;
    st->re_bits[1] = 0ull;
    st->kconv = -1;
    st->committed = 0;
    st->flags = 0;
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

void launch_field_I(int P, int M, hipStream_t s, const FieldIArgs &a) {
    const int grid = (M + FIELD_OUT - (P - 1) - 1) / (FIELD_OUT - (P - 1));
    const int slen = FIELD_OUT + a.ntaps - 1;
    const size_t lds = sizeof(double) * ((size_t)(slen + P + 1) * (P + 2) + slen + a.ntaps + FIELD_OUT);
#define ECPIC_F(PP) case PP: hipLaunchKernelGGL((k_field_I<PP>), dim3(grid), dim3(256), lds, s, a); break;
    switch (P) { ECPIC_F(2) ECPIC_F(3) ECPIC_F(4) ECPIC_F(5) }
#undef ECPIC_F
}

void launch_prep_records(int P, hipStream_t s, const DevStatus *st, const double *ay, const double *az,
                         const double *e, double *coefA, double *coefE, int M) {
    const int grid = (M + 255) / 256;
#define ECPIC_PR(PP) \
    case PP: hipLaunchKernelGGL((k_prep_records<PP>), dim3(grid), dim3(256), 0, s, st, ay, az, e, coefA, coefE, M); break;
    switch (P) { ECPIC_PR(2) ECPIC_PR(3) ECPIC_PR(4) ECPIC_PR(5) }
#undef ECPIC_PR
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
