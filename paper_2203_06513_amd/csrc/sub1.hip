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
#include <type_traits>

#include "sweep.hpp"

namespace ecpic {

// The sweep.  The block's own-cell coefficients stay in registers; the three
// cells' records are also staged in LDS, where the rare steps that enter a
// neighbour cell read them with a per-lane (position-dependent) address.  The
// waves of a block share only that staging: each wave takes its run of rows of
// the item, loads the next row while it computes the current one, and writes
// its own partial values (UnitI), which the field kernel assembles per cell.
// At the end the block counts the particles that would leave to the left,
// stay or leave to the right if the sweep's increment were committed, per item
// and per wave (the commit places the movers from them).
template <int P, typename T>
struct Own {
    T ay[P + 1], az[P + 1], eb[P];
};

template <int P, typename T>
struct LdsRec {   // one cell's coefficients in LDS
    T ay[P + 1], az[P + 1], eb[P];
};

template <typename T>
struct Lane {
    T t0, p0, d, t1, q0, A0y, A0z, g00;
    T sy, sz;   // the particle's spin (spin force only)
    int s;
    // adjoint scheme: |A0|^2, the momentum iterate P = p^{n+1} the increment
    // stands for, and gamma(x^n, P)
    T qa0, P, g10;
};

// The adjoint scheme (the discrete gradient with p varied first, at x^n, then
// x, at p^{n+1}) has delta = dt (p0 + P) / (gamma(x0, p0) + gamma(x0, P)); for
// a given delta this is solved for P in closed form.  With v = delta / dt,
// m^2 = 1 + |A0|^2 and b = p0 - v gamma(x0, p0), squaring
// v gamma(x0, P) = P + b gives (1 - v^2) P^2 + 2 b P + b^2 - v^2 m^2 = 0, and
// the root with P + b of the sign of v is
//   P = (v R - b) / (1 - v^2),   R = sqrt(b^2 + (1 - v^2) m^2).
template <typename T>
__device__ __forceinline__ T adjoint_momentum(T v, T p0, T g00, T m2) {
    const T b = fma(-v, g00, p0);
    const T om = fma(-v, v, (T)1);
    const T R = fsqrt(fma(b, b, om * m2));
    return fma(v, R, -b) * frcp(om);
}

// Gather at the step start, gamma there, the explicit first increment if asked,
// and the end point of the current increment.  xi0 - c is exact in FP64; the
// single precision sweeps round it once.
template <int P, typename T, bool EXPL, bool ADJ = false>
__device__ __forceinline__ void stage_gather(const Own<P, T> &o, Lane<T> &L, double xi0, int c, T dt_dx,
                                             int &flags, T dx_dt = (T)0) {
    const double t0 = xi0 - (double)c;
    wave_flag(flags, !(t0 >= 0.0), FLAG_ORDER);
    wave_flag(flags, !(t0 < 1.0), FLAG_ORDER);
    L.t0 = (T)fmin(fmax(t0, 0.0), 1.0);
    L.A0y = horner<P + 1>(o.ay, L.t0);
    L.A0z = horner<P + 1>(o.az, L.t0);
    L.q0 = fma(L.p0, L.p0, (T)1);
    if constexpr (ADJ) {
        L.qa0 = fma(L.A0y, L.A0y, L.A0z * L.A0z);
        L.g00 = fsqrt(L.q0 + L.qa0);
        if constexpr (EXPL) {   // P^(0) = p^n
            L.d = dt_dx * L.p0 * frcp(L.g00);
            L.P = L.p0;
            L.g10 = L.g00;
        } else {
            const T m2 = (T)1 + L.qa0;
            L.P = adjoint_momentum<T>(L.d * dx_dt, L.p0, L.g00, m2);
            L.g10 = fsqrt(fma(L.P, L.P, m2));
        }
    } else {
        L.g00 = fsqrt(L.q0 + L.A0y * L.A0y + L.A0z * L.A0z);
    }
    if constexpr (EXPL && !ADJ) L.d = dt_dx * L.p0 * frcp(L.g00);
    if constexpr (sizeof(T) == 8) end_point(xi0, L.d, c, L.t1, L.s, flags);
    else end_point(L.t0, L.d, L.t1, L.s, flags);
}

// A and gamma at the step's end with the new momentum (for the commit).
template <typename T>
struct PushEnd {
    T A1y, A1z, g11;
};

// Momentum update and next increment; anycross is wave-uniform.  ADJ: the
// adjoint scheme, whose force divides by gamma(x0, P) + gamma(x1, P) and whose
// next increment is that of the new momentum (dt (p0 + p1) / (gamma(x0, p0) +
// gamma(x0, p1))).  MOM: p1 is wanted (the commit); a sweep needs only the
// increment, which it then forms with one reciprocal instead of two (p1 and
// the flags' finiteness test take N = p1 (g00 + g01) in its place).
// SPIN: the force of the Zeeman energy, hbar (s_z DD_y - s_y DD_z) with DD the
// divided difference of dA/dx along the step (per cell, (A'(t1) - A'(t0))/(t1 -
// t0) / dx^2 with A' = dA/dt, from the same h_i); hbar_dx2 = hbar / dx^2.  It
// does not depend on p, so the adjoint takes it unchanged.  DN = false: only the
// momentum is wanted (the commit), so the next increment and its reciprocal are
// not formed (dn is left unset).
template <int P, typename T, bool ADJ = false, bool MOM = true, bool SPIN = false, bool DN = true>
__device__ __forceinline__ void stage_push(const Own<P, T> &o, const LdsRec<P, T> *rec, bool anycross,
                                           const Lane<T> &L, T dt, T dt_dx, T inv_dx, T &p1, T &dn, int &flags,
                                           PushEnd<T> *pe = nullptr, T hbar_dx2 = (T)0) {
    const T zero = (T)0, one = (T)1;
    const T t1c = fmin(fmax(L.t1, zero), one);
    T h[P];
    homog<P - 1>(fmin(L.t0, t1c), fmax(L.t0, t1c), h);
    T LE = pmean<P>(o.eb, h);
    T DAy = divdiff<P>(o.ay, h), DAz = divdiff<P>(o.az, h);
    T DDy = (T)0, DDz = (T)0;
    if constexpr (SPIN) {
        DDy = divdiff2<P>(o.ay, h);
        DDz = divdiff2<P>(o.az, h);
    }
    T A1y, A1z;
    if (anycross) {
        // record of the cell holding t1 (s = floor(t1) in {-1, 0, 1})
        const LdsRec<P, T> &nb = rec[L.s + 1];
        const T tl = L.t1 - (T)L.s;
        A1y = horner<P + 1>(nb.ay, tl);
        A1z = horner<P + 1>(nb.az, tl);
        if (L.s != 0) {
            // piece inside cell c + s: [0, t1 - 1] or [t1 + 1, 1]
            T hb[P];
            homog<P - 1>(L.s > 0 ? zero : tl, L.s > 0 ? tl : one, hb);
            const T sA = t1c - L.t0, sB = L.t1 - t1c;
            const T inv = frcp(L.t1 - L.t0);
            LE = (sA * LE + sB * pmean<P>(nb.eb, hb)) * inv;
            DAy = (sA * DAy + sB * divdiff<P>(nb.ay, hb)) * inv;
            DAz = (sA * DAz + sB * divdiff<P>(nb.az, hb)) * inv;
            if constexpr (SPIN) {   // dA/dx is continuous at the knot (degree >= 2)
                DDy = (sA * DDy + sB * divdiff2<P>(nb.ay, hb)) * inv;
                DDz = (sA * DDz + sB * divdiff2<P>(nb.az, hb)) * inv;
            }
        }
    } else {
        // A at the end point from the divided difference: A1 = A0 + (t1 - t0) DA
        // (the same value as evaluating A there, in two operations instead of
        // 2P; and (A0 + A1).DA (t1 - t0) = |A1|^2 - |A0|^2 then holds to rounding)
        const T dt1 = L.t1 - L.t0;
        A1y = fma(dt1, DAy, L.A0y);
        A1z = fma(dt1, DAz, L.A0z);
    }
    if constexpr (SPIN) LE = fma(hbar_dx2, fma(L.sz, DDy, -L.sy * DDz), LE);
    const T qa1 = A1y * A1y + A1z * A1z;
    T g11;
    if constexpr (ADJ) {
        g11 = fsqrt(fma(L.P, L.P, one) + qa1);
        const T F = LE - ((L.A0y + A1y) * DAy + (L.A0z + A1z) * DAz) * inv_dx * frcp(L.g10 + g11);
        p1 = fma(dt, F, L.p0);
        const T g10n = fsqrt(fma(p1, p1, one) + L.qa0);
        dn = dt_dx * (L.p0 + p1) * frcp(L.g00 + g10n);
    } else if constexpr (MOM) {
        const T g01 = fsqrt(L.q0 + qa1);
        const T F = LE - ((L.A0y + A1y) * DAy + (L.A0z + A1z) * DAz) * inv_dx * frcp(L.g00 + g01);
        p1 = fma(dt, F, L.p0);
        g11 = fsqrt(fma(p1, p1, one) + qa1);
        if constexpr (DN) dn = dt_dx * (L.p0 + p1) * frcp(g01 + g11);
    } else {
        // with U = g00 + g01 and N = p1 U = p0 U + dt (LE U - X):
        //   gamma(p1, A1) = sqrt(U^2 (1 + |A1|^2) + N^2) / U, so
        //   d^(k+1) = (dt/dx) (p0 U + N) / (g01 U + sqrt(U^2 (1 + |A1|^2) + N^2))
        const T g01 = fsqrt(L.q0 + qa1);
        const T U = L.g00 + g01;
        const T X = ((L.A0y + A1y) * DAy + (L.A0z + A1z) * DAz) * inv_dx;
        const T N = fma(dt, fma(LE, U, -X), L.p0 * U);
        const T W = fma(N, N, U * U * (one + qa1));
        dn = dt_dx * fma(L.p0, U, N) * frcp(fma(g01, U, fsqrt(W)));
        p1 = N;
        g11 = (T)0;
    }
    if (pe) {
        pe->A1y = A1y;
        pe->A1z = A1z;
        pe->g11 = g11;
    }
    const T big = sizeof(T) == 8 ? (T)1.0e300 : (T)1.0e30f;
    if constexpr (DN) wave_flag(flags, !(fabs(dn) < big), FLAG_NONFINITE);
    wave_flag(flags, !(fabs(p1) < big), FLAG_NONFINITE);
}

// The records of cells c-1, c, c+1 into LDS, one value per thread; the caller
// synchronises before reading them.
template <int P, typename T>
__device__ __forceinline__ void stage_records(LdsRec<P, T> *rec, const double *coefA, const double *coefE, int c) {
    constexpr int NA = RecA<P>::N, NE = RecE<P>::N;
    const double *ra = coefA + (size_t)(rec_index(c) - 1) * NA;
    const double *re = coefE + (size_t)(rec_index(c) - 1) * NE;
    const int t = threadIdx.x;
    if (t < 3 * NA) {
        const int r = t / NA, i = t % NA;
        if (i <= P) rec[r].ay[i] = (T)ra[t];
        else rec[r].az[i - P - 1] = (T)ra[t];
    } else if (t < 3 * NA + 3 * NE) {
        const int u = t - 3 * NA, r = u / NE, i = u % NE;
        rec[r].eb[i] = (T)re[u];
    }
}

// The block's own cell (record 1) from LDS into registers.  Reading them from
// LDS rather than global memory keeps the particle loop's memory waits
// counting only its own row loads and stores.  (Moving them to scalar
// registers, since they are wave-uniform, took the quintic sweep from three to
// four waves per SIMD but did not make it faster, and made the cubic one 12 %
// slower.)
template <int P, typename T>
__device__ __forceinline__ void own_from_lds(const LdsRec<P, T> *rec, Own<P, T> &o1) {
#pragma unroll
    for (int i = 0; i <= P; ++i) { o1.ay[i] = rec[1].ay[i]; o1.az[i] = rec[1].az[i]; }
#pragma unroll
    for (int i = 0; i < P; ++i) o1.eb[i] = rec[1].eb[i];
}

// Has sweep k-1 met the tolerance?  Records kconv if so.  Only FP64 sweeps
// (index >= first64) can end the iteration.  rxb, reb: the residual slots of
// sweep k-1, loaded by the caller.
__device__ __forceinline__ bool prev_converged(DevStatus *st, int k, int first64, double dx, double tol,
                                               bool writer, unsigned long long rxb, unsigned long long reb) {
    if (k <= first64) return false;
    const double r = fmax(dbits(rxb) * dx, dbits(reb));
    if (writer && k - 1 < MAX_HIST) st->res_hist[k - 1] = r;
    if (writer && k - 1 - first64 < 4) st->res_first[k - 1 - first64] = r;
    if (r <= tol) {
        if (writer) { st->kconv = k - 1; st->res = r; }
        return true;
    }
    return false;
}

__device__ __forceinline__ bool prev_converged(DevStatus *st, int k, int first64, double dx, double tol,
                                               bool writer) {
    return prev_converged(st, k, first64, dx, tol, writer, st->rx_bits[(k - 1) & 1], st->re_bits[(k - 1) & 1]);
}

template <int P>
__device__ __forceinline__ void to_double(const Moments<P> &m, Moments<P> &o) { o = m; }
template <int P>
__device__ __forceinline__ void to_double(const Moments32<P> &m, Moments<P> &o) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
        o.A[i] = (double)m.A[i] + (double)m.cA[i];
        o.R[i] = (double)m.R[i] + (double)m.cR[i];
        o.L[i] = (double)m.L[i] + (double)m.cL[i];
    }
}

// One Picard sweep in precision T.  T = double is the method itself; T = float
// is the cheap first phase of the precision form: the same map with the
// particle arithmetic, the increments (a float iterate) and the per-lane
// moments (compensated) in single precision, while the partials, the field
// update and the convergence test stay in FP64.  A float sweep never ends the
// iteration and is never committed; the first FP64 sweep after it reads its
// float increments (d32in).
// Where d^(k) comes from: computed explicitly (first sweep), read back from the
// previous FP64 sweep, or read from the last float sweep of the precision form.
// START_PREV: the first sweep of a substep reads d^(0) from the increment the
// last commit took (the previous step's converged displacement, kept in the
// current order by that commit).
enum : int { START_READ = 0, START_EXPLICIT = 1, START_FLOAT = 2, START_PREV = 3 };

// The queue of crossing lanes (see the sweep loop, degree >= 4): per wave, in
// dynamic LDS, the particles to redo: position, momentum and increment as
// loaded, and the index.  (Reloading them from memory instead, when a row of
// them has gathered some 30 rows later, fetched whole lines again for 8 bytes
// each: 5 bytes per particle and sweep more HBM traffic at degree 5.)
constexpr int QCAP = 2 * WAVE;
struct QueueW {
    double *x, *p, *d;
    int *i;
};
inline size_t queue_lds_bytes(int block) { return (size_t)(block / WAVE) * QCAP * (3 * sizeof(double) + sizeof(int)); }
__device__ __forceinline__ QueueW queue_of_wave(double *base, int wid) {
    double *w = base + (size_t)wid * QCAP * 7 / 2;   // 3 doubles and an int per slot (QCAP even)
    return QueueW{w, w + QCAP, w + 2 * QCAP, reinterpret_cast<int *>(w + 3 * QCAP)};
}

template <int P, bool SEIDEL, typename T, int START, bool ADJ, bool SPIN>
__device__ __forceinline__ void sweep_I_item(const SweepIArgs &a, int item, LdsRec<P, T> *rec, double *queue) {
    static_assert(!ADJ || SEIDEL, "the adjoint scheme deposits the increment it has just produced");
    static_assert(!SPIN || (sizeof(T) == 8 && START != START_FLOAT), "spin runs the plain FP64 sweeps");
    constexpr bool F64 = sizeof(T) == 8;
    using MO = typename std::conditional<F64, Moments<P>, Moments32<P>>::type;
    DevStatus *st = a.st;
    const int k = a.k;
    // the item count, the status words and the item's description are loaded
    // together, so the start costs one memory round trip instead of three
    const int n_items = *a.items.n_items;
    const int sgate = st->gate, sflags = st->flags, skconv = st->kconv;
    const unsigned long long rxb = st->rx_bits[(k - 1) & 1], reb = st->re_bits[(k - 1) & 1];
    const int c = a.items.cell[item];
    const int beg = a.items.begin[item], end = a.items.begin[item + 1];
    asm volatile("" ::"s"(n_items), "s"(sgate), "s"(sflags), "s"(skconv), "s"(rxb), "s"(reb), "s"(c), "s"(beg),
                 "s"(end));
    if (item >= n_items) return;
    if (!sgate | sflags | (skconv >= 0)) return;
    if (F64 && prev_converged(st, k, a.first64, a.dx, a.tol, threadIdx.x == 0, rxb, reb)) return;
    const T *din;
    T *dout;
    if constexpr (F64) {
        din = (k & 1) ? a.d1 : a.d0;
        dout = (k & 1) ? a.d0 : a.d1;
    } else {
        din = (k & 1) ? a.f1 : a.f0;
        dout = (k & 1) ? a.f0 : a.f1;
    }
    const float *d32in = a.d32in;   // FP64 sweep right after the float ones (START_FLOAT)
    const double *coefE = (k & 1) ? a.coefE1 : a.coefE0;
    constexpr bool explicit_start = START == START_EXPLICIT;
    constexpr bool from_float = F64 && START == START_FLOAT;
    constexpr bool from_prev = START == START_PREV;
    const double *dprev = a.dprev;
    // d^(0) is kept in FP64 where a Jacobi commit may take it
    constexpr bool keep_start = F64 && !SEIDEL && (explicit_start || from_float || from_prev);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
    int wb, we;
    wave_range(beg, end, wid, nw, wb, we);
    // first row of this wave (clamped index: lanes past the run recompute its
    // last particle and discard it)
    int ia = wb + lane;
    double nx = 0.0, np = 0.0;
    T nd = (T)0;
    float nf = 0.0f;   // the float increment (from_float; converted at use)
    double nsy = 0.0, nsz = 0.0;   // spin (SPIN)
    if (wb < we) {
        const int il = min(ia, we - 1);
        nx = a.xi[il];
        np = a.p[il];
        if constexpr (from_float) nf = d32in[il];
        else if constexpr (from_prev) nd = (T)dprev[il];
        else if constexpr (!explicit_start) nd = din[il];
        if constexpr (SPIN) { nsy = a.sy[il]; nsz = a.sz[il]; }
    }
    stage_records<P, T>(rec, a.coefA, coefE, c);
    __syncthreads();
    Own<P, T> o1;
    own_from_lds<P, T>(rec, o1);
    // Every load issued so far (the first row, the records) completes here, so
    // the loop's memory waits only ever concern the loop's own loads and stores.
    __builtin_amdgcn_s_waitcnt(0);
    MO mo{};
    const T dt = (T)a.dt, dt_dx = (T)a.dt_dx, inv_dx = (T)a.inv_dx, dx_dt = (T)a.dx_dt;
    const T hbar_dx2 = (T)a.hbar_dx2;
    T rmax = (T)0;
    int flags = 0;
    int nleft = 0, nstay = 0, nright = 0;
    // A row's new increments are stored at the start of the next row, just
    // before its prefetch: the wait for those loads then also covers a store
    // issued a whole row earlier, instead of one issued moments before.
    T pend = (T)0;
    int pend_i = -1;
    // Lanes whose step crosses a cell boundary (from d^(k) for the push, or
    // from d^(k+1) for the Seidel deposit) need the neighbour-cell terms; they
    // are few, so the row is computed with the own-cell terms only, and such a
    // lane's particle is queued (its index, in LDS) and redone with the full
    // terms once a whole row of them has gathered (the rest after the wave's
    // last row).  Without the queue every row holding one crossing lane would
    // run the neighbour code for all 64 lanes.
    const QueueW q = queue_of_wave(queue, wid);
    int qn = 0;   // queued particles (wave-uniform)
    auto redo = [&](int qb, int n) {   // queued particles qb .. qb + n - 1, with every term
        const bool qv = lane < n;
        const int qs = qb + (qv ? lane : 0);
        const int qi = q.i[qs];
        Lane<T> Lq;
        const double xq = q.x[qs];
        Lq.p0 = (T)q.p[qs];
        if constexpr (!explicit_start) Lq.d = (T)q.d[qs];
        if constexpr (SPIN) { Lq.sy = a.sy[qi]; Lq.sz = a.sz[qi]; }
        stage_gather<P, T, explicit_start, ADJ>(o1, Lq, xq, c, dt_dx, flags, dx_dt);
        const bool cr = __ballot(Lq.s != 0) != 0;
        T pq, dq;
        stage_push<P, T, ADJ, false, SPIN>(o1, rec, cr, Lq, dt, dt_dx, inv_dx, pq, dq, flags, nullptr, hbar_dx2);
        flags |= FLAG_QUEUED;
        if (qv) {
            if constexpr (keep_start) ((k & 1) ? a.d1 : a.d0)[qi] = Lq.d;
            dout[qi] = dq;
            rmax = fmax(rmax, fabs(dq - Lq.d));
        }
        const T w = qv ? (T)1 : (T)0;
        int sc;
        if constexpr (SEIDEL) {
            T tq;
            if constexpr (F64) end_point(xq, dq, c, tq, sc, flags);
            else end_point(Lq.t0, dq, tq, sc, flags);
            stage_deposit<P, T>(mo, __ballot(sc != 0) != 0, Lq.t0, tq, sc, w);
        } else {
            sc = Lq.s;
            stage_deposit<P, T>(mo, cr, Lq.t0, Lq.t1, Lq.s, w);
        }
        if constexpr (F64) {
            const uint64_t qmask = __builtin_amdgcn_ballot_w64(qv);
            nleft += __popcll(__builtin_amdgcn_ballot_w64(sc < 0) & qmask);
            nright += __popcll(__builtin_amdgcn_ballot_w64(sc > 0) & qmask);
            nstay += __popcll(__builtin_amdgcn_ballot_w64(sc == 0) & qmask);
        }
    };
    // The queue pays at high degree, where the neighbour terms cost more
    // (measured: 11 % faster at degree 5, 10 % slower at degree 3).  At degree
    // 3 a row with a crossing lane computes the neighbour terms for all lanes.
    if constexpr (P >= 4) {
        for (int row = wb; row < we; row += WAVE, ia += WAVE) {
            Lane<T> La;
            const double xi0 = nx;
            La.p0 = (T)np;
            La.d = from_float ? (T)nf : nd;
            La.sy = (T)nsy;
            La.sz = (T)nsz;
            const bool valid = ia < we;
            if (pend_i >= 0) dout[pend_i] = pend;
            {   // prefetch the next row (unconditionally: the last row reloads its last particle)
                const int il = min(ia + WAVE, we - 1);
                nx = a.xi[il];
                np = a.p[il];
                if constexpr (from_float) nf = d32in[il];
                else if constexpr (from_prev) nd = (T)dprev[il];
                else if constexpr (!explicit_start) nd = din[il];
                if constexpr (SPIN) { nsy = a.sy[il]; nsz = a.sz[il]; }
            }
            stage_gather<P, T, explicit_start, ADJ>(o1, La, xi0, c, dt_dx, flags, dx_dt);
            // own-cell terms for every lane; a crossing lane's result is discarded
            // (it stays finite: its end point is clamped into (-1, 2) and |d| < dt/dx < 1)
            T pa, dna;
            stage_push<P, T, ADJ, false, SPIN>(o1, rec, false, La, dt, dt_dx, inv_dx, pa, dna, flags, nullptr,
                                               hbar_dx2);
            bool cross = La.s != 0;
            T ta = La.t1;
            if constexpr (SEIDEL) {
                int sc;
                if constexpr (F64) end_point(xi0, dna, c, ta, sc, flags);
                else end_point(La.t0, dna, ta, sc, flags);
                cross = cross || sc != 0;
            }
            const bool live = valid && !cross;
            if (live) {
                if constexpr (keep_start) ((k & 1) ? a.d1 : a.d0)[ia] = La.d;
                rmax = fmax(rmax, fabs(dna - La.d));
            }
            pend = dna;
            pend_i = live ? ia : -1;
            // a live lane's step stays in the cell: own-cell deposit, and it stays
            stage_deposit<P, T>(mo, false, La.t0, ta, 0, live ? (T)1 : (T)0);
            const uint64_t lmask = __builtin_amdgcn_ballot_w64(live);
            if constexpr (F64) nstay += __popcll(lmask);
            const uint64_t dmask = __builtin_amdgcn_ballot_w64(valid && cross);
            if (dmask) {
                const uint64_t below = lane == 0 ? 0ull : (~0ull >> (WAVE - lane));
                if (valid && cross) {
                    const int qs = qn + __popcll(dmask & below);
                    q.i[qs] = ia;
                    q.x[qs] = xi0;
                    q.p[qs] = (double)La.p0;
                    q.d[qs] = (double)La.d;
                }
                qn += __popcll(dmask);
                if (qn >= WAVE) {
                    redo(0, WAVE);
                    qn -= WAVE;
                    if (lane < qn) {   // move the rest to the front
                        const int vi = q.i[WAVE + lane];
                        const double vx = q.x[WAVE + lane], vp = q.p[WAVE + lane], vd = q.d[WAVE + lane];
                        q.i[lane] = vi;
                        q.x[lane] = vx;
                        q.p[lane] = vp;
                        q.d[lane] = vd;
                    }
                }
            }
        }
        if (qn > 0) redo(0, qn);
    } else {
        for (int row = wb; row < we; row += WAVE, ia += WAVE) {
            Lane<T> La;
            const double xi0 = nx;
            La.p0 = (T)np;
            La.d = from_float ? (T)nf : nd;
            La.sy = (T)nsy;
            La.sz = (T)nsz;
            const bool valid = ia < we;
            const uint64_t vmask = __builtin_amdgcn_ballot_w64(valid);
            if (pend_i >= 0) dout[pend_i] = pend;
            {   // prefetch the next row (unconditionally: the last row reloads its last particle)
                const int il = min(ia + WAVE, we - 1);
                nx = a.xi[il];
                np = a.p[il];
                if constexpr (from_float) nf = d32in[il];
                else if constexpr (from_prev) nd = (T)dprev[il];
                else if constexpr (!explicit_start) nd = din[il];
                if constexpr (SPIN) { nsy = a.sy[il]; nsz = a.sz[il]; }
            }
            stage_gather<P, T, explicit_start, ADJ>(o1, La, xi0, c, dt_dx, flags, dx_dt);
            const bool cross1 = __ballot(La.s != 0) != 0;
            T pa, dna;
            stage_push<P, T, ADJ, false, SPIN>(o1, rec, cross1, La, dt, dt_dx, inv_dx, pa, dna, flags, nullptr,
                                               hbar_dx2);
            if (valid) {
                if constexpr (keep_start) ((k & 1) ? a.d1 : a.d0)[ia] = La.d;
                rmax = fmax(rmax, fabs(dna - La.d));
            }
            pend = dna;
            pend_i = valid ? ia : -1;
            const T w = valid ? (T)1 : (T)0;
            int sc;   // cell change of the increment a commit after this sweep would take
            if (SEIDEL) {
                T ta;
                if constexpr (F64) end_point(xi0, dna, c, ta, sc, flags);
                else end_point(La.t0, dna, ta, sc, flags);
                stage_deposit<P, T>(mo, __ballot(sc != 0) != 0, La.t0, ta, sc, w);
            } else {
                sc = La.s;
                stage_deposit<P, T>(mo, cross1, La.t0, La.t1, La.s, w);
            }
            if constexpr (F64) {
                nleft += __popcll(__builtin_amdgcn_ballot_w64(sc < 0) & vmask);
                nright += __popcll(__builtin_amdgcn_ballot_w64(sc > 0) & vmask);
                nstay += __popcll(__builtin_amdgcn_ballot_w64(sc == 0) & vmask);
            }
        }
    }
    if (pend_i >= 0) dout[pend_i] = pend;
    Moments<P> md;
    to_double<P>(mo, md);
    const double slot = moments_to_slots<P>(md);
    const double rm = wave_max_dpp((double)rmax);
    const int fl = flags;   // wave-uniform (set through wave_flag)
    double *out = a.part + ((size_t)item * nw + wid) * UnitI<P>::N;
    double v = slot;
    v = lane == P + 2 ? rm : v;
    v = lane == P + 3 ? (double)fl : v;
    if (lane < UnitI<P>::N) out[lane] = v;
    // the wave's mover counts; the commit forms the item totals and the
    // prefixes over waves itself, so waves end without waiting for each other
    if constexpr (F64)
        if (lane < 3) a.wcnt[((size_t)item * nw + wid) * 3 + lane] = lane == 0 ? nleft : (lane == 1 ? nstay : nright);
}

// One block per work item; the grid may exceed the item count (the count of a
// step enqueued ahead is only known on the device) and the extra blocks exit.
// One kernel per start mode (the host knows it), so that each is allocated the
// registers it needs rather than the most any mode needs.  ADJ: the adjoint
// scheme (FP64, Seidel map, explicit start or read).
template <int P, bool SEIDEL, typename T, int START, bool ADJ, bool SPIN = false>
__global__ void __launch_bounds__(MAX_BLOCK) k_sweep_I(SweepIArgs a) {
    __shared__ LdsRec<P, T> rec[3];   // cells c-1, c, c+1
    extern __shared__ double queue[];   // the waves' queues (degree >= 4)
    sweep_I_item<P, SEIDEL, T, START, ADJ, SPIN>(a, blockIdx.x, rec, queue);
}

// Sum of the wave partials of cell c (its items times wpi waves each): the P+2
// current slots, the max of the residuals and the OR of the flags.
template <int P>
__device__ __forceinline__ void cell_partials_I(const ItemList &it, bool one_each, const double *part, int c,
                                                int wpi, double (&v)[P + 2], double &rx, int &flags) {
#pragma unroll
    for (int q = 0; q < P + 2; ++q) v[q] = 0.0;
    // with one item per cell the item index is the cell: no dependent load
    const int u0 = (one_each ? c : it.cell_first[c]) * wpi;
    const int u1 = one_each ? u0 + wpi : it.cell_first[c + 1] * wpi;
    for (int u = u0; u < u1; ++u) {
        const double *w = part + (size_t)u * UnitI<P>::N;
#pragma unroll
        for (int q = 0; q < P + 2; ++q) v[q] += w[q];
        rx = fmax(rx, w[P + 2]);
        flags |= (int)w[P + 3];
    }
}

// cell_partials_I with one item per cell and WPI waves per item: unit c * WPI + w,
// all loads issued before any is used.
template <int P, int WPI>
__device__ __forceinline__ void cell_partials_one(const double *part, int c, double (&v)[P + 2], double &rx,
                                                  int &flags) {
    constexpr int N = UnitI<P>::N;
    double u[WPI][N];
#pragma unroll
    for (int w = 0; w < WPI; ++w)
#pragma unroll
        for (int q = 0; q < N; ++q) u[w][q] = part[((size_t)c * WPI + w) * N + q];
#pragma unroll
    for (int q = 0; q < P + 2; ++q) {
        v[q] = 0.0;
#pragma unroll
        for (int w = 0; w < WPI; ++w) v[q] += u[w][q];
    }
#pragma unroll
    for (int w = 0; w < WPI; ++w) {
        rx = fmax(rx, u[w][P + 2]);
        flags |= (int)u[w][P + 3];
    }
}

template <int P>
__device__ __forceinline__ void cell_partials_one(const double *part, int c, int wpi, double (&v)[P + 2],
                                                  double &rx, int &flags) {
    switch (wpi) {
        case 1: cell_partials_one<P, 1>(part, c, v, rx, flags); break;
        case 2: cell_partials_one<P, 2>(part, c, v, rx, flags); break;
        case 3: cell_partials_one<P, 3>(part, c, v, rx, flags); break;
        default: cell_partials_one<P, 4>(part, c, v, rx, flags); break;
    }
}

// The commit's destinations need no scan over the cells.  A particle moves at
// most one cell, so the particles that end in cells [0, c) are those that
// started there, plus the left-movers of cell c and the right-movers of cell
// M-1 (periodic), minus the right-movers of cell c-1 and the left-movers of
// cell 0:
//   nstart[c] = start[c] + L_c - R_{c-1} + R_{M-1} - L_0,   nstart[0] = 0,
// with start[c] the first particle of cell c in the current order and L, S, R
// a cell's left-movers, stayers and right-movers.  Each cell's value (and its
// new count R_{c-1} + S_c + L_{c+1}) is local, so the field kernel after each
// FP64 sweep forms them for its cells from the sweep's mover counts: the last
// field kernel to run is that of the sweep the commit takes.  Only an item
// list with other than one item per cell needs a prefix over the cells; the
// commit builds it.

// L, S, R of cell c and its first particle in the current order.  With one
// item per cell only the cell index addresses the loads; otherwise they follow
// the list, and base gets each item's movers before it in its cell.
__device__ __forceinline__ void cell_movers(const ItemList &it, const int32_t *wcnt, int wpi, int32_t *base,
                                            bool one_each, int c, bool write_base, int (&t)[3], int &start) {
    if (one_each) {
        start = it.begin[c];
        const int32_t *q = wcnt + (size_t)c * wpi * 3;   // the cell's wpi triples, contiguous
        t[0] = t[1] = t[2] = 0;
        for (int w = 0; w < wpi; ++w) { t[0] += q[3 * w]; t[1] += q[3 * w + 1]; t[2] += q[3 * w + 2]; }
        return;
    }
    const int lo = it.cell_first[c], hi = it.cell_first[c + 1];
    start = it.begin[lo];   // an empty cell starts where the next item does
    t[0] = t[1] = t[2] = 0;
    for (int i = lo; i < hi; ++i) {
        if (write_base) { base[i * 3 + 0] = t[0]; base[i * 3 + 1] = t[1]; base[i * 3 + 2] = t[2]; }
        for (int w = 0; w < wpi; ++w) {
            const int32_t *q = wcnt + ((size_t)i * wpi + w) * 3;
            t[0] += q[0]; t[1] += q[1]; t[2] += q[2];
        }
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
    // commit data: L, S, R of cells cb0-2 .. cb0+TILE, the current start of
    // cells cb0-1 .. cb0+TILE (both mod M), L, S, R of cells 0 and M-1
    __shared__ int tl[TILE + 3][3];
    __shared__ int sl[TILE + 2];
    __shared__ int ends[2][3];
    __shared__ int notone_s;
    DevStatus *st = a.st;
    // the status is tested once the loads that do not depend on it are issued
    const int sgate = st->gate, sflags = st->flags, skconv = st->kconv;
    const bool one_each = a.items.n_items[1] != 0;
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
    double *enw = enl + FIELD_OUT;   // e_x^n on the block's cells
    const double *ek = k == 0 ? a.en : ((k & 1) ? a.ek1 : a.ek0);
    // One memory round trip before the status test: this quad's output cell,
    // the first taps, e_x^n on the block's cells and the first round of
    // partials, loaded as if item c were cell c (in bounds whatever the list
    // holds) and kept if it is (a list with several items per cell is followed
    // only after the test).  The empty asm keeps the loads above the branch.
    const int quad = threadIdx.x >> 2, ql = threadIdx.x & 3;
    const int jq = j0 + quad, jqm = imod(jq, M);
    const int t0 = threadIdx.x;
    const double en_q = a.en[jqm + HALO];
    const double ek_q = ek[jqm + HALO];
    const double tap0 = a.taps[min(t0, a.ntaps - 1)];
    const double enw0 = a.en[imod(j0 + min(t0, FIELD_OUT - 1), M) + HALO];
    double rx0 = 0.0, v0[NS];
    int fl0 = 0;
    cell_partials_one<P>(a.part, imod(clo + min(t0, clen - 1), M), a.wpi, v0, rx0, fl0);
    asm volatile("" ::"v"(en_q), "v"(ek_q), "v"(tap0), "v"(enw0), "v"(rx0), "v"(fl0));
#pragma unroll
    for (int q = 0; q < NS; ++q) asm volatile("" ::"v"(v0[q]));
    if (!sgate | sflags | (skconv >= 0)) return;
    // commit data (FP64 sweeps): thread t < TILE + 3 takes the movers of cell
    // cb0 - 2 + t and the start of cell cb0 - 1 + t, threads 254 and 255 those
    // of cells 0 and M - 1.  Their loads are issued here and used once the
    // partials are summed.
    const bool cw = k >= a.first64;
    const int cb0 = blockIdx.x * TILE;
    const int mcell = t0 >= 254 ? (t0 == 254 ? 0 : M - 1) : imod(cb0 - 2 + min(t0, TILE + 2), M);
    const int scell = imod(cb0 - 1 + min(t0, TILE + 1), M);
    const bool mload = cw && (t0 < TILE + 3 || t0 >= 254), sload = cw && t0 < TILE + 2;
    const bool own = t0 >= 2 && t0 < TILE + 2 && cb0 - 2 + t0 < M;   // base for the block's own cells
    // Read as if item c were cell c (in bounds for any list), with no branch
    // but the lane's own predicate, so that nothing waits for them before use;
    // a list with several items per cell is followed where they are used.
    int raw[MAX_WAVES][3] = {}, st0 = 0;
    if (mload) {
        const int32_t *q = a.wcnt + (size_t)mcell * a.wpi * 3;   // the cell's wpi triples, contiguous
#pragma unroll
        for (int w = 0; w < MAX_WAVES; ++w) {
            const int ww = min(w, a.wpi - 1);
            raw[w][0] = q[3 * ww]; raw[w][1] = q[3 * ww + 1]; raw[w][2] = q[3 * ww + 2];
        }
    }
    if (sload) st0 = a.items.begin[scell];
    if (t0 < a.ntaps) tp[t0] = tap0;
    for (int t = t0 + blockDim.x; t < a.ntaps; t += blockDim.x) tp[t] = a.taps[t];
    if (t0 < FIELD_OUT) enw[t0] = enw0;
    double rx = 0.0;
    int flags = 0;
    if (one_each && t0 < clen) {
        rx = rx0;
        flags = fl0;
    }
    for (int t = threadIdx.x; t < clen; t += blockDim.x) {
        double v[NS];
        if (one_each && t == t0) {
#pragma unroll
            for (int q = 0; q < NS; ++q) v[q] = v0[q];
        } else {
            cell_partials_I<P>(a.items, one_each, a.part, imod(clo + t, M), a.wpi, v, rx, flags);
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) cp[q * clen + t] = v[q];   // slot-major: consecutive cells, banks
    }
    __syncthreads();
    for (int t = threadIdx.x; t < slen; t += blockDim.x) {
        double sum = 0.0;
#pragma unroll
        for (int r = 0; r < NS; ++r) sum += cp[(P + 1 - r) * clen + t + r];   // cell (j-1+r): slot P+1-r
        S[t] = sum;
    }
    if (cw) {
        int mv[3] = {0, 0, 0};
        if (one_each) {
#pragma unroll
            for (int w = 0; w < MAX_WAVES; ++w) {
                const int u = w < a.wpi ? 1 : 0;
                mv[0] += u * raw[w][0]; mv[1] += u * raw[w][1]; mv[2] += u * raw[w][2];
            }
        } else {   // through the item list; base for the block's own cells
            int dummy;
            if (mload) cell_movers(a.items, a.wcnt, a.wpi, a.base, false, mcell, own, mv, dummy);
            if (sload) st0 = a.items.begin[a.items.cell_first[scell]];   // an empty cell starts where the next item does
        }
        if (t0 < TILE + 3) { tl[t0][0] = mv[0]; tl[t0][1] = mv[1]; tl[t0][2] = mv[2]; }
        if (t0 >= 254) { ends[t0 - 254][0] = mv[0]; ends[t0 - 254][1] = mv[1]; ends[t0 - 254][2] = mv[2]; }
        if (t0 < TILE + 2) sl[t0] = st0;
        if (t0 == 0) notone_s = 0;
    }
    __syncthreads();
    // the commit data of the block's cells, stored before the convolution so
    // that the stores complete behind it
    if (cw && t0 < TILE && cb0 + t0 < M) {
        // new start of cell cb0 + q (mod M), q in [-1, TILE]: slots q + 1 of sl
        // and q + 2 of tl (L of the cell), q + 1 of tl (R of the cell before)
        const int c = cb0 + t0;
        const int wrap = ends[1][2] - ends[0][0];   // R_{M-1} - L_0
        auto nstart_of = [&](int q) {
            const int cq = cb0 + q;
            return (cq == 0 || cq == M) ? 0 : sl[q + 1] + tl[q + 2][0] - tl[q + 1][2] + wrap;
        };
        const int ns = nstart_of(t0), nsm = nstart_of(t0 - 1), nsp = nstart_of(t0 + 1);
        const int Rm = tl[t0 + 1][2], Sm = tl[t0 + 1][1], Rmm = tl[t0][2];
        const int Lp = c == M - 1 ? ends[0][0] : tl[t0 + 3][0];
        const int cnt = Rm + tl[t0 + 2][1] + Lp;   // R_{c-1} + S_c + L_{c+1}
        a.cbase[c * 3 + 0] = nsm + Rmm + Sm;      // left-movers: after R_{c-2} and S_{c-1} in cell c-1
        a.cbase[c * 3 + 1] = ns + Rm;             // stayers: after R_{c-1}
        a.cbase[c * 3 + 2] = nsp;                 // right-movers: first in cell c+1
        a.nstart[c] = ns;
        a.nstart[M + 1 + c] = cnt;
        a.items_next.cell[c] = c;                 // the list if every cell has one item
        a.items_next.begin[c] = ns;
        a.items_next.cell_first[c] = c;
        if (items_of(cnt, a.chunk) != 1) notone_s = 1;
    }
    double *eout = (k & 1) ? a.ek0 : a.ek1;
    double *Eout = ((k + 1) & 1) ? a.coefE1 : a.coefE0;
    double re = 0.0;
    {
        // S_{j - m} for m = mlo + i sits at S[quad + mhi - m] = S[quad + ntaps - 1 - i]
        // (four chains per lane, so that several LDS reads are in flight)
        const double *Sq = S + quad + a.ntaps - 1;
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
        int i = ql;
        for (; i + 12 < a.ntaps; i += 16) {
            acc0 = fma(tp[i], Sq[-i], acc0);
            acc1 = fma(tp[i + 4], Sq[-i - 4], acc1);
            acc2 = fma(tp[i + 8], Sq[-i - 8], acc2);
            acc3 = fma(tp[i + 12], Sq[-i - 12], acc3);
        }
        for (; i < a.ntaps; i += 4) acc0 = fma(tp[i], Sq[-i], acc0);
        double conv = (acc0 + acc1) + (acc2 + acc3);
        conv += dpp_d<0xB1>(conv);   // quad_perm [1,0,3,2]
        conv += dpp_d<0x4E>(conv);   // quad_perm [2,3,0,1]
        const double enew = en_q - a.w * conv;
        if (ql == 0) {
            enl[quad] = enew;
            if (quad >= P - 1 && jq < M) {
                store_padded(eout, M, jqm, enew);
                if (cw) store_padded(a.ex_next, M, jqm, enew);   // e_x^{n+1} if this sweep is committed
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
            make_recE<P>([&](int jj) { return 0.5 * (enw[jj - j0] + enl[jj - j0]); }, j, r);
            for (int i = 0; i < P; ++i) store_record(Eout, M, j, RecE<P>::N, i, r[i]);
        }
    }
    re = wave_max_dpp(re);
    rx = wave_max_dpp(rx);
    flags = wave_or_bits<4>(flags);
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
        if (flags & FLAG_ERRORS) atomicOr(&st->flags, flags & FLAG_ERRORS);
        if (flags & FLAG_QUEUED) atomicOr(&st->queued, 1);
        if (cw && notone_s) atomicOr(&st->scan_multi, 1);
        if (blockIdx.x == 0) {   // clear the slots field kernel k+1 accumulates into
            st->rx_bits[(k + 1) & 1] = 0ull;
            st->re_bits[(k + 1) & 1] = 0ull;
        }
    }
}

// Records of a substep start: A-records of a_perp and E-records of e.
template <int P>
__global__ void __launch_bounds__(256) k_prep_records(DevStatus *st_init, const double *ay, const double *az,
                                                      const double *e, double *coefA, double *coefE, int M) {
    if (st_init && blockIdx.x == 0 && threadIdx.x == 0) init_status(st_init, nullptr);
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
};

__device__ __forceinline__ CommitPick commit_pick(const CommitIArgs &a, int kc) {
    CommitPick r;
    if (a.seidel) {
        r.d = ((kc + 1) & 1) ? a.d1 : a.d0;     // delta^(kc+1)
        r.coefE = ((kc + 1) & 1) ? a.coefE1 : a.coefE0;
    } else {
        r.d = (kc & 1) ? a.d1 : a.d0;           // delta^(kc)
        r.coefE = (kc & 1) ? a.coefE1 : a.coefE0;
    }
    return r;
}

// One training pair of the learned warm start: the particle's features at the
// step start and the converged increments (see mlp.hip for the definitions).
template <int P>
__device__ __forceinline__ void record_pair(const CommitIArgs &a, const Own<P, double> &o, int c, int pid, double xi0,
                                            double p0, double d, double p1) {
    constexpr int D = ws_d(P);
    const int64_t slot = a.rec.base + pid / a.rec.stride;
    if (slot >= a.rec.cap) return;
    const double t0 = xi0 - (double)c;
    const double Ay = horner<P + 1>(o.ay, t0), Az = horner<P + 1>(o.az, t0);
    const double g0 = sqrt(1.0 + p0 * p0 + Ay * Ay + Az * Az);
    float *f = a.rec.feat + slot * D;
    f[0] = (float)(t0 - 0.5);
    f[1] = (float)p0;
    f[2] = (float)(g0 - 1.0);
    for (int j = -P; j <= P + 1; ++j) {
        const int jj = imod(c + j, a.M) + HALO;
        f[3 + j + P] = (float)a.rec.ay[jj];
        f[3 + 2 * (P + 1) + j + P] = (float)a.rec.az[jj];
        f[3 + 4 * (P + 1) + j + P] = (float)a.rec.ex[jj];
    }
    a.rec.targ[slot * 2] = (float)((d * a.dx - a.dt * p0 / g0) / (a.dt * a.dt));
    a.rec.targ[slot * 2 + 1] = (float)((p1 - p0) / a.dt);
}

// Block 0 of the commit: the Subsystem II status, reset and gated on the commit,
// and, when the commit happens, the new item list completed (or built whole
// when some cell of the new order has other than one item), its count and the
// commit mark.  Every thread of the block calls it.
__device__ __forceinline__ void commit_finish(const CommitIArgs &a, int kc, int multi, int *lds) {
    if (threadIdx.x == 0 && a.stII) {   // Subsystem II may run only after this commit
        init_status(a.stII, nullptr);
        a.stII->gate = kc >= 0 ? 1 : 0;
    }
    if (kc < 0) return;
    const int M = a.M;
    if (multi && a.list_kernel) {   // k_commit_list builds the list
        if (threadIdx.x == 0) a.st->committed = 1;
        return;
    }
    int n_next = M;
    if (multi) {
        n_next = build_items(a.nstart + (M + 1), a.nstart, M, a.chunk, a.N, a.items_next, lds);
    } else if (threadIdx.x == 0) {
        a.items_next.cell_first[M] = M;
        a.items_next.begin[M] = (int)a.N;
        a.items_next.n_items[0] = M;
        a.items_next.n_items[1] = 1;
    }
    if (threadIdx.x == 0) {
        a.st->n_items_next = n_next;
        a.st->scan_multi = 0;
        a.st->committed = 1;
    }
}

// The new item list when some cell of the new order has other than one item,
// built by one 1024-thread block after the scatter (launched when the current
// order has such cells; otherwise block 0 of the scatter builds it).
__global__ void __launch_bounds__(1024) k_commit_list(CommitIArgs a) {
    __shared__ int lds[16];
    const int committed = a.st->committed, multi = a.st->scan_multi;
    if (!committed || !multi) return;
    const int n_next = build_items(a.nstart + (a.M + 1), a.nstart, a.M, a.chunk, a.N, a.items_next, lds);
    if (threadIdx.x == 0) {
        a.st->n_items_next = n_next;
        a.st->scan_multi = 0;
    }
}

// Totals over the lanes of a wave of NV values per lane held in LDS, value u
// of lane i at col[u * stride + i]; lane u < NV returns total u.  A lane sums
// one value over a run of lanes (staggered, so that the lanes of a run read
// different banks), the runs' parts go to row 0 and lane u adds its value's
// parts, all in a fixed order.  Every thread of the block calls it (barriers);
// the caller has made the values visible.
template <int NV>
__device__ __forceinline__ double wave_totals_lds(double *col, int stride, int lane) {
    constexpr int G = WAVE / NV, S = (WAVE + G - 1) / G;   // runs per value, lanes per run
    const int u = lane % NV, g = lane / NV;
    double part = 0.0;
    if (g < G) {
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const int src = g * S + (i + u) % S;
            if (src < WAVE) part += col[u * stride + src];
        }
    }
    __syncthreads();   // every run is read before row 0 is overwritten
    if (g < G) col[g * NV + u] = part;
    __syncthreads();
    double t = 0.0;
    if (lane < NV)
#pragma unroll
        for (int k = 0; k < G; ++k) t += col[k * NV + lane];
    return t;
}

// Moves every particle to its place in the new cell order, with the committed
// momentum re-evaluated.  Each wave handles the same run of rows as in the
// sweep, so its movers of each kind are consecutive from its cell's base (the
// field kernel of the committed sweep formed it; an item adds the movers of
// the cell's earlier items, a wave those of the item's earlier waves); ballots
// rank them within a row.
//
// With part2 set the commit also forms the particle deposit of the first
// Subsystem II iterate.  That iterate needs only the committed (x, p) and the
// records of a^n and a^(0) = a^n - dt e^n, all fixed before Subsystem I
// starts, so the particle pass of iterate 0 is done here, on values already in
// registers, instead of by a pass of its own over the new order.  Each particle
// adds c_y t^j, c_z t^j (t its coordinate in the cell it lands in) to the
// moments of that cell: its own (in registers), or the neighbour a mover
// enters (per-lane slots in dynamic LDS, lane-major, so that the rare movers
// cost no registers across the loop).  A^n and gamma^n at the end point are
// those the push evaluated.  A wave writes 2 (P+3) slots, V0 indices
// c-P-1 .. c+1 for each component.
//
// ADJ: the commit of the adjoint scheme.  The committed increment is the
// sweep's delta^(kc+1); the momentum is the P that increment stands for (the
// closed form of adjoint_momentum), so no push is evaluated again.  It forms no
// Subsystem II deposit (the adjoint substep closes a step) and records nothing.
template <int P, bool RECORD, bool ADJ, bool SPIN>
__device__ __forceinline__ void commit_scatter_item(const CommitIArgs &a, int item) {
    static_assert(!(ADJ && RECORD), "pairs are recorded from the scheme's own commit");
    static_assert(!(SPIN && RECORD), "the learned warm start runs without spin");
    constexpr int NA = RecA<P>::N;
    __shared__ LdsRec<P, double> rec[3];   // cells c-1, c, c+1
    __shared__ double rk[3][NA];           // a^(0) records of cells c-1, c, c+1 (part2)
    __shared__ int lds[16];
    extern __shared__ double mvl[];        // part2: per wave [left, right][y, z][P+1][64 lanes] mover moments
    // item count, status words, the residual slots of the last sweep and the
    // item description in one memory round trip
    const int n_items = a.items.n_items[0], one_each = a.items.n_items[1];
    const int sgate = a.st->gate, sflags = a.st->flags, skconv = a.st->kconv, smulti = a.st->scan_multi;
    const unsigned long long rxb = a.st->rx_bits[(a.nsweeps - 1) & 1], reb = a.st->re_bits[(a.nsweeps - 1) & 1];
    const int c = a.items.cell[item];
    const int beg = a.items.begin[item], end = a.items.begin[item + 1];
    asm volatile("" ::"s"(n_items), "s"(one_each), "s"(sgate), "s"(sflags), "s"(skconv), "s"(smulti), "s"(rxb),
                 "s"(reb), "s"(c), "s"(beg), "s"(end));
    // the converged sweep: recorded by an earlier sweep's start, else the test
    // of the last enqueued sweep, made here by every block (block 0 records it)
    int kc = -1;
    if (sgate && !sflags) {
        kc = skconv;
        if (kc < 0 && prev_converged(a.st, a.nsweeps, a.first64, a.dx, a.tol, item == 0 && threadIdx.x == 0, rxb, reb))
            kc = a.nsweeps - 1;
    }
    if (item == 0) commit_finish(a, kc, smulti, lds);
    if (item >= n_items || kc < 0) return;   // the commit runs on a converged, unflagged substep
    const CommitPick pk = commit_pick(a, kc);
    const int M = a.M;
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
    int wb, we;
    wave_range(beg, end, wid, nw, wb, we);
    stage_records<P, double>(rec, a.coefA, pk.coefE, c);
    const bool dep2 = a.part2 != nullptr;
    if (dep2)
        for (int t = threadIdx.x; t < 3 * NA; t += blockDim.x)
            (&rk[0][0])[t] = a.coefAk0[(size_t)(rec_index(c) - 1) * NA + t];
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    const int32_t *cb = a.cbase + (size_t)c * 3;
    int run0 = cb[0], run1 = cb[1], run2 = cb[2];
    if (!one_each) {   // movers of the cell's earlier items
        const int32_t *bs = a.base + (size_t)item * 3;
        run0 += bs[0]; run1 += bs[1]; run2 += bs[2];
    }
    for (int w = 0; w < wid; ++w) {   // movers of the item's earlier waves
        const int32_t *n = a.wcnt + ((size_t)item * nw + w) * 3;
        run0 += n[0]; run1 += n[1]; run2 += n[2];
    }
    int flags = 0;
    __syncthreads();
    Own<P, double> o1;
    own_from_lds<P, double>(rec, o1);
    double my[P + 1], mz[P + 1];               // moments of the particles that stay in cell c
#pragma unroll
    for (int j = 0; j <= P; ++j) { my[j] = 0.0; mz[j] = 0.0; }
    // the wave's mover slots: value u of lane l at col[u * WAVE + l] (a constant
    // stride, so the slots of one lane provably differ)
    constexpr int NM = 4 * (P + 1);
    double *const col = mvl + (size_t)wid * NM * WAVE;
    if (dep2)
#pragma unroll
        for (int u = 0; u < NM; ++u) col[u * WAVE + lane] = 0.0;
    // the next row's loads are issued before the current row is computed
    double nx = 0.0, np = 0.0, nd = 0.0;
    double nsy = 0.0, nsz = 0.0;   // spin (SPIN)
    int32_t nid = 0;
    if (wb < we) {
        const int il = min(wb + lane, we - 1);
        nx = a.cur.xi[il];
        np = a.cur.p[il];
        nd = pk.d[il];
        nid = a.cur.id[il];
        if constexpr (SPIN) { nsy = a.cur.sy[il]; nsz = a.cur.sz[il]; }
    }
    __builtin_amdgcn_s_waitcnt(0);
    for (int r0 = wb; r0 < we; r0 += WAVE) {
        const int i = r0 + lane;
        const bool valid = i < we;
        const double xi0 = nx, p0 = np, d = nd;
        const double sy0 = nsy, sz0 = nsz;
        const int32_t pid = nid;
        {
            const int il = min(i + WAVE, we - 1);
            nx = a.cur.xi[il];
            np = a.cur.p[il];
            nd = pk.d[il];
            nid = a.cur.id[il];
            if constexpr (SPIN) { nsy = a.cur.sy[il]; nsz = a.cur.sz[il]; }
        }
        // the committed momentum: the map evaluated at the committed increment
        // (adjoint: the momentum that increment stands for)
        Lane<double> La;
        La.p0 = p0;
        La.d = d;
        La.sy = sy0;
        La.sz = sz0;
        double p1, dn;
        PushEnd<double> pe{0.0, 0.0, 0.0};
        stage_gather<P, double, false, ADJ>(o1, La, xi0, c, a.dt_dx, flags, a.dx_dt);
        const bool anymove = __ballot(La.s != 0) != 0;
        if constexpr (ADJ) {
            p1 = La.P;
            wave_flag(flags, !(fabs(p1) < 1.0e300), FLAG_NONFINITE);
        } else {
            stage_push<P, double, false, true, SPIN, false>(o1, rec, anymove, La, a.dt, a.dt_dx, a.inv_dx, p1, dn,
                                                            flags, &pe, a.hbar_dx2);
        }
        const int t = valid ? La.s + 1 : -1;   // 0 left, 1 stay, 2 right
        double xin = xi0 + d;
        if (xin >= (double)M) xin -= (double)M;
        else if (xin < 0.0) {
            xin += (double)M;
            if (xin >= (double)M) xin = __longlong_as_double(__double_as_longlong((double)M) - 1);
        }
        if constexpr (RECORD)
            if (valid && pid % a.rec.stride == a.rec.phase) record_pair<P>(a, o1, c, pid, xi0, p0, d, p1);
        if (!ADJ && dep2) {
            // the cell the particle lands in and its coordinate there, as the
            // particle pass over the new order would take them
            int dc = c + La.s;
            dc = dc < 0 ? dc + M : (dc >= M ? dc - M : dc);
            double tn = xin - (double)dc;
            wave_flag(flags, !(tn >= 0.0), FLAG_ORDER);
            wave_flag(flags, !(tn < 1.0), FLAG_ORDER);
            tn = fmin(fmax(tn, 0.0), 1.0);
            // a^(0) of the destination cell (per lane if the row has a mover)
            const double *ky = rk[anymove ? La.s + 1 : 1];
            const double Aky = horner<P + 1>(ky, tn), Akz = horner<P + 1>(ky + P + 1, tn);
            const double gk = fsqrt(fma(p1, p1, 1.0) + Aky * Aky + Akz * Akz);
            const double inv = (valid ? 1.0 : 0.0) * frcp(pe.g11 + gk);
            const double cy = (Aky + pe.A1y) * inv, cz = (Akz + pe.A1z) * inv;
            if (anymove) {
                const double ws = La.s == 0 ? 1.0 : 0.0;
                double tp = 1.0;
#pragma unroll
                for (int j = 0; j <= P; ++j) {
                    my[j] = fma(cy * ws, tp, my[j]);
                    mz[j] = fma(cz * ws, tp, mz[j]);
                    tp *= tn;
                }
                if (La.s != 0) {   // all loads, then all stores: one LDS round trip
                    double *mq = col + (La.s > 0 ? 2 * (P + 1) : 0) * WAVE + lane;
                    double v[2 * (P + 1)];
#pragma unroll
                    for (int u = 0; u < 2 * (P + 1); ++u) v[u] = mq[u * WAVE];
                    tp = 1.0;
#pragma unroll
                    for (int j = 0; j <= P; ++j) {
                        v[j] = fma(cy, tp, v[j]);
                        v[P + 1 + j] = fma(cz, tp, v[P + 1 + j]);
                        tp *= tn;
                    }
#pragma unroll
                    for (int u = 0; u < 2 * (P + 1); ++u) mq[u * WAVE] = v[u];
                }
            } else {
                double tp = 1.0;
#pragma unroll
                for (int j = 0; j <= P; ++j) {
                    my[j] = fma(cy, tp, my[j]);
                    mz[j] = fma(cz, tp, mz[j]);
                    tp *= tn;
                }
            }
        }
        const unsigned long long b0 = __ballot(t == 0), b1 = __ballot(t == 1), b2 = __ballot(t == 2);
        if (valid) {
            int dest;
            if (t == 0) dest = run0 + __popcll(b0 & lt);
            else if (t == 1) dest = run1 + __popcll(b1 & lt);
            else dest = run2 + __popcll(b2 & lt);
            a.nxt.xi[dest] = xin;
            a.nxt.p[dest] = p1;
            a.nxt.id[dest] = pid;
            if (a.dprev_out) a.dprev_out[dest] = d;
            if constexpr (SPIN) {   // Subsystem I leaves the spins as they are
                a.nxt.sx[dest] = a.cur.sx[i];
                a.nxt.sy[dest] = sy0;
                a.nxt.sz[dest] = sz0;
            }
        }
        run0 += __popcll(b0);
        run1 += __popcll(b1);
        run2 += __popcll(b2);
    }
    if (!ADJ && dep2) {   // block-uniform: every wave of the block takes part in the barriers
        // wave totals of the moments (movers from their LDS slots; then the
        // stayers, through the same slots), and lane q < 2 (P+3) forms slot q
        constexpr int NS1 = 2 * (P + 1);
        __syncthreads();   // the mover slots are complete
        const double tm = wave_totals_lds<NM>(col, WAVE, lane);
        double ty[3][P + 1], tz[3][P + 1];
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            ty[0][j] = readlane_d(tm, j);
            tz[0][j] = readlane_d(tm, P + 1 + j);
            ty[2][j] = readlane_d(tm, NS1 + j);
            tz[2][j] = readlane_d(tm, NS1 + P + 1 + j);
        }
        __syncthreads();   // row 0 of the slots (the parts) is read
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            col[j * WAVE + lane] = my[j];
            col[(P + 1 + j) * WAVE + lane] = mz[j];
        }
        __syncthreads();
        const double ts = wave_totals_lds<NS1>(col, WAVE, lane);
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            ty[1][j] = readlane_d(ts, j);
            tz[1][j] = readlane_d(ts, P + 1 + j);
        }
        constexpr Pieces<P> Bp{};
        constexpr int NW = P + 3;
        const int comp = lane / NW, qq = lane % NW;
        double out = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            // destination c - 1 + d: its slot q (V0 index c - 1 + d - P + q) is slot qq = q + d here
            const int q = qq - d, m = P - q;
            const bool in = q >= 0 && q <= P;
            const int mm = in ? m : 0;
#pragma unroll
            for (int j = 0; j <= P; ++j) out += in ? Bp.c[mm][j] * (comp == 0 ? ty[d][j] : tz[d][j]) : 0.0;
        }
        if (lane < 2 * NW) a.part2[((size_t)item * nw + wid) * 2 * NW + lane] = out;
    }
    if (flags && lane == 0) atomicOr(&a.st->flags, flags);   // flags is wave-uniform (wave_flag)
}

// One block per work item; the grid may exceed the item count (the count of a
// step enqueued ahead is only known on the device) and the extra blocks exit.
// RECORD: the step also writes training pairs of the learned warm start (a
// kernel of its own, so the plain one keeps its registers).
template <int P, bool RECORD, bool ADJ, bool SPIN = false>
__global__ void __launch_bounds__(MAX_BLOCK) k_commit_scatter(CommitIArgs a) {
    commit_scatter_item<P, RECORD, ADJ, SPIN>(a, blockIdx.x);
}


// ---- launchers ------------------------------------------------------------
template <int P, bool SEIDEL, typename T, bool ADJ, bool SPIN>
void launch_sweep_mode(const SweepIArgs &a, int grid, int block, size_t lds, hipStream_t s) {
    if (a.k == 0 && a.explicit_start)
        launch_k((k_sweep_I<P, SEIDEL, T, START_EXPLICIT, ADJ, SPIN>), dim3(grid), dim3(block), lds, s, a);
    else if (!ADJ && a.k == 0 && a.dprev)
        launch_k((k_sweep_I<P, SEIDEL, T, START_PREV, ADJ, SPIN>), dim3(grid), dim3(block), lds, s, a);
    else if constexpr (!SPIN && !ADJ && sizeof(T) == 8) {
        if (a.d32in)
            launch_k((k_sweep_I<P, SEIDEL, T, START_FLOAT, ADJ>), dim3(grid), dim3(block), lds, s, a);
        else
            launch_k((k_sweep_I<P, SEIDEL, T, START_READ, ADJ>), dim3(grid), dim3(block), lds, s, a);
    } else
        launch_k((k_sweep_I<P, SEIDEL, T, START_READ, ADJ, SPIN>), dim3(grid), dim3(block), lds, s, a);
}

// spin (a.sy non-null) runs the FP64 sweeps only; the host refuses the
// precision form and the learned start with spin
void launch_sweep_I(int P, bool seidel, bool fp32, bool adj, int grid, int block, hipStream_t s,
                    const SweepIArgs &a) {
    const size_t lds = P >= 4 ? queue_lds_bytes(block) : 0;   // the queue is used from degree 4 on
    const bool spin = a.sy != nullptr;
#define ECPIC_SW(PP)                                                                                  \
    case PP:                                                                                          \
        if (adj) {                                                                                    \
            if (spin) launch_sweep_mode<PP, true, double, true, true>(a, grid, block, lds, s);        \
            else launch_sweep_mode<PP, true, double, true, false>(a, grid, block, lds, s);            \
        } else if (fp32) {                                                                            \
            if (seidel) launch_sweep_mode<PP, true, float, false, false>(a, grid, block, lds, s);     \
            else launch_sweep_mode<PP, false, float, false, false>(a, grid, block, lds, s);           \
        } else if (spin) {                                                                            \
            if (seidel) launch_sweep_mode<PP, true, double, false, true>(a, grid, block, lds, s);     \
            else launch_sweep_mode<PP, false, double, false, true>(a, grid, block, lds, s);           \
        } else {                                                                                      \
            if (seidel) launch_sweep_mode<PP, true, double, false, false>(a, grid, block, lds, s);    \
            else launch_sweep_mode<PP, false, double, false, false>(a, grid, block, lds, s);          \
        }                                                                                             \
        break;
    switch (P) { ECPIC_SW(2) ECPIC_SW(3) ECPIC_SW(4) ECPIC_SW(5) }
#undef ECPIC_SW
}

void launch_field_I(int P, int M, hipStream_t s, const FieldIArgs &a) {
    const int grid = (M + FIELD_OUT - (P - 1) - 1) / (FIELD_OUT - (P - 1));
    const int slen = FIELD_OUT + a.ntaps - 1;
    const size_t lds = sizeof(double) * ((size_t)(slen + P + 1) * (P + 2) + slen + a.ntaps + 2 * FIELD_OUT);
#define ECPIC_F(PP) case PP: launch_k((k_field_I<PP>), dim3(grid), dim3(256), lds, s, a); break;
    switch (P) { ECPIC_F(2) ECPIC_F(3) ECPIC_F(4) ECPIC_F(5) }
#undef ECPIC_F
}

void launch_prep_records(int P, hipStream_t s, DevStatus *st, const double *ay, const double *az,
                         const double *e, double *coefA, double *coefE, int M) {
    const int grid = (M + 255) / 256;
#define ECPIC_PR(PP) \
    case PP: launch_k((k_prep_records<PP>), dim3(grid), dim3(256), 0, s, st, ay, az, e, coefA, coefE, M); break;
    switch (P) { ECPIC_PR(2) ECPIC_PR(3) ECPIC_PR(4) ECPIC_PR(5) }
#undef ECPIC_PR
}

void launch_commit_I(int P, bool adj, int grid, int block, hipStream_t s, const CommitIArgs &a) {
    const size_t lds = (a.part2 && !adj) ? sizeof(double) * 4 * (P + 1) * (size_t)block : 0;   // mover moments
    const bool spin = a.cur.sx != nullptr;
#define ECPIC_C(PP)                                                                                     \
    case PP:                                                                                            \
        if (adj) {                                                                                      \
            if (spin) launch_k((k_commit_scatter<PP, false, true, true>), dim3(grid), dim3(block), lds, s, a); \
            else launch_k((k_commit_scatter<PP, false, true>), dim3(grid), dim3(block), lds, s, a);     \
        } else if (spin)                                                                                \
            launch_k((k_commit_scatter<PP, false, false, true>), dim3(grid), dim3(block), lds, s, a);   \
        else if (a.rec.stride > 0)                                                                      \
            launch_k((k_commit_scatter<PP, true, false>), dim3(grid), dim3(block), lds, s, a);          \
        else                                                                                            \
            launch_k((k_commit_scatter<PP, false, false>), dim3(grid), dim3(block), lds, s, a);         \
        break;
    switch (P) { ECPIC_C(2) ECPIC_C(3) ECPIC_C(4) ECPIC_C(5) }
#undef ECPIC_C
    if (a.list_kernel) launch_k(k_commit_list, dim3(1), dim3(1024), 0, s, a);
}



}  // namespace ecpic
