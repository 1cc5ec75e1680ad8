// Host runtime of libecpic: context, device buffers, the Picard drivers of the
// two substeps, the Lie-Trotter step and the C-ABI entry points of ecpic.h.
//
// Picard driver.  Every kernel of a substep reads the device-resident status
// (sweep count, convergence, error flags) and turns into a no-op once the
// substep has converged or failed.  The host therefore enqueues as many
// sweeps as the previous step needed, then the commit, then Subsystem II
// (gated on Subsystem I's commit), and synchronises once per step; only when
// a substep needs more sweeps than predicted does it enqueue more.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/ecpic.h"
#include "internal.hpp"

namespace ecpic {
void launch_sweep_I(int P, bool seidel, bool fp32, bool adj, int grid, int block, hipStream_t s,
                    const SweepIArgs &a);
void launch_field_I(int P, int M, hipStream_t s, const FieldIArgs &a);
void launch_commit_I(int P, bool adj, int grid, int block, hipStream_t s, const CommitIArgs &a);
void launch_sweep_II(int P, int grid, int block, hipStream_t s, const SweepIIArgs &a);
void launch_field_II(int P, int M, hipStream_t s, const FieldIIArgs &a);
void launch_prep_records(int P, hipStream_t s, DevStatus *st, const double *ay, const double *az,
                         const double *e, double *coefA, double *coefE, int M);
void launch_begin_step(int P, hipStream_t s, DevStatus *stI, const DevStatus *gate_src, DevStatus *stII,
                       const double *ayn, const double *azn,
                       const double *eyn, const double *ezn, const double *exn, double dt, double *coefA,
                       double *coefE0, double *coefAk0, int do_II, const double *m0, const double *kr, double r2,
                       double ck, const double *taps, int ntaps, int mlo, int M, double *E0y, double *E0z);
void launch_step_join(int P, hipStream_t s, DevStatus *st, const DevStatus *stI, DevStatus *mirror,
                      DevStatus *stI_next, const double *eyn, const double *ezn, const double *ayn, const double *azn,
                      const double *ey0, const double *ey1, const double *ez0, const double *ez1, double *ey_next,
                      double *ez_next, double *ay_next, double *az_next, int nsweeps, double tol,
                      const double *exn_next, double dt, double *coefA, double *coefE0, double *coefAk0,
                      const double *m0, const double *kr, double r2, double ck, const double *taps, int ntaps,
                      int mlo, int M, double *E0y, double *E0z);
void launch_conv(int grid, hipStream_t s, const double *in, double *out, const double *taps, int ntaps, int mlo,
                 double alpha, int M);
void launch_commit_II(int grid, hipStream_t s, DevStatus *st, const DevStatus *stI, DevStatus *mirror,
                      const double *eyn, const double *ezn, const double *ayn, const double *azn, const double *ey0,
                      const double *ey1, const double *ez0, const double *ez1, double *ey_next, double *ez_next,
                      double *ay_next, double *az_next, double half_dt, int M, int nsweeps, double tol);
void launch_energy(int P, int grid, int block, hipStream_t s, const double *xi, const double *p, ItemList items,
                   const double *ay, const double *az, double *part);
void launch_energy_final(hipStream_t s, const double *part, const int32_t *n_items, double w, const double *ex,
                         const double *ey, const double *ez, const double *ay, const double *az,
                         const double *m0, const double *m1, const double *kr, int P, int M, double dx,
                         double *out);
void launch_charge(int P, int grid, int block, hipStream_t s, const double *xi, ItemList items, double *part,
                   double w, int M, double *rho);
void launch_gauss(hipStream_t s, const double *rho, const double *ex, const double *m1, int P, int M, double dx,
                  double *r, unsigned long long *maxbits);
void launch_poisson_rhs(hipStream_t s, const double *rho, int M, double dx, double *u);
void launch_pad(hipStream_t s, const double *in, double *out, double alpha, int M);
void launch_unpad(hipStream_t s, const double *in, double *out, int M);
void launch_init_particles(hipStream_t s, const double *x, const double *p, int64_t n, double L, double inv_dx,
                           int M, double *xi, double *pp, int32_t *key, int32_t *val);
void radix_sort(hipStream_t s, int32_t *k0, int32_t *v0, int32_t *k1, int32_t *v1, int64_t n, int key_bits,
                int32_t *hist, int32_t **kres, int32_t **vres);
void launch_gather_sorted(hipStream_t s, const int32_t *val, const double *xi_t, const double *p_t, int64_t n,
                          double *xi, double *p, int32_t *id);
void launch_count_cells(hipStream_t s, const int32_t *key, int64_t n, int32_t *count);
void launch_count_cells_xi(hipStream_t s, const double *xi, int64_t n, int M, int32_t *count);
void launch_items_from_counts(hipStream_t s, const int32_t *count, int32_t *start, int M, int chunk, int64_t N,
                              ItemList out);
void launch_unpermute(hipStream_t s, const double *xi, const double *p, const int32_t *id, int64_t n, double dx,
                      double *x_out, double *p_out);
void launch_deposit_segments(int P, hipStream_t s, const double *x0, const double *x1, int64_t n, double inv_dx,
                             double dx, double w, int M, double *J, int *flags);
void launch_copy(hipStream_t s, const double *in, double *out, int64_t n);
int noalloc_init(int dev);
void launch_spin_rotate(int P, int grid, hipStream_t s, const SpinArgs &a, int M);
void launch_spin_deposit(int P, int grid, hipStream_t s, const SpinArgs &a, int M);
void launch_spin_source(int P, hipStream_t s, const double *spart, const ItemList &items, int M, double coef,
                        const double *taps, int ntaps, int mlo, double *E0y, double *E0z);
void launch_spin_energy(int P, int grid, hipStream_t s, const SpinArgs &a, int M);
void launch_spin_in(hipStream_t s, const double *ix, const double *iy, const double *iz, const int32_t *id,
                    int64_t n, double *sx, double *sy, double *sz);
void launch_spin_out(hipStream_t s, const double *sx, const double *sy, const double *sz, const int32_t *id,
                     int64_t n, double *ox, double *oy, double *oz);
double *noalloc_scratch(int dev);
int noalloc_max_cells();
void launch_deposit_noalloc(int P, hipStream_t s, const double *x0, const double *x1, int64_t n, double inv_dx,
                            double dx, double w, int M, double *scr, double *J, int32_t *flags);
void launch_ws_predict(int P, int grid, int block, hipStream_t s, const SweepIArgs &a);
void launch_ws_init(int P, hipStream_t s, float *theta, uint64_t seed);
void launch_ws_stats(hipStream_t s, const float *feat, const float *targ, int64_t n, int D, float *mu, float *sd,
                     float *prange);
void launch_ws_step(int P, hipStream_t s, float *theta, float *m, float *v, const float *mu, const float *sd,
                    const float *feat, const float *targ, int64_t n, int direct, uint64_t seed, int64_t step, int B,
                    float *pgrad, float *ploss, float lr, int update, float *grad_out, float *loss_out);
void launch_ws_w2_bf16(int P, hipStream_t s, const float *theta, unsigned short *w2b);
void launch_ws_table(int P, hipStream_t s, const WsNet &net, const unsigned short *w2b, const double *coefA,
                     const double *ay, const double *az, const double *ex, int M, float *table);
}  // namespace ecpic

using namespace ecpic;

namespace {

// ---- closed-form matrix rows (Section 3.1) ---------------------------------
// The mass matrix of degree-d B-splines on a uniform grid is dx times the
// circulant whose row holds the cardinal B-spline of degree 2d+1 at the
// integers, i.e. Eulerian numbers A(2d+1, k)/(2d+1)!.
int64_t eulerian(int n, int k) {
    int64_t s = 0;
    for (int j = 0; j <= k; ++j) {
        int64_t b = 1;
        for (int q = 1; q <= j; ++q) b = b * (n + 1 - j + q) / q;   // C(n+1, j)
        int64_t pw = 1;
        for (int q = 0; q < n; ++q) pw *= (k + 1 - j);
        s += (j % 2 == 0) ? b * pw : -b * pw;
    }
    return s;
}

std::vector<double> mass_row(int d) {   // length 2d+1, dimensionless
    const int n = 2 * d + 1;
    double f = 1.0;
    for (int q = 2; q <= n; ++q) f *= q;
    std::vector<double> r(n);
    for (int k = 0; k < n; ++k) r[k] = (double)eulerian(n, k) / f;
    return r;
}

// First row of the periodic inverse of a symmetric banded circulant (row of
// half width b), from its eigenvalues lambda_k = sum_s row_s cos(2 pi k s/M):
// c_m = (1/M) sum_k cos(2 pi k m/M) / lambda_k.  Entries are kept while
// |c_m| > rel |c_0|; if that reaches half the period all M entries are used.
void inverse_taps(const std::vector<double> &row, int M, double rel, std::vector<double> &taps, int &mlo) {
    const int b = ((int)row.size() - 1) / 2;
    const long double tw = 2.0L * 3.14159265358979323846264338327950288L / (long double)M;
    std::vector<long double> inv(M);
    for (int k = 0; k < M; ++k) {
        long double lam = 0.0L;
        for (int s = -b; s <= b; ++s) lam += (long double)row[s + b] * cosl(tw * (long double)(((int64_t)k * (s + M)) % M));
        inv[k] = 1.0L / lam;
    }
    auto coef = [&](int m) {
        long double s = 0.0L;
        for (int k = 0; k < M; ++k) s += inv[k] * cosl(tw * (long double)(((int64_t)k * m) % M));
        return (double)(s / (long double)M);
    };
    const double c0 = coef(0);
    int T = 0;
    const int half = (M - 1) / 2;
    std::vector<double> c(1, c0);
    while (T < half) {
        const double v = coef(T + 1);
        c.push_back(v);
        ++T;
        if (std::fabs(v) < rel * std::fabs(c0) && T >= 2) break;
    }
    if (T >= half) {   // full period
        mlo = -half;
        const int cnt = M;
        taps.assign(cnt, 0.0);
        for (int i = 0; i < cnt; ++i) {
            const int m = mlo + i;
            taps[i] = coef(((m % M) + M) % M);
        }
        return;
    }
    mlo = -T;
    taps.assign(2 * T + 1, 0.0);
    for (int m = -T; m <= T; ++m) taps[m + T] = c[std::abs(m)];
}

struct Prof {
    bool on = false;
    std::map<std::string, std::pair<double, int64_t>> acc;
    std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e;
        hipEventCreate(&e);
        return e;
    }
};

}  // namespace

namespace ecpic {
constexpr int STEP_BATCH = 16;   // steps enqueued before the host reads their statuses
constexpr int MAX_WAVES_PER_ITEM = 4;
thread_local LaunchEvents g_launch_events;
}

struct ecpic_ctx {
    ecpic_config cfg{};
    int M = 0, P = 0, kmax = 50, block = 256, chunk = 2048, max_items = 0;
    int64_t N = 0;
    double L = 0, dx = 0, inv_dx = 0, w = 0, dt = 0, tol = 0;
    bool seidel = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;

    Particles pb[2]{};
    int cur = 0;
    double *dbuf[2]{};
    float *fbuf[2]{};          // single precision iterate (precision form)
    int k32 = 0;               // FP32 sweeps opening each Subsystem I substep

    // learned warm start: network (theta, Adam moments, normalisation), the
    // per-cell tables, recorded training pairs and training scratch
    int wsD = 0, wsNP = 0;
    float *ws_theta = nullptr, *ws_m = nullptr, *ws_v = nullptr;
    float *ws_norm = nullptr;  // mu[D+2] | sd[D+2] | prange[2]
    float *ws_table = nullptr;
    unsigned short *ws_w2b = nullptr;   // W2 in BF16 for the tables
    float *ws_feat = nullptr, *ws_targ = nullptr;
    int64_t ws_cap = 0, ws_base = 0;
    int ws_stride = 0, ws_phase = 0;
    float *ws_pgrad = nullptr, *ws_ploss = nullptr, *ws_loss = nullptr;
    int ws_pblocks = 0;
    bool ws_ready = false, ws_on = false;
    ItemList items[2]{};
    int icur = 0;
    int n_items_host = 0;
    int32_t *wcnt = nullptr, *base = nullptr, *cbase = nullptr, *nstart = nullptr;
    double *part = nullptr;

    // padded fields: [0]/[1] = current / next (swapped on commit)
    double *ex[2]{}, *ey[2]{}, *ez[2]{}, *ay[2]{}, *az[2]{};
    int exc = 0, trc = 0;
    double *ek[2]{};
    double *eyk[2]{}, *ezk[2]{};
    double *E0y = nullptr, *E0z = nullptr;
    double *coefA = nullptr, *coefE[2]{}, *coefAk[2]{};
    double *taps1 = nullptr, *tapsA = nullptr;
    int nt1 = 0, mlo1 = 0, ntA = 0, mloA = 0;
    // (M0 + dt^2 K / 4)^{-1} taps of every time step Subsystem II has run with
    // (tapsA, ntA, mloA point at those of the current dt)
    struct Taps {
        double *dev;
        int n, mlo;
    };
    std::map<double, Taps> tapsA_by_dt;
    std::vector<double> m0row, m1row, krow;

    // Statuses of up to STEP_BATCH steps enqueued ahead, pair by pair (Subsystem
    // I, II), with their pinned host mirrors; stI, stII, h, hdev point at the
    // pair of the step being enqueued or inspected.
    DevStatus *st_ring = nullptr;
    struct HostMirror {
        DevStatus I, II;
        int32_t n_items_next;
    } *h_ring = nullptr, *h_ring_dev = nullptr;   // host address, device address
    DevStatus *stI = nullptr, *stII = nullptr;
    HostMirror *h = nullptr;
    DevStatus *hdev = nullptr;   // device address of h->I (the Subsystem II commit writes it)
    static_assert(offsetof(HostMirror, II) == sizeof(DevStatus), "statuses are copied as one block");

    double *rho = nullptr, *rvec = nullptr, *uvec = nullptr, *out5 = nullptr, *part_e = nullptr;
    double *ex_save = nullptr;   // e_x at the start of a symmetric step (its rollback)
    bool symmetric = false;      // steps are I(dt/2), II(dt), adjoint I(dt/2)
    unsigned long long *maxbits = nullptr;
    int32_t *count = nullptr;
    bool have_particles = false;
    // previous-step warm start: the increment each commit took, in the new order
    bool ws_prev = false;
    double *dprev = nullptr;
    bool have_prev = false;   // dprev holds the increments of the current order
    int guessI = 4, guessII = 4, guessIadj = 4;
    bool exact_items = true;   // n_items_host is the item count of the step being enqueued
    // inside ecpic_step: the Subsystem I commit forms the particle deposit of
    // the first Subsystem II iterate, which then has no particle pass of its own
    bool fuse_II = false;
    // the Subsystem I substep being enqueued is the adjoint scheme (FP64 sweeps
    // from the explicit start, Seidel map)
    bool adjoint = false;
    int kI = 0, kII = 0;   // sweeps / iterations enqueued in the current substeps
    // spin: the particles carry spins (both buffers), hbar couples them
    bool spin = false;
    double hbar = 0.0;
    double *spart = nullptr;        // [max_items][2 deg] spin deposit per item (Subsystem II source)
    double *epart = nullptr;        // [max_items] Zeeman sum per item
    std::vector<double> h_epart;
    Prof prof;
};

namespace {

#define HIPCHK(x)                                                                                   \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) {                                                                     \
            std::fprintf(stderr, "ecpic: %s failed: %s (%s:%d)\n", #x, hipGetErrorString(e_), __FILE__, \
                         __LINE__);                                                                 \
            return ECPIC_EDEVICE;                                                                   \
        }                                                                                           \
    } while (0)

template <typename T>
int dalloc(T **p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc((void **)p, n * sizeof(T)) != hipSuccess) return ECPIC_ENOMEM;
    return ECPIC_OK;
}

void flush_prof(ecpic_ctx *c) {
    for (auto &pe : c->prof.pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
            auto &a = c->prof.acc[pe.first];
            a.first += ms;
            a.second += 1;
        }
        c->prof.pool.push_back(pe.second.first);
        c->prof.pool.push_back(pe.second.second);
    }
    c->prof.pending.clear();
}

// Launch timed when profiling is on: the events are taken by the kernels'
// dispatch packets (launch_k), so they span the kernels' execution only.
template <typename F>
void timed(ecpic_ctx *c, const char *name, F &&launch) {
    if (!c->prof.on) { launch(); return; }
    hipEvent_t a = c->prof.get(), b = c->prof.get();
    g_launch_events = {a, b};
    launch();
    g_launch_events = {};
    c->prof.pending.push_back({name, {a, b}});
}

int sync(ecpic_ctx *c) {
    HIPCHK(hipStreamSynchronize(c->stream));
    flush_prof(c);
    return ECPIC_OK;
}

int particle_grid(ecpic_ctx *c, bool exact) { return std::max(1, exact ? c->n_items_host : c->max_items); }

// Point the current statuses at pair j of the ring.
void set_slot(ecpic_ctx *c, int j) {
    c->stI = c->st_ring + 2 * j;
    c->stII = c->stI + 1;
    c->h = c->h_ring + j;
    c->hdev = c->h_ring_dev ? &c->h_ring_dev[j].I : nullptr;
}

// ---- Subsystem I ----------------------------------------------------------
SweepIArgs sweep_args(ecpic_ctx *c) {
    SweepIArgs a{};
    a.xi = c->pb[c->cur].xi;
    a.p = c->pb[c->cur].p;
    a.d0 = c->dbuf[0];
    a.d1 = c->dbuf[1];
    a.f0 = c->fbuf[0];
    a.f1 = c->fbuf[1];
    a.first64 = c->k32;
    a.items = c->items[c->icur];
    a.coefA = c->coefA;
    a.coefE0 = c->coefE[0];
    a.coefE1 = c->coefE[1];
    a.part = c->part;
    a.wcnt = c->wcnt;
    a.st = c->stI;
    a.dt = c->dt;
    a.dt_dx = c->dt / c->dx;
    a.dx_dt = c->dx / c->dt;
    a.inv_dx = c->inv_dx;
    a.dx = c->dx;
    a.tol = c->tol;
    a.explicit_start = 1;
    if (c->spin && c->hbar != 0.0) {   // the spin force (hbar = 0: the plain sweeps, spins untouched)
        a.sy = c->pb[c->cur].sy;
        a.sz = c->pb[c->cur].sz;
        a.hbar_dx2 = c->hbar / (c->dx * c->dx);
    }
    return a;
}

// Index of the first FP64 sweep of a Subsystem I substep: after the predictor
// pass (learned warm start) and the FP32 sweeps (precision form); the adjoint
// substep has neither.
int first64_of(const ecpic_ctx *c) { return c->adjoint ? 0 : (c->ws_on ? 1 : 0) + c->k32; }

void enqueue_sweeps_I(ecpic_ctx *c, int count) {
    SweepIArgs a = sweep_args(c);
    FieldIArgs f{};
    f.items = c->items[c->icur];
    f.part = c->part;
    f.taps = c->taps1;
    f.ntaps = c->nt1;
    f.mlo = c->mlo1;
    f.en = c->ex[c->exc];
    f.ek0 = c->ek[0];
    f.ek1 = c->ek[1];
    f.coefE0 = c->coefE[0];
    f.coefE1 = c->coefE[1];
    f.st = c->stI;
    f.w = c->w;
    f.M = c->M;
    f.wpi = c->block / 64;
    f.wcnt = c->wcnt;
    f.cbase = c->cbase;
    f.nstart = c->nstart;
    f.base = c->base;
    f.items_next = c->items[c->icur ^ 1];
    f.ex_next = c->ex[c->exc ^ 1];
    f.chunk = c->chunk;
    const int gridp = particle_grid(c, c->exact_items);
    const int mlp = (c->ws_on && !c->adjoint) ? 1 : 0;
    const int first64 = first64_of(c);
    a.first64 = first64;
    f.first64 = first64;
    a.dprev = (!mlp && !c->adjoint && c->ws_prev && c->have_prev) ? c->dprev : nullptr;
    a.explicit_start = !mlp && !a.dprev;
    a.ws = WsNet{c->ws_theta, c->ws_norm, c->ws_norm + (c->wsD + 2), c->ws_norm + 2 * (c->wsD + 2)};
    a.ws_table = c->ws_table;
    for (int i = 0; i < count; ++i) {
        a.k = f.k = c->kI++;
        if (mlp && a.k == 0) {   // the predictor pass takes the place of sweep 0
            timed(c, "ws_predict", [&] { launch_ws_predict(c->P, gridp, c->block, c->stream, a); });
        } else {
            const bool fp32 = a.k < first64;
            a.d32in = (c->k32 > 0 && !c->adjoint && a.k == first64) ? c->fbuf[first64 & 1] : nullptr;
            timed(c, c->adjoint ? "sweep_I_adj" : (fp32 ? "sweep_I32" : "sweep_I"), [&] {
                launch_sweep_I(c->P, c->seidel || c->adjoint, fp32, c->adjoint, gridp, c->block, c->stream, a);
            });
        }
        timed(c, "field_I", [&] { launch_field_I(c->P, c->M, c->stream, f); });
    }
}

// Picard sweeps of the last Subsystem I substep (the predictor pass not
// counted) and how many of them ran in FP32.
int sweeps_done_I(const ecpic_ctx *c) {
    const int n = c->h->I.kconv >= 0 ? c->h->I.kconv + 1 : c->kI;
    return (c->ws_on && !c->adjoint) ? n - 1 : n;
}
int fp32_sweeps_done_I(const ecpic_ctx *c) {
    if (c->adjoint) return 0;
    return std::min(std::max(c->kI - (c->ws_on ? 1 : 0), 0), c->k32);
}

// Residuals of the last Subsystem I substep's first FP64 sweeps (each recorded
// by the convergence test that follows the sweep; 0 past the last).
void first_residuals_I(const ecpic_ctx *c, double *r) {
    for (int i = 0; i < 4; ++i) r[i] = c->h->I.res_first[i];
}

void enqueue_commit_I(ecpic_ctx *c) {
    CommitIArgs a{};
    a.cur = c->pb[c->cur];
    a.nxt = c->pb[c->cur ^ 1];
    a.d0 = c->dbuf[0];
    a.d1 = c->dbuf[1];
    a.items = c->items[c->icur];
    a.items_next = c->items[c->icur ^ 1];
    a.coefA = c->coefA;
    a.coefE0 = c->coefE[0];
    a.coefE1 = c->coefE[1];
    a.stII = c->stII;
    a.wcnt = c->wcnt;
    a.base = c->base;
    a.cbase = c->cbase;
    a.nstart = c->nstart;
    a.st = c->stI;
    a.dt = c->dt;
    a.dt_dx = c->dt / c->dx;
    a.dx_dt = c->dx / c->dt;
    a.inv_dx = c->inv_dx;
    a.dx = c->dx;
    a.tol = c->tol;
    a.M = c->M;
    a.chunk = c->chunk;
    a.hbar_dx2 = c->hbar / (c->dx * c->dx);   // cur / nxt carry the spins when there are any
    a.seidel = c->seidel || c->adjoint;
    a.wpi = c->block / 64;
    a.nsweeps = c->kI;
    a.first64 = first64_of(c);
    // the last known order decides where a list with several items per cell is built
    a.list_kernel = c->n_items_host != c->M ? 1 : 0;
    if (c->fuse_II && !c->adjoint) {
        a.coefAk0 = c->coefAk[0];   // a^(0), formed by the step's start
        a.part2 = c->part;
    }
    if (c->ws_stride > 0 && c->ws_feat && !c->adjoint) {   // record training pairs of this step
        a.rec.feat = c->ws_feat;
        a.rec.targ = c->ws_targ;
        a.rec.cap = c->ws_cap;
        a.rec.base = c->ws_base;
        a.rec.stride = c->ws_stride;
        a.rec.phase = c->ws_phase;
        a.rec.ay = c->ay[c->trc];
        a.rec.az = c->az[c->trc];
        a.rec.ex = c->ex[c->exc];
    }
    a.N = c->N;
    if (c->ws_prev) {   // the next substep starts from this commit's increments
        a.dprev_out = c->dprev;
        c->have_prev = true;
    }
    timed(c, c->adjoint ? "commit_I_adj" : "commit_I",
          [&] { launch_commit_I(c->P, c->adjoint, particle_grid(c, c->exact_items), c->block, c->stream, a); });
}

// ---- Subsystem II ---------------------------------------------------------
struct IIView {
    const double *xi, *p;
    ItemList items;
    bool exact;
    bool fused;            // iterate 0's deposit comes from the commit just enqueued ...
    ItemList items_commit; // ... indexed by the item list of the order it left
};

void enqueue_iters_II(ecpic_ctx *c, const IIView &v, int count) {
    SweepIIArgs a{};
    a.xi = v.xi;
    a.p = v.p;
    a.items = v.items;
    a.coefAn = c->coefA;   // a_perp^n: Subsystem I leaves it alone
    a.coefAk0 = c->coefAk[0];
    a.coefAk1 = c->coefAk[1];
    a.part = c->part;
    a.st = c->stII;
    a.tol = c->tol;
    FieldIIArgs f{};
    f.items = v.items;
    f.part = c->part;
    f.taps = c->tapsA;
    f.ntaps = c->ntA;
    f.mlo = c->mloA;
    f.E0y = c->E0y;
    f.E0z = c->E0z;
    f.eyn = c->ey[c->trc];
    f.ezn = c->ez[c->trc];
    f.ayn = c->ay[c->trc];
    f.azn = c->az[c->trc];
    f.ey0 = c->eyk[0];
    f.ey1 = c->eyk[1];
    f.ez0 = c->ezk[0];
    f.ez1 = c->ezk[1];
    f.coefAk0 = c->coefAk[0];
    f.coefAk1 = c->coefAk[1];
    f.st = c->stII;
    f.coef = c->dt * c->w / c->dx;
    f.half_dt = 0.5 * c->dt;
    f.M = c->M;
    f.wpi = c->block / 64;
    const int gridp = particle_grid(c, v.exact);
    for (int i = 0; i < count; ++i) {
        a.k = f.k = c->kII++;
        if (a.k == 0 && v.fused) {
            FieldIIArgs f0 = f;
            f0.items = v.items_commit;
            f0.wide = 1;
            timed(c, "field_II", [&] { launch_field_II(c->P, c->M, c->stream, f0); });
            continue;
        }
        timed(c, "sweep_II", [&] { launch_sweep_II(c->P, gridp, c->block, c->stream, a); });
        timed(c, "field_II", [&] { launch_field_II(c->P, c->M, c->stream, f); });
    }
}

void enqueue_commit_II(ecpic_ctx *c) {
    const int t = c->trc, n = t ^ 1;
    timed(c, "commit_II", [&] {
        launch_commit_II((c->M + 255) / 256, c->stream, c->stII, c->stI, c->hdev, c->ey[t], c->ez[t], c->ay[t], c->az[t],
                         c->eyk[0], c->eyk[1], c->ezk[0], c->ezk[1], c->ey[n], c->ez[n], c->ay[n], c->az[n],
                         0.5 * c->dt, c->M, c->kII, c->tol);
    });
}

// The host's view of both statuses: already written by the Subsystem II commit
// (mirrored), or copied (stII = stI + 1, and I, II adjacent in the mirror).
int read_status(ecpic_ctx *c, bool mirrored) {
    if (!mirrored || !c->hdev)
        HIPCHK(hipMemcpyAsync(&c->h->I, c->stI, 2 * sizeof(DevStatus), hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

int flags_to_status(int32_t f) {
    if (f & FLAG_NONFINITE) return ECPIC_ENONFINITE;
    if (f & FLAG_CFL) return ECPIC_ECFL;
    if (f & FLAG_ORDER) return ECPIC_EDEVICE;
    return ECPIC_OK;
}

// The predictor's tables of the learned warm start (when it is on), from this
// step's a_perp^n and e_x^n.
void enqueue_ws_table(ecpic_ctx *c) {
    if (!c->ws_on) return;
    WsNet net{c->ws_theta, c->ws_norm, c->ws_norm + (c->wsD + 2), c->ws_norm + 2 * (c->wsD + 2)};
    timed(c, "ws_table", [&] {
        launch_ws_table(c->P, c->stream, net, c->ws_w2b, c->coefA, c->ay[c->trc], c->az[c->trc], c->ex[c->exc],
                        c->M, c->ws_table);
    });
}

// Start of a step (do_I and do_II), or of one substep: statuses, the records
// of a^n (both substeps), of e_x^n (Subsystem I) and of a^(0), and E0
// (Subsystem II).  In a full step the Subsystem I commit resets the Subsystem
// II status, gated on its own success.
void enqueue_begin(ecpic_ctx *c, bool do_I, bool do_II, const DevStatus *gate_src = nullptr) {
    if (do_I) c->kI = 0;
    if (do_II) c->kII = 0;
    const double r = c->dt / (2.0 * c->dx);
    const int t = c->trc;
    timed(c, "begin", [&] {
        launch_begin_step(c->P, c->stream, do_I ? c->stI : nullptr, gate_src, (do_II && !do_I) ? c->stII : nullptr, c->ay[t],
                          c->az[t], c->ey[t], c->ez[t], do_I ? c->ex[c->exc] : nullptr, c->dt, c->coefA,
                          do_I ? c->coefE[0] : nullptr, c->coefAk[0], do_II ? 1 : 0, c->m0row.data(), c->krow.data(),
                          r * r, c->dt / (c->dx * c->dx), c->tapsA, c->ntA, c->mloA, c->M, c->E0y, c->E0z);
    });
    if (do_I) enqueue_ws_table(c);
}

// Slots of the training pairs advance after every committed Subsystem I step.
void advance_records(ecpic_ctx *c) {
    if (c->ws_stride <= 0) return;
    c->ws_base += (c->N + c->ws_stride - 1) / c->ws_stride;
    c->ws_phase = (c->ws_phase + 1) % c->ws_stride;
}

// Finish Subsystem I (more sweeps / commit) after a status read.
int finish_I(ecpic_ctx *c, bool *recommitted) {
    *recommitted = false;
    while (true) {
        const DevStatus &s = c->h->I;
        if (s.flags) return flags_to_status(s.flags);
        if (s.committed) return ECPIC_OK;
        if (s.kconv < 0) {
            if (c->kI >= c->kmax) return ECPIC_ENOTCONV;
            enqueue_sweeps_I(c, std::min(2, c->kmax - c->kI));
        }
        enqueue_commit_I(c);
        *recommitted = true;
        int rc = read_status(c, false);
        if (rc) return rc;
    }
}

int finish_II(ecpic_ctx *c, const IIView &v) {
    while (true) {
        const DevStatus &s = c->h->II;
        if (s.flags) return flags_to_status(s.flags);
        if (!s.gate) return ECPIC_ESTATE;
        if (s.committed) return ECPIC_OK;
        if (s.kconv < 0) {
            if (c->kII >= c->kmax) return ECPIC_ENOTCONV;
            enqueue_iters_II(c, v, std::min(2, c->kmax - c->kII));
        }
        enqueue_commit_II(c);
        int rc = read_status(c, true);
        if (rc) return rc;
    }
}

// A substep call with its own time step: dt (and with Subsystem II the
// matrix taps of that step) hold for the call, the configured ones after it.
struct DtScope {
    ecpic_ctx *c;
    double dt;
    double *taps;
    int n, mlo;
    explicit DtScope(ecpic_ctx *x) : c(x), dt(x->dt), taps(x->tapsA), n(x->ntA), mlo(x->mloA) {}
    ~DtScope() {
        c->dt = dt;
        c->tapsA = taps;
        c->ntA = n;
        c->mloA = mlo;
    }
};

// ---- spin ------------------------------------------------------------------
SpinArgs spin_args(ecpic_ctx *c) {
    SpinArgs a{};
    const Particles &d = c->pb[c->cur];
    a.xi = d.xi;
    a.sx = d.sx;
    a.sy = d.sy;
    a.sz = d.sz;
    a.items = c->items[c->icur];
    a.ay = c->ay[c->trc];
    a.az = c->az[c->trc];
    a.inv_dx = c->inv_dx;
    a.spart = c->spart;
    a.epart = c->epart;
    return a;
}

// The spin source of Subsystem II over the current dt, added to the constant
// part E0 of its iteration (after the start kernel formed E0): the deposit of
// (s_y, s_z) on V1, -/+ hbar G^T of it, times dt, through (M0 + dt^2 K/4)^{-1}.
void enqueue_spin_source(ecpic_ctx *c) {
    if (!c->spin || c->hbar == 0.0 || c->N == 0) return;
    const SpinArgs a = spin_args(c);
    timed(c, "spin_deposit", [&] { launch_spin_deposit(c->P, std::max(1, c->n_items_host), c->stream, a, c->M); });
    const double coef = c->hbar * c->dt * c->w / (c->dx * c->dx);   // G^T's 1/dx, the taps' 1/dx
    timed(c, "spin_source", [&] {
        launch_spin_source(c->P, c->stream, c->spart, c->items[c->icur], c->M, coef, c->tapsA, c->ntA, c->mloA,
                           c->E0y, c->E0z);
    });
}

// Subsystem III over h (any sign): one pass over the current order.
int substep_spin(ecpic_ctx *c, double h) {
    if (c->N == 0) return ECPIC_OK;
    SpinArgs a = spin_args(c);
    a.h = h;
    timed(c, "spin_rotate", [&] { launch_spin_rotate(c->P, std::max(1, c->n_items_host), c->stream, a, c->M); });
    return sync(c);
}

// One Subsystem I substep over dt on its own (the scheme, or its adjoint):
// start, the expected number of sweeps, commit, one status read, more sweeps if
// needed.  Nothing is committed on failure.
int substep_I(ecpic_ctx *c, double dt, ecpic_iter_stats *stats, bool adjoint) {
    if (!c || !(dt > 0.0) || !(dt < c->dx)) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    DtScope scope(c);
    c->dt = dt;
    struct Adj {
        ecpic_ctx *c;
        Adj(ecpic_ctx *x, bool on) : c(x) { c->adjoint = on; }
        ~Adj() { c->adjoint = false; }
    } adj(c, adjoint);
    const bool had_prev = c->have_prev;
    int &guess = adjoint ? c->guessIadj : c->guessI;
    enqueue_begin(c, true, false);
    enqueue_sweeps_I(c, std::min(guess, c->kmax));
    enqueue_commit_I(c);
    int rc = read_status(c, false);
    bool again = false;
    if (!rc) rc = finish_I(c, &again);
    if (stats) {
        stats->sweeps = sweeps_done_I(c);
        stats->fp32_sweeps = fp32_sweeps_done_I(c);
        stats->residual = c->h->I.res;
        stats->crossing_queue = c->h->I.queued;
        first_residuals_I(c, stats->residual_hist);
    }
    if (rc) {
        c->have_prev = had_prev;   // no commit: the increments are those of before
        return rc;
    }
    guess = std::max(1, c->h->I.kconv + 1);
    c->cur ^= 1;
    c->icur ^= 1;
    c->exc ^= 1;
    c->n_items_host = c->h->I.n_items_next;
    if (!adjoint) advance_records(c);
    return ECPIC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

const char *ecpic_strerror(int s) {
    switch (s) {
        case ECPIC_OK: return "ok";
        case ECPIC_EINVAL: return "invalid argument or configuration";
        case ECPIC_ENOMEM: return "out of memory";
        case ECPIC_ENOTCONV: return "Picard iteration did not converge; step rolled back";
        case ECPIC_EDEVICE: return "HIP device error or no usable gfx950 device";
        case ECPIC_ENONFINITE: return "non-finite value in the state";
        case ECPIC_ECFL: return "a particle moved a full cell or more in one step";
        case ECPIC_ESTATE: return "call out of order";
        default: return "unknown status";
    }
}

}  // extern "C"

// ---- context life cycle and state I/O ----------------------------------------
namespace {

int check_device(int dev) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0 || dev < 0 || dev >= n) return ECPIC_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return ECPIC_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        std::fprintf(stderr, "ecpic: device %d is %s, this library is built for gfx950\n", dev, prop.gcnArchName);
        return ECPIC_EDEVICE;
    }
    return ECPIC_OK;
}

void free_all(ecpic_ctx *c) {
    auto F = [](void *p) { if (p) hipFree(p); };
    for (int b = 0; b < 2; ++b) {
        F(c->pb[b].xi); F(c->pb[b].p); F(c->pb[b].id); F(c->dbuf[b]); F(c->fbuf[b]);
        F(c->pb[b].sx); F(c->pb[b].sy); F(c->pb[b].sz);
        F(c->items[b].cell); F(c->items[b].begin); F(c->items[b].cell_first); F(c->items[b].n_items);
        F(c->ex[b]); F(c->ey[b]); F(c->ez[b]); F(c->ay[b]); F(c->az[b]);
        F(c->ek[b]); F(c->eyk[b]); F(c->ezk[b]);
    }
    F(c->wcnt); F(c->base); F(c->cbase); F(c->nstart); F(c->part);
    F(c->E0y); F(c->E0z); F(c->taps1); F(c->dprev);
    F(c->spart); F(c->epart);
    for (auto &t : c->tapsA_by_dt) F(t.second.dev);
    F(c->coefA); F(c->coefE[0]); F(c->coefE[1]); F(c->coefAk[0]); F(c->coefAk[1]);
    F(c->st_ring);
    F(c->ws_theta); F(c->ws_m); F(c->ws_v); F(c->ws_norm); F(c->ws_table); F(c->ws_feat); F(c->ws_targ);
    F(c->ws_pgrad); F(c->ws_ploss); F(c->ws_loss); F(c->ws_w2b);
    F(c->rho); F(c->rvec); F(c->uvec); F(c->out5); F(c->part_e); F(c->maxbits); F(c->count); F(c->ex_save);
    if (c->h_ring) hipHostFree(c->h_ring);
    for (auto &e : c->prof.pool) hipEventDestroy(e);
    for (auto &pe : c->prof.pending) { hipEventDestroy(pe.second.first); hipEventDestroy(pe.second.second); }
    if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
}

// The first row of (M0^ + r^2 K^)^{-1}, r = dt / (2 dx), the Subsystem II
// matrix of time step dt, made current; computed once per time step and kept
// for the context's lifetime.
int select_tapsA(ecpic_ctx *c, double dt) {
    auto it = c->tapsA_by_dt.find(dt);
    if (it == c->tapsA_by_dt.end()) {
        std::vector<double> tA, arow(2 * c->P + 1);
        const double r = dt / (2.0 * c->dx);
        for (int k = 0; k <= 2 * c->P; ++k) arow[k] = c->m0row[k] + r * r * c->krow[k];
        int mlo = 0;
        inverse_taps(arow, c->M, 1e-18, tA, mlo);
        double *d = nullptr;
        if (dalloc(&d, tA.size())) return ECPIC_ENOMEM;
        if (hipMemcpyAsync(d, tA.data(), sizeof(double) * tA.size(), hipMemcpyHostToDevice, c->stream) !=
                hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            hipFree(d);
            return ECPIC_EDEVICE;
        }
        it = c->tapsA_by_dt.emplace(dt, ecpic_ctx::Taps{d, (int)tA.size(), mlo}).first;
    }
    c->tapsA = it->second.dev;
    c->ntA = it->second.n;
    c->mloA = it->second.mlo;
    return ECPIC_OK;
}

int alloc_all(ecpic_ctx *c) {
    const int M = c->M, MP = M + 2 * HALO;
    const int64_t N = c->N;
    int rc = 0;
    for (int b = 0; b < 2; ++b) {
        rc |= dalloc(&c->pb[b].xi, N); rc |= dalloc(&c->pb[b].p, N); rc |= dalloc(&c->pb[b].id, N);
        if (c->spin) { rc |= dalloc(&c->pb[b].sx, N); rc |= dalloc(&c->pb[b].sy, N); rc |= dalloc(&c->pb[b].sz, N); }
        rc |= dalloc(&c->dbuf[b], N);
        if (c->k32 > 0) rc |= dalloc(&c->fbuf[b], N);
        rc |= dalloc(&c->items[b].cell, c->max_items); rc |= dalloc(&c->items[b].begin, c->max_items + 1);
        rc |= dalloc(&c->items[b].cell_first, M + 1); rc |= dalloc(&c->items[b].n_items, 2);
        rc |= dalloc(&c->ex[b], MP); rc |= dalloc(&c->ey[b], MP); rc |= dalloc(&c->ez[b], MP);
        rc |= dalloc(&c->ay[b], MP); rc |= dalloc(&c->az[b], MP);
        rc |= dalloc(&c->ek[b], MP); rc |= dalloc(&c->eyk[b], MP); rc |= dalloc(&c->ezk[b], MP);
    }
    rc |= dalloc(&c->base, (size_t)c->max_items * 3);
    rc |= dalloc(&c->cbase, (size_t)c->M * 3);
    rc |= dalloc(&c->wcnt, (size_t)c->max_items * (c->block / 64) * 3);
    rc |= dalloc(&c->nstart, (size_t)2 * M + 1);
    // per item and wave: Subsystem I P+4 values, Subsystem II 2 (P+1)
    rc |= dalloc(&c->part, (size_t)c->max_items * (c->block / 64) * std::max(2 * (c->P + 3), c->P + 4));
    rc |= dalloc(&c->E0y, M); rc |= dalloc(&c->E0z, M);
    const size_t nrec = (size_t)(M + 2);
    rc |= dalloc(&c->coefA, nrec * 2 * (c->P + 1));
    rc |= dalloc(&c->coefAk[0], nrec * 2 * (c->P + 1)); rc |= dalloc(&c->coefAk[1], nrec * 2 * (c->P + 1));
    rc |= dalloc(&c->coefE[0], nrec * c->P); rc |= dalloc(&c->coefE[1], nrec * c->P);
    rc |= dalloc(&c->st_ring, 2 * STEP_BATCH);
    if (c->ws_prev) rc |= dalloc(&c->dprev, N);
    c->wsD = ws_d(c->P);
    c->wsNP = ws_nparams(c->wsD);
    rc |= dalloc(&c->ws_theta, c->wsNP); rc |= dalloc(&c->ws_m, c->wsNP); rc |= dalloc(&c->ws_v, c->wsNP);
    rc |= dalloc(&c->ws_norm, 2 * (c->wsD + 2) + 2); rc |= dalloc(&c->ws_table, (size_t)M * WS_NT * WS_NP);
    rc |= dalloc(&c->ws_loss, 1); rc |= dalloc(&c->ws_w2b, (size_t)WS_H * (WS_H + 4));

    rc |= dalloc(&c->rho, M); rc |= dalloc(&c->rvec, M); rc |= dalloc(&c->uvec, M);
    rc |= dalloc(&c->out5, 8); rc |= dalloc(&c->part_e, c->max_items); rc |= dalloc(&c->maxbits, 1);
    rc |= dalloc(&c->count, M);
    if (c->symmetric || c->spin) rc |= dalloc(&c->ex_save, MP);
    if (c->spin) {
        rc |= dalloc(&c->spart, (size_t)c->max_items * 2 * c->P);
        rc |= dalloc(&c->epart, c->max_items);
    }
    if (rc) return ECPIC_ENOMEM;
    if (hipHostMalloc((void **)&c->h_ring, sizeof(*c->h_ring) * STEP_BATCH, hipHostMallocMapped) != hipSuccess)
        return ECPIC_ENOMEM;
    if (hipHostGetDevicePointer((void **)&c->h_ring_dev, c->h_ring, 0) != hipSuccess) c->h_ring_dev = nullptr;
    set_slot(c, 0);
    // fields start at zero, items empty
    for (int b = 0; b < 2; ++b) {
        for (double *f : {c->ex[b], c->ey[b], c->ez[b], c->ay[b], c->az[b], c->ek[b], c->eyk[b], c->ezk[b]})
            launch_pad(c->stream, nullptr, f, 0.0, M);
    }
    HIPCHK(hipMemsetAsync(c->count, 0, sizeof(int32_t) * M, c->stream));
    for (int b = 0; b < 2; ++b)   // both lists valid (empty) from the start
        launch_items_from_counts(c->stream, c->count, c->nstart, M, c->chunk, 0, c->items[b]);
    HIPCHK(hipMemsetAsync(c->st_ring, 0, sizeof(DevStatus) * 2 * STEP_BATCH, c->stream));
    // closed-form rows and inverse taps
    c->m0row = mass_row(c->P);
    c->m1row = mass_row(c->P - 1);
    c->krow.assign(2 * c->P + 1, 0.0);
    for (int k = -c->P; k <= c->P; ++k) {
        auto m = [&](int q) { return (q >= -(c->P - 1) && q <= c->P - 1) ? c->m1row[q + c->P - 1] : 0.0; };
        c->krow[k + c->P] = 2.0 * m(k) - m(k - 1) - m(k + 1);
    }
    std::vector<double> t1;
    inverse_taps(c->m1row, M, 1e-18, t1, c->mlo1);
    c->nt1 = (int)t1.size();
    if (dalloc(&c->taps1, t1.size())) return ECPIC_ENOMEM;
    HIPCHK(hipMemcpyAsync(c->taps1, t1.data(), sizeof(double) * t1.size(), hipMemcpyHostToDevice, c->stream));
    rc = sync(c);
    if (rc) return rc;
    return select_tapsA(c, c->dt);
}

int upload_padded(ecpic_ctx *c, const double *host, double *dev_pad) {
    if (!host) {
        launch_pad(c->stream, nullptr, dev_pad, 0.0, c->M);
        return ECPIC_OK;
    }
    HIPCHK(hipMemcpyAsync(c->uvec, host, sizeof(double) * c->M, hipMemcpyHostToDevice, c->stream));
    launch_pad(c->stream, c->uvec, dev_pad, 1.0, c->M);
    return sync(c);
}

int download_padded(ecpic_ctx *c, const double *dev_pad, double *host) {
    if (!host) return ECPIC_OK;
    launch_unpad(c->stream, dev_pad, c->rvec, c->M);
    HIPCHK(hipMemcpyAsync(host, c->rvec, sizeof(double) * c->M, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

// Sort arbitrary device arrays (x, p) into the context (cell-sorted, ids).
int load_particles_dev(ecpic_ctx *c, const double *x, const double *p) {
    const int64_t N = c->N;
    int32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr, *v1 = nullptr, *hist = nullptr;
    double *xt = nullptr, *pt = nullptr;
    const int64_t nblk = (N + 4095) / 4096;
    int rc = dalloc(&k0, N) | dalloc(&v0, N) | dalloc(&k1, N) | dalloc(&v1, N) | dalloc(&hist, 16 * nblk + 1) |
             dalloc(&xt, N) | dalloc(&pt, N);
    if (rc == ECPIC_OK) {
        Particles &d = c->pb[c->cur];
        if (N > 0) {
            launch_init_particles(c->stream, x, p, N, c->L, c->inv_dx, c->M, xt, pt, k0, v0);
            int bits = 0;
            while ((1 << bits) < c->M) ++bits;
            int32_t *ks, *vs;
            radix_sort(c->stream, k0, v0, k1, v1, N, std::max(bits, 1), hist, &ks, &vs);
            launch_gather_sorted(c->stream, vs, xt, pt, N, d.xi, d.p, d.id);
            hipMemsetAsync(c->count, 0, sizeof(int32_t) * c->M, c->stream);
            launch_count_cells(c->stream, ks, N, c->count);
        } else {
            hipMemsetAsync(c->count, 0, sizeof(int32_t) * c->M, c->stream);
        }
        launch_items_from_counts(c->stream, c->count, c->nstart, c->M, c->chunk, N, c->items[c->icur]);
        hipMemcpyAsync(&c->h->n_items_next, c->items[c->icur].n_items, sizeof(int32_t), hipMemcpyDeviceToHost,
                       c->stream);
        rc = sync(c);
        c->n_items_host = c->h->n_items_next;
    }
    for (void *q : {(void *)k0, (void *)v0, (void *)k1, (void *)v1, (void *)hist, (void *)xt, (void *)pt})
        if (q) hipFree(q);
    if (rc == ECPIC_OK && c->spin && N > 0) {   // a new state: spins zero until set_spins
        const Particles &d = c->pb[c->cur];
        for (double *q : {d.sx, d.sy, d.sz})
            if (hipMemsetAsync(q, 0, sizeof(double) * N, c->stream) != hipSuccess) rc = ECPIC_EDEVICE;
        if (rc == ECPIC_OK) rc = sync(c);
    }
    if (rc == ECPIC_OK) c->have_particles = true;
    c->have_prev = false;   // a new order: no previous increments
    return rc;
}

}  // namespace

extern "C" {

int ecpic_create(const ecpic_config *cfg, ecpic_ctx **out) {
    if (!cfg || !out) return ECPIC_EINVAL;
    *out = nullptr;
    const ecpic_config &g = *cfg;
    if (!(g.L > 0.0) || g.degree < 2 || g.degree > MAX_DEG || g.M < g.degree + 3 || g.n_particles < 0 ||
        g.n_particles > (int64_t)0x7fffffff - 1 || !(g.dt > 0.0) || !(g.dt < g.L / g.M) || !(g.picard_tol > 0.0) ||
        g.picard_max_iter < 0 || (g.precision != ECPIC_FP64 && g.precision != ECPIC_FP32_MIXED) ||
        g.fp32_sweeps < 0 || g.fp32_sweeps > 16 || g.sweep_guess < 0 ||
        (g.map != ECPIC_MAP_JACOBI && g.map != ECPIC_MAP_SEIDEL) ||
        (g.warmstart != ECPIC_WS_EXPLICIT && g.warmstart != ECPIC_WS_PREVIOUS && g.warmstart != ECPIC_WS_MLP) ||
        g.weight < 0.0 || g.waves_per_item < 0 || g.waves_per_item > MAX_WAVES_PER_ITEM ||
        (g.splitting != ECPIC_LIE_TROTTER && g.splitting != ECPIC_SYMMETRIC) ||
        (g.item_particles != 0 && (g.item_particles < MIN_CHUNK || g.item_particles > MAX_CHUNK ||
                                   (g.item_particles & (g.item_particles - 1)) != 0)) ||
        (g.spin != 0 && g.spin != 1) || !std::isfinite(g.hbar) || (!g.spin && g.hbar != 0.0) ||
        (g.spin && (g.precision != ECPIC_FP64 || g.warmstart == ECPIC_WS_MLP)))
        return ECPIC_EINVAL;
    int rc = check_device(g.device);
    if (rc) return rc;
    if (hipSetDevice(g.device) != hipSuccess) return ECPIC_EDEVICE;
    // the fixed scratch of ecpic_deposit_current_noalloc on this device (if its
    // address cannot be taken, only that call fails, with EDEVICE)
    noalloc_init(g.device);
    ecpic_ctx *c = new ecpic_ctx();
    c->cfg = g;
    c->device = g.device;
    c->M = g.M;
    c->P = g.degree;
    c->N = g.n_particles;
    c->L = g.L;
    c->dx = g.L / g.M;
    c->inv_dx = (double)g.M / g.L;
    c->w = g.weight > 0.0 ? g.weight : (g.n_particles > 0 ? g.L / (double)g.n_particles : 0.0);
    c->dt = g.dt;
    c->tol = g.picard_tol;
    c->kmax = g.picard_max_iter > 0 ? std::min(g.picard_max_iter, MAX_HIST) : 50;
    c->seidel = g.map == ECPIC_MAP_SEIDEL;
    c->k32 = g.precision == ECPIC_FP32_MIXED ? (g.fp32_sweeps > 0 ? g.fp32_sweeps : 2) : 0;
    c->guessI = c->guessII = g.sweep_guess > 0 ? g.sweep_guess : 4;
    c->ws_prev = g.warmstart == ECPIC_WS_PREVIOUS;
    c->symmetric = g.splitting == ECPIC_SYMMETRIC;
    c->spin = g.spin != 0;
    c->hbar = g.hbar;
    const double ppc = g.M > 0 ? (double)g.n_particles / g.M : 0.0;
    // One work item per cell where the cells allow (the item list is then the
    // cell index, and the commit needs no list-building pass): items hold up to
    // twice the mean count, from MIN_CHUNK to MAX_CHUNK particles.
    c->chunk = MIN_CHUNK;
    if (g.item_particles > 0) c->chunk = g.item_particles;
    else while (c->chunk < MAX_CHUNK && c->chunk < 2.0 * ppc) c->chunk *= 2;
    // Waves per work item: enough items x waves to give every SIMD (1024 on the
    // chip) about four waves, and otherwise as few waves per item as possible,
    // so each wave streams many rows of particles (measured best on the pump
    // and Langmuir workloads).
    if (g.waves_per_item > 0) {
        c->block = 64 * g.waves_per_item;
    } else {
        const double items = (double)g.M * std::max(1.0, std::ceil(ppc / c->chunk));
        const int wpi = (int)std::min(4.0, std::max(1.0, std::ceil(4096.0 / items)));
        c->block = 64 * wpi;
    }
    c->max_items = (int)(g.M + g.n_particles / c->chunk + 2);
    if (g.stream) {
        c->stream = (hipStream_t)g.stream;
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) { delete c; return ECPIC_EDEVICE; }
        c->own_stream = true;
    }
    rc = alloc_all(c);
    if (rc) {
        free_all(c);
        delete c;
        return rc;
    }
    *out = c;
    return ECPIC_OK;
}

int ecpic_destroy(ecpic_ctx *c) {
    if (!c) return ECPIC_OK;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
    return ECPIC_OK;
}

int ecpic_set_particles(ecpic_ctx *c, const double *x, const double *p, int64_t n) {
    if (!c || n != c->N || (n > 0 && (!x || !p))) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    double *dx_ = nullptr, *dp_ = nullptr;
    if (dalloc(&dx_, n) || dalloc(&dp_, n)) { if (dx_) hipFree(dx_); return ECPIC_ENOMEM; }
    int rc = ECPIC_OK;
    if (n > 0) {
        if (hipMemcpyAsync(dx_, x, sizeof(double) * n, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(dp_, p, sizeof(double) * n, hipMemcpyHostToDevice, c->stream) != hipSuccess)
            rc = ECPIC_EDEVICE;
    }
    if (rc == ECPIC_OK) rc = load_particles_dev(c, dx_, dp_);
    hipFree(dx_);
    hipFree(dp_);
    return rc;
}

int ecpic_set_particles_dev(ecpic_ctx *c, const double *x, const double *p, int64_t n) {
    if (!c || n != c->N || (n > 0 && (!x || !p))) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    return load_particles_dev(c, x, p);
}

int ecpic_get_particles_dev(ecpic_ctx *c, double *x, double *p, int64_t n) {
    if (!c || n != c->N || (n > 0 && (!x || !p))) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    const Particles &d = c->pb[c->cur];
    launch_unpermute(c->stream, d.xi, d.p, d.id, n, c->dx, x, p);
    return sync(c);
}

int ecpic_get_particles(ecpic_ctx *c, double *x, double *p, int64_t n) {
    if (!c || n != c->N || (n > 0 && (!x || !p))) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    double *dx_ = nullptr, *dp_ = nullptr;
    if (dalloc(&dx_, n) || dalloc(&dp_, n)) { if (dx_) hipFree(dx_); return ECPIC_ENOMEM; }
    int rc = ecpic_get_particles_dev(c, dx_, dp_, n);
    if (rc == ECPIC_OK && n > 0) {
        if (hipMemcpy(x, dx_, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(p, dp_, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess)
            rc = ECPIC_EDEVICE;
    }
    hipFree(dx_);
    hipFree(dp_);
    return rc;
}

int ecpic_set_spins(ecpic_ctx *c, const double *sx, const double *sy, const double *sz, int64_t n) {
    if (!c || !c->spin || n != c->N || (n > 0 && (!sx || !sy || !sz))) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    if (n == 0) return ECPIC_OK;
    double *t[3] = {nullptr, nullptr, nullptr};
    if (dalloc(&t[0], n) || dalloc(&t[1], n) || dalloc(&t[2], n)) {
        for (double *q : t) if (q) hipFree(q);
        return ECPIC_ENOMEM;
    }
    int rc = ECPIC_OK;
    const double *in[3] = {sx, sy, sz};
    for (int k = 0; k < 3 && rc == ECPIC_OK; ++k)
        if (hipMemcpyAsync(t[k], in[k], sizeof(double) * n, hipMemcpyHostToDevice, c->stream) != hipSuccess)
            rc = ECPIC_EDEVICE;
    const Particles &d = c->pb[c->cur];
    if (rc == ECPIC_OK) launch_spin_in(c->stream, t[0], t[1], t[2], d.id, n, d.sx, d.sy, d.sz);
    if (rc == ECPIC_OK) rc = sync(c);
    for (double *q : t) hipFree(q);
    return rc;
}

int ecpic_get_spins(ecpic_ctx *c, double *sx, double *sy, double *sz, int64_t n) {
    if (!c || !c->spin || n != c->N || (n > 0 && (!sx || !sy || !sz))) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    if (n == 0) return ECPIC_OK;
    double *t[3] = {nullptr, nullptr, nullptr};
    if (dalloc(&t[0], n) || dalloc(&t[1], n) || dalloc(&t[2], n)) {
        for (double *q : t) if (q) hipFree(q);
        return ECPIC_ENOMEM;
    }
    const Particles &d = c->pb[c->cur];
    launch_spin_out(c->stream, d.sx, d.sy, d.sz, d.id, n, t[0], t[1], t[2]);
    int rc = ECPIC_OK;
    double *out[3] = {sx, sy, sz};
    for (int k = 0; k < 3 && rc == ECPIC_OK; ++k)
        if (hipMemcpyAsync(out[k], t[k], sizeof(double) * n, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
            rc = ECPIC_EDEVICE;
    if (rc == ECPIC_OK) rc = sync(c);
    for (double *q : t) hipFree(q);
    return rc;
}

int ecpic_set_fields(ecpic_ctx *c, const double *ex, const double *ey, const double *ez, const double *ay,
                     const double *az) {
    if (!c) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    int rc = upload_padded(c, ex, c->ex[c->exc]);
    if (!rc) rc = upload_padded(c, ey, c->ey[c->trc]);
    if (!rc) rc = upload_padded(c, ez, c->ez[c->trc]);
    if (!rc) rc = upload_padded(c, ay, c->ay[c->trc]);
    if (!rc) rc = upload_padded(c, az, c->az[c->trc]);
    if (!rc) rc = sync(c);
    return rc;
}

int ecpic_get_fields(ecpic_ctx *c, double *ex, double *ey, double *ez, double *ay, double *az) {
    if (!c) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    int rc = download_padded(c, c->ex[c->exc], ex);
    if (!rc) rc = download_padded(c, c->ey[c->trc], ey);
    if (!rc) rc = download_padded(c, c->ez[c->trc], ez);
    if (!rc) rc = download_padded(c, c->ay[c->trc], ay);
    if (!rc) rc = download_padded(c, c->az[c->trc], az);
    return rc;
}

int ecpic_deposit_charge(ecpic_ctx *c, double *rho) {
    if (!c || !rho) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    launch_charge(c->P, particle_grid(c, true), c->block, c->stream, c->pb[c->cur].xi, c->items[c->icur], c->part,
                  c->w, c->M, c->rho);
    HIPCHK(hipMemcpyAsync(rho, c->rho, sizeof(double) * c->M, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

int ecpic_solve_gauss(ecpic_ctx *c) {
    if (!c) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    launch_charge(c->P, particle_grid(c, true), c->block, c->stream, c->pb[c->cur].xi, c->items[c->icur], c->part,
                  c->w, c->M, c->rho);
    launch_poisson_rhs(c->stream, c->rho, c->M, c->dx, c->uvec);
    launch_conv((c->M + 255) / 256, c->stream, c->uvec, c->rvec, c->taps1, c->nt1, c->mlo1, 1.0 / c->dx, c->M);
    launch_pad(c->stream, c->rvec, c->ex[c->exc], 1.0, c->M);
    return sync(c);
}

int ecpic_gauss_residual(ecpic_ctx *c, double *linf, double *vec) {
    if (!c || !linf) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    launch_charge(c->P, particle_grid(c, true), c->block, c->stream, c->pb[c->cur].xi, c->items[c->icur], c->part,
                  c->w, c->M, c->rho);
    HIPCHK(hipMemsetAsync(c->maxbits, 0, sizeof(unsigned long long), c->stream));
    launch_gauss(c->stream, c->rho, c->ex[c->exc], c->m1row.data(), c->P, c->M, c->dx, c->rvec, c->maxbits);
    unsigned long long bits = 0;
    HIPCHK(hipMemcpyAsync(&bits, c->maxbits, sizeof(bits), hipMemcpyDeviceToHost, c->stream));
    if (vec) HIPCHK(hipMemcpyAsync(vec, c->rvec, sizeof(double) * c->M, hipMemcpyDeviceToHost, c->stream));
    int rc = sync(c);
    std::memcpy(linf, &bits, sizeof(double));
    return rc;
}

int ecpic_energy(ecpic_ctx *c, ecpic_energy_parts *out) {
    if (!c || !out) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    const Particles &d = c->pb[c->cur];
    launch_energy(c->P, particle_grid(c, true), c->block, c->stream, d.xi, d.p, c->items[c->icur], c->ay[c->trc],
                  c->az[c->trc], c->part_e);
    launch_energy_final(c->stream, c->part_e, c->items[c->icur].n_items, c->w, c->ex[c->exc], c->ey[c->trc],
                        c->ez[c->trc], c->ay[c->trc], c->az[c->trc], c->m0row.data(), c->m1row.data(),
                        c->krow.data(), c->P, c->M, c->dx, c->out5);
    double h5[5];
    HIPCHK(hipMemcpyAsync(h5, c->out5, sizeof(h5), hipMemcpyDeviceToHost, c->stream));
    double zee = 0.0;
    const int ni = c->n_items_host;
    if (c->spin && c->hbar != 0.0 && c->N > 0 && ni > 0) {   // per-item sums, added here in item order
        launch_spin_energy(c->P, ni, c->stream, spin_args(c), c->M);
        c->h_epart.resize(ni);
        HIPCHK(hipMemcpyAsync(c->h_epart.data(), c->epart, sizeof(double) * ni, hipMemcpyDeviceToHost, c->stream));
    }
    int rc = sync(c);
    if (c->spin && c->hbar != 0.0 && c->N > 0 && ni > 0) {
        for (int i = 0; i < ni; ++i) zee += c->h_epart[i];
        zee *= c->hbar * c->w;
    }
    out->kinetic = h5[0]; out->e_long = h5[1]; out->e_trans = h5[2]; out->b_trans = h5[3];
    out->total = h5[4] + zee;
    out->zeeman = zee;
    return rc;
}

int ecpic_deposit_current(ecpic_ctx *c, const double *x0, const double *x1, int64_t n, double *J) {
    if (!c || !J || n < 0 || (n > 0 && (!x0 || !x1))) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    double *a = nullptr, *b = nullptr, *dJ = nullptr;
    int *fl = nullptr;
    if (dalloc(&a, n) || dalloc(&b, n) || dalloc(&dJ, c->M) || dalloc(&fl, 1)) {
        for (void *q : {(void *)a, (void *)b, (void *)dJ, (void *)fl}) if (q) hipFree(q);
        return ECPIC_ENOMEM;
    }
    int rc = ECPIC_OK;
    if (n > 0) {
        hipMemcpyAsync(a, x0, sizeof(double) * n, hipMemcpyHostToDevice, c->stream);
        hipMemcpyAsync(b, x1, sizeof(double) * n, hipMemcpyHostToDevice, c->stream);
    }
    hipMemsetAsync(dJ, 0, sizeof(double) * c->M, c->stream);
    hipMemsetAsync(fl, 0, sizeof(int), c->stream);
    launch_deposit_segments(c->P, c->stream, a, b, n, c->inv_dx, c->dx, c->w, c->M, dJ, fl);
    int hf = 0;
    hipMemcpyAsync(J, dJ, sizeof(double) * c->M, hipMemcpyDeviceToHost, c->stream);
    hipMemcpyAsync(&hf, fl, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    rc = sync(c);
    if (!rc && hf) rc = ECPIC_ECFL;
    for (void *q : {(void *)a, (void *)b, (void *)dJ, (void *)fl}) hipFree(q);
    return rc;
}

// Asynchronous, allocation-free variant of ecpic_deposit_current (device
// arrays, fixed scratch; see noalloc.hip).
int ecpic_deposit_current_noalloc(ecpic_ctx *c, const double *x0, const double *x1, int64_t n, double *J,
                                  int32_t *flags) {
    if (!c || !J || n < 0 || (n > 0 && (!x0 || !x1))) return ECPIC_EINVAL;
    if (c->M > noalloc_max_cells()) {
        std::fprintf(stderr, "ecpic_deposit_current_noalloc: %d cells exceed the %d of its fixed scratch\n", c->M,
                     noalloc_max_cells());
        return ECPIC_EINVAL;
    }
    if (hipSetDevice(c->device) != hipSuccess) return ECPIC_EDEVICE;
    double *scr = noalloc_scratch(c->device);
    if (!scr) return ECPIC_EDEVICE;
    launch_deposit_noalloc(c->P, c->stream, x0, x1, n, c->inv_dx, c->dx, c->w, c->M, scr, J, flags);
    return hipGetLastError() == hipSuccess ? ECPIC_OK : ECPIC_EDEVICE;
}

// ---- substeps and steps -------------------------------------------------------
int ecpic_substep_particles(ecpic_ctx *c, double dt, ecpic_iter_stats *stats) {
    return substep_I(c, dt, stats, false);
}

int ecpic_substep_particles_adjoint(ecpic_ctx *c, double dt, ecpic_iter_stats *stats) {
    return substep_I(c, dt, stats, true);
}

int ecpic_substep_spin(ecpic_ctx *c, double dt) {
    if (!c || !c->spin || !std::isfinite(dt)) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    return substep_spin(c, dt);
}

int ecpic_substep_fields(ecpic_ctx *c, double dt, ecpic_iter_stats *stats) {
    if (!c || !(dt > 0.0) || !(dt < c->dx)) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    DtScope scope(c);
    int rc0 = select_tapsA(c, dt);
    if (rc0) return rc0;
    c->dt = dt;
    enqueue_begin(c, false, true);
    enqueue_spin_source(c);
    IIView v{c->pb[c->cur].xi, c->pb[c->cur].p, c->items[c->icur], true, false, {}};
    enqueue_iters_II(c, v, std::min(c->guessII, c->kmax));
    enqueue_commit_II(c);
    int rc = read_status(c, true);
    if (!rc) rc = finish_II(c, v);
    if (stats) {
        stats->sweeps = c->h->II.kconv >= 0 ? c->h->II.kconv + 1 : c->kII;
        stats->fp32_sweeps = 0;
        stats->residual = c->h->II.res;
        stats->crossing_queue = 0;
        for (double &r : stats->residual_hist) r = 0.0;
    }
    if (rc) return rc;
    c->guessII = std::max(1, c->h->II.kconv + 1);
    c->trc ^= 1;
    return ECPIC_OK;
}

namespace {

// Host bookkeeping of one step, as it stood when the step was enqueued.
struct StepSnap {
    int cur, icur, exc, trc, n_items;
    int64_t ws_base;
    int ws_phase;
    bool exact, have_prev;
};

StepSnap snap(const ecpic_ctx *c) {
    return {c->cur, c->icur, c->exc, c->trc, c->n_items_host, c->ws_base, c->ws_phase, c->exact_items, c->have_prev};
}

void restore(ecpic_ctx *c, const StepSnap &q) {
    c->cur = q.cur; c->icur = q.icur; c->exc = q.exc; c->trc = q.trc;
    c->n_items_host = q.n_items; c->ws_base = q.ws_base; c->ws_phase = q.ws_phase; c->exact_items = q.exact;
    c->have_prev = q.have_prev;
}

// Buffers swap after a committed step.
void advance(ecpic_ctx *c) {
    c->cur ^= 1;
    c->icur ^= 1;
    c->exc ^= 1;
    c->trc ^= 1;
    advance_records(c);
}

void step_stats(const ecpic_ctx *c, ecpic_iter_stats *sI, ecpic_iter_stats *sII) {
    if (sI) {
        sI->sweeps = sweeps_done_I(c);
        sI->fp32_sweeps = fp32_sweeps_done_I(c);
        sI->residual = c->h->I.res;
        sI->crossing_queue = c->h->I.queued;
        sI->sweeps_adjoint = 0;
        first_residuals_I(c, sI->residual_hist);
    }
    if (sII) {
        sII->sweeps = c->h->II.kconv >= 0 ? c->h->II.kconv + 1 : c->kII;
        sII->fp32_sweeps = 0;
        sII->residual = c->h->II.res;
        sII->crossing_queue = 0;
        sII->sweeps_adjoint = 0;
        for (double &r : sII->residual_hist) r = 0.0;
    }
}

// Steps run substep by substep: the symmetric composition (Subsystem I over
// dt/2, II over dt, the adjoint Subsystem I over dt/2) and steps with spin
// (Lie-Trotter I, II, III; symmetric I(dt/2), III(dt/2), II(dt), III(dt/2),
// adjoint I(dt/2)).  A failed step is rolled back: a substep commits nothing on
// failure, and the buffers the committed substeps of the step left behind still
// hold the step's start (Subsystem III turns the spins of the order Subsystem I
// has just written, never those of the step's start), except e_x and the item
// list, which the closing adjoint substep's field kernels overwrite while
// iterating (they are the spare buffers of that substep): e_x is saved before
// it and the list rebuilt from the particles on failure.
int step_unbatched(ecpic_ctx *c, int32_t nsteps, ecpic_iter_stats *sI, ecpic_iter_stats *sII,
                   int32_t *steps_done) {
    const bool sym = c->symmetric, spin = c->spin;
    const double dt = c->dt, h = sym ? 0.5 * c->dt : c->dt;
    for (int n = 0; n < nsteps; ++n) {
        const StepSnap q = snap(c);
        ecpic_iter_stats a{}, b{}, d{};
        int rc = substep_I(c, h, &a, false);
        if (!rc && sym && spin) rc = substep_spin(c, h);
        if (!rc) rc = ecpic_substep_fields(c, dt, &b);
        if (!rc && spin) rc = substep_spin(c, h);
        bool closing = false;
        if (!rc && sym) {
            HIPCHK(hipMemcpyAsync(c->ex_save, c->ex[q.exc], sizeof(double) * (c->M + 2 * HALO),
                                  hipMemcpyDeviceToDevice, c->stream));
            closing = true;
            rc = substep_I(c, h, &d, true);
        }
        if (sI) { sI[n] = a; sI[n].sweeps_adjoint = d.sweeps; }
        if (sII) sII[n] = b;
        if (rc) {
            const bool committed = c->cur != q.cur || c->trc != q.trc;
            restore(c, q);
            if (committed) c->have_prev = false;   // the increments kept are of an order undone
            if (closing) {   // e_x and the item list of the step's start, as they were
                HIPCHK(hipMemcpyAsync(c->ex[c->exc], c->ex_save, sizeof(double) * (c->M + 2 * HALO),
                                      hipMemcpyDeviceToDevice, c->stream));
                HIPCHK(hipMemsetAsync(c->count, 0, sizeof(int32_t) * c->M, c->stream));
                launch_count_cells_xi(c->stream, c->pb[c->cur].xi, c->N, c->M, c->count);
                launch_items_from_counts(c->stream, c->count, c->nstart, c->M, c->chunk, c->N, c->items[c->icur]);
                const int rs = sync(c);
                if (rs) return rs;
            }
            if (steps_done) *steps_done = n;
            return rc;
        }
        if (steps_done) *steps_done = n + 1;
    }
    return ECPIC_OK;
}

// The Subsystem II commit of the step in slot j joined to the start of the
// step in slot j + 1 (one kernel instead of a commit and a start); the
// buffers advance in between, as after a separate commit.
void enqueue_join(ecpic_ctx *c, int j) {
    const int t = c->trc, n = t ^ 1;
    DevStatus *st = c->stII;
    const DevStatus *stI = c->stI;
    DevStatus *mirror = c->hdev;
    const int nsw = c->kII;
    advance(c);
    set_slot(c, j + 1);
    c->kI = 0;
    c->kII = 0;
    const double r = c->dt / (2.0 * c->dx);
    timed(c, "join", [&] {
        launch_step_join(c->P, c->stream, st, stI, mirror, c->stI, c->ey[t], c->ez[t], c->ay[t], c->az[t], c->eyk[0],
                         c->eyk[1], c->ezk[0], c->ezk[1], c->ey[n], c->ez[n], c->ay[n], c->az[n], nsw, c->tol,
                         c->ex[c->exc], c->dt, c->coefA, c->coefE[0], c->coefAk[0], c->m0row.data(),
                         c->krow.data(), r * r, c->dt / (c->dx * c->dx), c->tapsA, c->ntA, c->mloA, c->M, c->E0y,
                         c->E0z);
    });
    enqueue_ws_table(c);
}

}  // namespace

int ecpic_step(ecpic_ctx *c, int32_t nsteps, ecpic_iter_stats *sI, ecpic_iter_stats *sII, int32_t *steps_done) {
    if (!c || nsteps < 0) return ECPIC_EINVAL;
    if (!c->have_particles) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    if (steps_done) *steps_done = 0;
    if (c->symmetric || c->spin) return step_unbatched(c, nsteps, sI, sII, steps_done);
    struct FuseII {   // every commit of a step feeds the step's first Subsystem II iterate
        ecpic_ctx *c;
        explicit FuseII(ecpic_ctx *x) : c(x) { c->fuse_II = true; }
        ~FuseII() { c->fuse_II = false; }
    } fuse(c);
    int done = 0;
    while (done < nsteps) {
        // Enqueue a batch of steps, each gated on the one before having
        // committed, with the current sweep-count guesses; the host reads all
        // their statuses once at the end.
        const int K = std::min(STEP_BATCH, nsteps - done);
        const int gI = std::min(c->guessI, c->kmax), gII = std::min(c->guessII, c->kmax);
        StepSnap snaps[STEP_BATCH];
        c->exact_items = true;
        for (int j = 0; j < K; ++j) {
            snaps[j] = snap(c);
            set_slot(c, j);
            if (j == 0) enqueue_begin(c, true, true);   // later steps are started by the join before them
            enqueue_sweeps_I(c, gI);
            enqueue_commit_I(c);   // also resets the Subsystem II status, gated on the commit
            // Subsystem II runs on the order the commit just made, whose item
            // count only the device knows: launch for the largest count
            IIView v{c->pb[c->cur ^ 1].xi, c->pb[c->cur ^ 1].p, c->items[c->icur ^ 1], false, true, c->items[c->icur]};
            enqueue_iters_II(c, v, gII);
            // the commit writes this step's statuses into the host mirror; the
            // next step's start, gated on it, runs in the same kernel
            if (j + 1 < K) {
                enqueue_join(c, j);
            } else {
                enqueue_commit_II(c);
                advance(c);
            }
            c->exact_items = false;   // the item count of the next step is only known on the device
        }
        int rc = sync(c);
        if (rc) return rc;
        // The next batch enqueues as many sweeps as the most any step of this
        // one needed: a sweep past convergence exits at once, a missing one
        // costs a status round trip.
        int needI = 1, needII = 1;
        for (int j = 0; j < K; ++j) {
            set_slot(c, j);
            c->kI = gI;
            c->kII = gII;
            const DevStatus &I = c->h->I, &II = c->h->II;
            const bool ok = I.committed && II.committed && !I.flags && !II.flags;
            if (ok) {
                step_stats(c, sI ? sI + done + j : nullptr, sII ? sII + done + j : nullptr);
                needI = std::max(needI, I.kconv + 1);
                needII = std::max(needII, II.kconv + 1);
                c->guessI = needI;
                c->guessII = needII;
                if (j == K - 1) {
                    c->n_items_host = I.n_items_next;
                    c->exact_items = true;
                }
                continue;
            }
            // Step j needs more than was enqueued (or failed): the steps behind
            // it were gated off.  Finish it from its own state as a lone step.
            restore(c, snaps[j]);
            c->exact_items = true;
            if (j > 0) c->n_items_host = c->h_ring[j - 1].I.n_items_next;
            IIView v{c->pb[c->cur ^ 1].xi, c->pb[c->cur ^ 1].p, c->items[c->icur ^ 1], false, true, c->items[c->icur]};
            bool again = false;
            rc = finish_I(c, &again);
            if (!rc && again) {   // Subsystem I needed extra sweeps: run II now
                c->kII = 0;
                enqueue_iters_II(c, v, gII);
                enqueue_commit_II(c);
                rc = read_status(c, true);
            }
            if (!rc) rc = finish_II(c, v);
            step_stats(c, sI ? sI + done + j : nullptr, sII ? sII + done + j : nullptr);
            if (rc) {   // nothing swapped: the step is rolled back
                if (steps_done) *steps_done = done + j;
                return rc;
            }
            c->guessI = std::max(needI, c->h->I.kconv + 1);
            c->guessII = std::max(needII, c->h->II.kconv + 1);
            advance(c);
            c->n_items_host = c->h->I.n_items_next;
            c->exact_items = true;
            done += j + 1;
            if (steps_done) *steps_done = done;
            goto next_batch;
        }
        done += K;
        if (steps_done) *steps_done = done;
    next_batch:;
    }
    set_slot(c, 0);
    return ECPIC_OK;
}

// ---- learned warm start ------------------------------------------------------
int ecpic_ws_record(ecpic_ctx *c, int32_t stride, int64_t capacity) {
    if (!c || stride < 0 || (stride > 0 && capacity <= 0)) return ECPIC_EINVAL;
    if (stride > 0 && c->spin) return ECPIC_EINVAL;   // the learned start runs without spin
    hipSetDevice(c->device);
    if (sync(c)) return ECPIC_EDEVICE;
    if (stride == 0) { c->ws_stride = 0; return ECPIC_OK; }
    if (capacity != c->ws_cap) {
        if (c->ws_feat) hipFree(c->ws_feat);
        if (c->ws_targ) hipFree(c->ws_targ);
        c->ws_feat = nullptr; c->ws_targ = nullptr; c->ws_cap = 0;
        if (dalloc(&c->ws_feat, (size_t)capacity * c->wsD) || dalloc(&c->ws_targ, (size_t)capacity * 2))
            return ECPIC_ENOMEM;
        c->ws_cap = capacity;
    }
    c->ws_stride = stride;
    c->ws_phase = 0;
    c->ws_base = 0;
    return ECPIC_OK;
}

int ecpic_ws_records(ecpic_ctx *c, int64_t *n) {
    if (!c || !n) return ECPIC_EINVAL;
    *n = std::min(c->ws_base, c->ws_cap);
    return ECPIC_OK;
}

int ecpic_ws_get_records(ecpic_ctx *c, float *feat, float *targ, int64_t n) {
    if (!c || n < 0 || n > std::min(c->ws_base, c->ws_cap)) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    if (n == 0) return ECPIC_OK;
    if (feat) HIPCHK(hipMemcpyAsync(feat, c->ws_feat, sizeof(float) * n * c->wsD, hipMemcpyDeviceToHost, c->stream));
    if (targ) HIPCHK(hipMemcpyAsync(targ, c->ws_targ, sizeof(float) * n * 2, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

int ecpic_ws_n_params(ecpic_ctx *c, int64_t *n) {
    if (!c || !n) return ECPIC_EINVAL;
    *n = c->wsNP + 2 * (c->wsD + 2) + 2;
    return ECPIC_OK;
}

static int ws_scratch(ecpic_ctx *c, int nblk) {
    if (nblk <= c->ws_pblocks) return ECPIC_OK;
    if (c->ws_pgrad) hipFree(c->ws_pgrad);
    if (c->ws_ploss) hipFree(c->ws_ploss);
    c->ws_pgrad = nullptr; c->ws_ploss = nullptr; c->ws_pblocks = 0;
    if (dalloc(&c->ws_pgrad, (size_t)nblk * c->wsNP) || dalloc(&c->ws_ploss, nblk)) return ECPIC_ENOMEM;
    c->ws_pblocks = nblk;
    return ECPIC_OK;
}

int ecpic_ws_train(ecpic_ctx *c, const ecpic_ws_train_config *tc, float *final_loss) {
    if (!c || !tc || tc->steps < 0 || tc->batch < 0 || tc->batch % 32 || tc->lr < 0.0f) return ECPIC_EINVAL;
    const int64_t n = std::min(c->ws_base, c->ws_cap);
    if (n < 1) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    const int steps = tc->steps ? tc->steps : 2000, B = tc->batch ? tc->batch : 1024;
    const float lr = tc->lr > 0.0f ? tc->lr : 1e-3f;
    int rc = ws_scratch(c, B / 32);
    if (rc) return rc;
    float *mu = c->ws_norm, *sd = c->ws_norm + (c->wsD + 2), *pr = c->ws_norm + 2 * (c->wsD + 2);
    launch_ws_init(c->P, c->stream, c->ws_theta, tc->seed);
    HIPCHK(hipMemsetAsync(c->ws_m, 0, sizeof(float) * c->wsNP, c->stream));
    HIPCHK(hipMemsetAsync(c->ws_v, 0, sizeof(float) * c->wsNP, c->stream));
    launch_ws_stats(c->stream, c->ws_feat, c->ws_targ, n, c->wsD, mu, sd, pr);
    for (int t = 0; t < steps; ++t)
        launch_ws_step(c->P, c->stream, c->ws_theta, c->ws_m, c->ws_v, mu, sd, c->ws_feat, c->ws_targ, n, 0,
                       tc->seed, t, B, c->ws_pgrad, c->ws_ploss, lr, 1, nullptr,
                       (t == steps - 1) ? c->ws_loss : nullptr);
    launch_ws_w2_bf16(c->P, c->stream, c->ws_theta, c->ws_w2b);
    float l = 0.0f;
    if (steps > 0) HIPCHK(hipMemcpyAsync(&l, c->ws_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    rc = sync(c);
    if (rc) return rc;
    if (final_loss) *final_loss = l;
    c->ws_ready = true;
    return ECPIC_OK;
}

int ecpic_ws_get_weights(ecpic_ctx *c, float *w, int64_t n) {
    int64_t need = 0;
    if (!c || !w || ecpic_ws_n_params(c, &need) || n != need) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    HIPCHK(hipMemcpyAsync(w, c->ws_theta, sizeof(float) * c->wsNP, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(w + c->wsNP, c->ws_norm, sizeof(float) * (need - c->wsNP), hipMemcpyDeviceToHost,
                          c->stream));
    return sync(c);
}

int ecpic_ws_set_weights(ecpic_ctx *c, const float *w, int64_t n) {
    int64_t need = 0;
    if (!c || !w || ecpic_ws_n_params(c, &need) || n != need) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    HIPCHK(hipMemcpyAsync(c->ws_theta, w, sizeof(float) * c->wsNP, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->ws_norm, w + c->wsNP, sizeof(float) * (need - c->wsNP), hipMemcpyHostToDevice,
                          c->stream));
    launch_ws_w2_bf16(c->P, c->stream, c->ws_theta, c->ws_w2b);
    int rc = sync(c);
    if (!rc) c->ws_ready = true;
    return rc;
}

int ecpic_ws_enable(ecpic_ctx *c, int32_t on) {
    if (!c) return ECPIC_EINVAL;
    if (on && !c->ws_ready) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    c->ws_on = on != 0;
    return ECPIC_OK;
}

int ecpic_ws_grad(ecpic_ctx *c, const float *x, const float *y, int64_t n, float *grad, float *loss) {
    if (!c || !x || !y || !grad || n < 1 || n > (1 << 20)) return ECPIC_EINVAL;
    if (!c->ws_ready) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    const int D = c->wsD, nblk = (int)((n + 31) / 32);
    int rc = ws_scratch(c, nblk);
    if (rc) return rc;
    float *dx = nullptr, *dy = nullptr, *dn = nullptr, *dg = nullptr;
    rc = dalloc(&dx, (size_t)n * D) | dalloc(&dy, (size_t)n * 2) | dalloc(&dn, 2 * (D + 2)) | dalloc(&dg, c->wsNP);
    if (!rc) {
        std::vector<float> norm(2 * (D + 2), 0.0f);
        for (int i = 0; i < D + 2; ++i) norm[D + 2 + i] = 1.0f;   // inputs given normalised
        hipMemcpyAsync(dx, x, sizeof(float) * n * D, hipMemcpyHostToDevice, c->stream);
        hipMemcpyAsync(dy, y, sizeof(float) * n * 2, hipMemcpyHostToDevice, c->stream);
        hipMemcpyAsync(dn, norm.data(), sizeof(float) * norm.size(), hipMemcpyHostToDevice, c->stream);
        launch_ws_step(c->P, c->stream, c->ws_theta, c->ws_m, c->ws_v, dn, dn + D + 2, dx, dy, n, 1, 0, 0, 0,
                       c->ws_pgrad, c->ws_ploss, 0.0f, 0, dg, c->ws_loss);
        hipMemcpyAsync(grad, dg, sizeof(float) * c->wsNP, hipMemcpyDeviceToHost, c->stream);
        float l = 0.0f;
        hipMemcpyAsync(&l, c->ws_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream);
        rc = sync(c);
        if (loss) *loss = l;
    } else {
        rc = ECPIC_ENOMEM;
    }
    for (void *q : {(void *)dx, (void *)dy, (void *)dn, (void *)dg}) if (q) hipFree(q);
    return rc;
}

int ecpic_ws_table(ecpic_ctx *c, float *table) {
    if (!c || !table) return ECPIC_EINVAL;
    if (!c->ws_ready) return ECPIC_ESTATE;
    hipSetDevice(c->device);
    WsNet net{c->ws_theta, c->ws_norm, c->ws_norm + (c->wsD + 2), c->ws_norm + 2 * (c->wsD + 2)};
    launch_prep_records(c->P, c->stream, nullptr, c->ay[c->trc], c->az[c->trc], c->ex[c->exc], c->coefA,
                        c->coefE[0], c->M);
    launch_ws_table(c->P, c->stream, net, c->ws_w2b, c->coefA, c->ay[c->trc], c->az[c->trc], c->ex[c->exc], c->M, c->ws_table);
    HIPCHK(hipMemcpyAsync(table, c->ws_table, sizeof(float) * c->M * WS_NT * WS_NP, hipMemcpyDeviceToHost,
                          c->stream));
    return sync(c);
}

int ecpic_profile_enable(ecpic_ctx *c, int32_t enable) {
    if (!c) return ECPIC_EINVAL;
    sync(c);
    c->prof.on = enable != 0;
    if (c->prof.on) c->prof.acc.clear();
    return ECPIC_OK;
}

int ecpic_bandwidth_probe(ecpic_ctx *c, int64_t bytes, int32_t reps, double *ms_per_copy) {
    if (!c || bytes < 16 || reps < 1 || !ms_per_copy) return ECPIC_EINVAL;
    hipSetDevice(c->device);
    const int64_t n = (bytes / 16) * 2;
    double *a = nullptr, *b = nullptr;
    if (dalloc(&a, n) || dalloc(&b, n)) { if (a) hipFree(a); return ECPIC_ENOMEM; }
    hipMemsetAsync(a, 0, sizeof(double) * n, c->stream);
    launch_copy(c->stream, a, b, n);
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    hipEventRecord(e0, c->stream);
    for (int r = 0; r < reps; ++r) launch_copy(c->stream, (r & 1) ? b : a, (r & 1) ? a : b, n);
    hipEventRecord(e1, c->stream);
    int rc = sync(c);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    *ms_per_copy = (double)ms / reps;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(a);
    hipFree(b);
    return rc;
}

int ecpic_kernel_time(ecpic_ctx *c, const char *name, double *ms, int64_t *launches) {
    if (!c || !name || !ms || !launches) return ECPIC_EINVAL;
    sync(c);
    auto it = c->prof.acc.find(name);
    *ms = it == c->prof.acc.end() ? 0.0 : it->second.first;
    *launches = it == c->prof.acc.end() ? 0 : it->second.second;
    return ECPIC_OK;
}

}  // extern "C"
