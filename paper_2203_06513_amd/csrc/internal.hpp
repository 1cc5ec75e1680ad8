// Internal definitions shared by the runtime and the kernels of libecpic.
//
// Data layout in HBM (one context):
//   particles   SoA, cell-sorted, double-buffered:  xi = x/dx in [0, M) (f64),
//               p (f64), id (i32, index given at set_particles); the Picard
//               iterate d = delta/dx (f64) lives in two more buffers.
//   work items  the sorted array is cut into items (cell, [begin, end)) of at
//               most `chunk` particles of one cell; one thread block per item.
//   fields      every coefficient vector is stored padded with HALO periodic
//               copies on both sides, f_pad[j + HALO] = f[j mod M] for
//               j in [-HALO, M + HALO), so a cell's window is contiguous.
//   partials    per item, the (deg+2) current / (deg+1) charge sums of its
//               particles, assembled per cell in a fixed order (deterministic,
//               no floating-point atomics).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecpic {

constexpr int HALO = 8;
constexpr int MAX_DEG = 5;
constexpr int MAX_HIST = 128;
// Particles of one work item (a cell, or a part of a cell holding more): at least
// MIN_CHUNK, raised to twice the mean particles per cell (a power of two, at most
// MAX_CHUNK) so that cells normally hold one item each.
constexpr int MIN_CHUNK = 2048;
constexpr int MAX_CHUNK = 16384;

// Error bits raised by kernels.
enum : int32_t { FLAG_NONFINITE = 1, FLAG_CFL = 2, FLAG_ORDER = 4 };
// Not an error: a sweep's wave partials carry it when the wave redid crossing
// lanes through its queue; the field kernel moves it into DevStatus::queued.
constexpr int32_t FLAG_QUEUED = 8;
constexpr int32_t FLAG_ERRORS = FLAG_NONFINITE | FLAG_CFL | FLAG_ORDER;

// Picard bookkeeping of one substep, device-resident.  The host enqueues
// sweeps with their index k; sweep k first decides whether sweep k-1 already met
// the tolerance (from the maxima of sweep k-1, kept in slot (k-1)&1) and, if so,
// records kconv = k-1 and does nothing.  Every kernel of the substep is a no-op
// once kconv >= 0 or an error flag is set, so the host can enqueue sweeps ahead
// of knowing the outcome and synchronise once per step.
struct DevStatus {
    unsigned long long rx_bits[2];   // max |d^(k+1) - d^(k)| (cell units) of sweep k, slot k&1, as bits
                                     // (gathered from the sweep's partials by the field kernel)
    unsigned long long re_bits[2];   // max field increment of sweep k, slot k&1, as bits
    int32_t kconv;                   // sweep index that met the tolerance, -1 before
    int32_t committed;
    int32_t flags;                   // FLAG_* bits
    int32_t gate;                    // substep allowed to run (Subsystem II waits on I)
    int32_t fp32_sweeps;             // sweeps done in FP32 (precision form)
    int32_t n_items_next;            // item count of the re-sorted particles (Subsystem I commit)
    int32_t scan_multi;              // a field kernel of the substep saw a cell with other than one item
    int32_t queued;                  // some sweep of the substep redid crossing lanes through its queue
    double res;                      // residual of sweep kconv (length / field units)
    double res_first[4];             // residuals of the first four FP64 sweeps (0 if not run)
    double res_hist[MAX_HIST];       // residual of each evaluated sweep
};

struct ItemList {
    int32_t *cell;        // [max_items]
    int32_t *begin;       // [max_items + 1]
    int32_t *cell_first;  // [M + 1]: first item of each cell
    int32_t *n_items;     // device [2]: the item count, and 1 if every cell has exactly one item
                          // (item c is then cell c), else 0
};

struct Particles {
    double *xi;
    double *p;
    int32_t *id;
    double *sx, *sy, *sz;   // spins (null without spin); Subsystem I carries them with the sort
};

// ---- learned warm start ----------------------------------------------------
// A multilayer perceptron D -> 64 -> 64 -> 2 (GELU, tanh form) predicts the
// converged increment of Subsystem I from a particle's local state.  It is
// evaluated per cell on a WS_NT x WS_NP grid of (local coordinate, momentum)
// nodes and the particles interpolate their cell's table.
constexpr int WS_H = 64;
constexpr int WS_NT = 8, WS_NP = 8;
__host__ __device__ constexpr int ws_d(int P) { return 3 + 6 * (P + 1); }
__host__ __device__ constexpr int ws_nparams(int D) { return WS_H * D + WS_H + WS_H * WS_H + WS_H + 2 * WS_H + 2; }

struct WsNet {
    const float *theta;      // [W1 (H x D) | b1 | W2 (H x H) | b2 | W3 (2 x H) | b3]
    const float *mu, *sd;    // [D + 2] normalisation of the features, then of the targets
    const float *prange;     // [2] momentum range of the table nodes
};

struct WsRecord {
    float *feat, *targ;      // [cap][D], [cap][2]
    int64_t cap;
    int64_t base;            // first slot of this step
    int32_t stride, phase;   // record the particles with id % stride == phase (stride 0: off)
    const double *ay, *az, *ex;   // padded a_perp^n, e_x^n
};

// ---- Subsystem I ---------------------------------------------------------
struct SweepIArgs {
    const double *xi, *p;
    double *d0, *d1;               // iterate buffers, d^(k) = k&1 ? d1 : d0
    float *f0, *f1;                // single precision iterate buffers (precision form), same parity
    const float *d32in;            // FP64 sweep reading d^(k) from a single precision buffer, or null
    ItemList items;
    const double *coefA;           // A-records of a_perp^n
    const double *coefE0, *coefE1; // E-records of ebar^(k) = (e^n + e^(k))/2, by parity of k
    double *part;                  // [max_items][waves per item][deg+4]: P+2 current slots, residual, flags
    int32_t *wcnt;                 // [max_items][waves per item][3] movers left / stay / right, per wave,
                                   // of the increment a commit after this sweep would take
    DevStatus *st;
    double dt, dt_dx, inv_dx, dx, tol;
    double dx_dt;                  // 1 / dt_dx (the adjoint scheme's velocity from an increment)
    int32_t explicit_start;        // 1: d^(0) = dt p / gamma; 0: d^(0) read from d0
    const double *dprev;           // non-null: d^(0) is the increment the last commit took (same order)
    int32_t k;                     // sweep index
    int32_t first64;               // index of the first FP64 sweep (0 for the plain method)
    // predictor pass of the learned warm start
    WsNet ws;
    const float *ws_table;         // [M][WS_NT * WS_NP] network outputs of this substep
    // spin force (sweeps compiled with it): s_y, s_z and hbar / dx^2
    const double *sy, *sz;
    double hbar_dx2;
};

struct FieldIArgs {
    ItemList items;
    const double *part;
    const double *taps;            // first row of the (dimensionless) M1 inverse
    int32_t ntaps, mlo;            // e_j = en_j - w sum_i taps[i] S_{j - (mlo + i)}
    const double *en;
    double *ek0, *ek1;
    double *coefE0, *coefE1;
    DevStatus *st;
    double w;
    int32_t M;
    int32_t k;
    int32_t wpi;                   // waves per item of the sweep (partials per item)
    // what a commit after this sweep needs (FP64 sweeps, k >= first64): the
    // destinations of each cell's movers, the new counts and starts, the new
    // item list if it has one item per cell, and e_x^{n+1}
    int32_t first64;
    const int32_t *wcnt;           // the sweep's per-wave mover counts
    int32_t *cbase;                // [M][3]
    int32_t *nstart;               // [2M + 1]: new start of each cell, N, new count of each cell
    int32_t *base;                 // [max_items][3] (only when some cell has several items)
    ItemList items_next;
    double *ex_next;               // padded
    int32_t chunk;
};

struct CommitIArgs {
    Particles cur, nxt;
    const double *d0, *d1;
    ItemList items, items_next;
    const double *coefA, *coefE0, *coefE1;
    DevStatus *stII;               // reset here, gated on this commit (null: leave it)
    const int32_t *wcnt;           // per-wave mover counts of the converged sweep (see SweepIArgs)
    int32_t *base;                 // [max_items][3] each item's movers of each kind before it in its cell
                                   // (written only when some cell has several items)
    int32_t *cbase;                // [M][3] destination of each cell's first mover of each kind
    int32_t *nstart;               // [2M + 1]: new start of each cell, N, new count of each cell
    DevStatus *st;
    double dt, dt_dx, inv_dx, dx, tol;
    double hbar_dx2;               // spin force (commits compiled with it; cur/nxt carry the spins)
    double dx_dt;                  // 1 / dt_dx
    int32_t M, chunk, seidel, wpi;
    int32_t nsweeps;               // sweeps enqueued so far (the last one may still need its test)
    int32_t first64;               // index of the first FP64 sweep
    int32_t list_kernel;           // a separate kernel builds a new item list with several items per cell
    // the first Subsystem II deposit at the committed positions (part2 null: not formed)
    const double *coefAk0;         // A-records of a^(0) = a^n - dt e^n
    double *part2;                 // [items][waves per item][2 (deg+3)], by the current item list
    WsRecord rec;                  // training pairs to record (rec.stride 0: none)
    double *dprev_out;             // non-null: the committed increment, in the new order
    int64_t N;
};

// ---- spin (Subsystem III, the Subsystem II source, the Zeeman energy) -------
struct SpinArgs {
    const double *xi;
    double *sx, *sy, *sz;
    ItemList items;
    const double *ay, *az;   // padded a_perp (current)
    double inv_dx;
    double h;                // rotation time (Subsystem III)
    double *spart;           // [items][2 deg] V1 sums of (s_y, s_z) per item (deposit pass)
    double *epart;           // [items] Zeeman sum per item (energy pass)
};

// ---- Subsystem II --------------------------------------------------------
struct SweepIIArgs {
    const double *xi, *p;
    ItemList items;
    const double *coefAn;                     // A-records of a_perp^n (those of Subsystem I)
    const double *coefAk0, *coefAk1;          // A-records of a^(k) = a^n - dt/2 (e^n + e^(k)), by parity
    double *part;                             // [max_items][waves per item][2 (deg+1)]
    DevStatus *st;
    double tol;
    int32_t k;
};

struct FieldIIArgs {
    ItemList items;
    const double *part;
    const double *taps;                       // first row of (M0^ + r^2 K^)^{-1}
    int32_t ntaps, mlo;
    const double *E0y, *E0z;                  // A^{-1} (constant right-hand side), unpadded
    const double *eyn, *ezn, *ayn, *azn;      // padded state at the substep start
    double *ey0, *ey1, *ez0, *ez1;            // padded iterates
    double *coefAk0, *coefAk1;
    DevStatus *st;
    double coef;                              // dt w / dx
    double half_dt;
    int32_t M;
    int32_t k;
    int32_t wpi;                              // waves per item of the particle pass
    int32_t wide;                             // iterate 0 from the commit's partials: items is the list
                                              // of the order before the commit, 2 (deg+3) per wave
};

// Kernel launches go through launch_k.  When a profiled launch has set the
// events below (runtime.hip, timed()), the dispatch packets themselves take the
// timestamps: the start event with the first kernel of the launch, the stop
// event with every one, so it ends at the last.  Unset, it is a plain launch.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents g_launch_events;

template <typename F, typename... Args>
inline void launch_k(F kernel, const dim3 &grid, const dim3 &block, size_t lds, hipStream_t s, Args... args) {
    LaunchEvents &e = g_launch_events;
    if (!e.start && !e.stop) {
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
        return;
    }
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, e.start, e.stop, 0u, args...);
    e.start = nullptr;
}

}  // namespace ecpic
