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

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecpic {

constexpr int HALO = 8;
constexpr int MAX_DEG = 5;
constexpr int MAX_HIST = 128;

// Error bits raised by kernels.
enum : int32_t { FLAG_NONFINITE = 1, FLAG_CFL = 2, FLAG_ORDER = 4 };

// Picard bookkeeping of one substep, device-resident.  Kernels read it to pick
// buffers and to skip work once the substep has converged or failed, so that
// the host can enqueue sweeps ahead of knowing the outcome.
struct DevStatus {
    unsigned long long rx_bits;   // running max |d^(k+1) - d^(k)| (cell units), as bits
    unsigned long long re_bits;   // running max field increment, as bits
    int32_t k;                    // sweeps completed
    int32_t converged;
    int32_t kconv;                // sweep index that met the tolerance
    int32_t committed;
    int32_t flags;                // FLAG_* bits
    uint32_t counter;             // blocks finished in the current field kernel
    int32_t gate;                 // substep allowed to run (Subsystem II waits on I)
    int32_t fp32_sweeps;          // sweeps done in FP32 (precision form)
    double res;                   // last residual (length / field units)
    double res_hist[MAX_HIST];
};

struct ItemList {
    int32_t *cell;        // [max_items]
    int32_t *begin;       // [max_items + 1]
    int32_t *cell_first;  // [M + 1]: first item of each cell
    int32_t *n_items;     // device scalar
};

struct Particles {
    double *xi;
    double *p;
    int32_t *id;
};

// ---- Subsystem I ---------------------------------------------------------
struct SweepIArgs {
    const double *xi, *p;
    double *d0, *d1;               // iterate buffers, d^(k) = k&1 ? d1 : d0
    ItemList items;
    const double *ay, *az;         // padded a_perp^n
    const double *en;              // padded e_x^n
    const double *ek0, *ek1;       // padded e_x iterates, e^(k) = k==0 ? en : (k&1 ? ek1 : ek0)
    double *part;                  // [max_items][deg+2]
    DevStatus *st;
    double dt, dt_dx, inv_dx;
    int32_t explicit_start;        // 1: d^(0) = dt p / gamma; 0: d^(0) read from d0
};

struct FieldIArgs {
    ItemList items;
    const double *part;
    const double *taps;            // first row of the (dimensionless) M1 inverse
    int32_t ntaps, mlo;            // e_j = en_j - w sum_i taps[i] S_{j - (mlo + i)}
    const double *en;
    double *ek0, *ek1;
    DevStatus *st;
    double w, tol, dx;
    int32_t M;
};

struct CommitIArgs {
    Particles cur, nxt;
    const double *d0, *d1;
    ItemList items, items_next;
    const double *ay, *az, *en, *ek0, *ek1;
    double *ex_next;               // padded e_x^{n+1}
    int32_t *cnt;                  // [max_items][3] movers left / stay / right
    int32_t *tot;                  // [M][3]
    int32_t *base;                 // [max_items][3]
    int32_t *nstart;               // [M + 1]
    DevStatus *st;
    double dt, dt_dx, inv_dx;
    int32_t M, chunk, seidel, explicit_start;
    int64_t N;
};

// ---- Subsystem II --------------------------------------------------------
struct SweepIIArgs {
    const double *xi, *p;
    ItemList items;
    const double *ayn, *azn, *eyn, *ezn;      // padded state at the substep start
    const double *ey0, *ey1, *ez0, *ez1;      // padded iterates
    double *part;                             // [max_items][2 (deg+1)]
    DevStatus *st;
    const DevStatus *gate;                    // Subsystem I status (must be committed)
    double half_dt;
};

struct FieldIIArgs {
    ItemList items;
    const double *part;
    const double *taps;                       // first row of (M0^ + r^2 K^)^{-1}
    int32_t ntaps, mlo;
    const double *E0y, *E0z;                  // A^{-1} (constant right-hand side), unpadded
    const double *eyn, *ezn;
    double *ey0, *ey1, *ez0, *ez1;
    DevStatus *st;
    const DevStatus *gate;
    double coef;                              // dt w / dx
    double tol;
    int32_t M;
};

}  // namespace ecpic
