/*
 * ecpic.h -- C-ABI of the MI355X (gfx950) library for the energy-conserving
 * particle-in-cell step of the reduced 1D relativistic Vlasov-Maxwell model
 * without spin (Li, "Energy conserving particle-in-cell methods for
 * relativistic Vlasov-Maxwell equations of laser-plasma interaction").
 *
 * State (Section 3.1, eq. dis): particle positions x_a and momenta p_a with a
 * common weight w, V1 coefficients e_x and V0 coefficients e_y, e_z, a_y,
 * a_z on a periodic uniform grid of M cells, B-splines of degree p (V0) and
 * p-1 (V1).  Units are those of the reduced model (Section 2.1): c = 1,
 * plasma frequency 1 at density 1, ions a uniform neutralising background.
 *
 * Every call returns an ecpic_status.  Unless stated otherwise:
 *   - host arrays are read or written during the call only and never kept;
 *   - device pointers (the *_dev calls) must be device memory of the context's
 *     device, stay valid for the call, and are accessed on the context's stream;
 *   - ECPIC_EINVAL leaves the state unchanged;
 *   - a context is bound to one device and one stream and is not thread-safe.
 * All computation of the step runs in HIP kernels on the GPU; there is no CPU
 * fallback, and ecpic_create fails with ECPIC_EDEVICE when no gfx950 device
 * is usable.
 *
 * Two choices a particle code usually exposes are fixed here:
 *   - the particles are re-sorted by cell at every Subsystem I commit (a
 *     stable three-way merge, since a particle moves at most one cell per
 *     step), so there is no sort interval to set;
 *   - every deposit is deterministic (per-wave partial sums assembled per cell
 *     in a fixed order, no floating-point atomics on the step's path), so two
 *     runs from one state agree bit for bit.
 */
#ifndef ECPIC_H
#define ECPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ecpic_ctx ecpic_ctx;

typedef enum {
    ECPIC_OK = 0,
    ECPIC_EINVAL = -1,     /* bad argument or configuration; state unchanged */
    ECPIC_ENOMEM = -2,     /* device or host allocation failed */
    ECPIC_ENOTCONV = -3,   /* Picard iteration hit picard_max_iter; the step is rolled back */
    ECPIC_EDEVICE = -4,    /* HIP runtime error or no usable device */
    ECPIC_ENONFINITE = -5, /* a NaN/Inf appeared; state undefined until set again */
    ECPIC_ECFL = -6,       /* a particle tried to move a full cell or more in one step */
    ECPIC_ESTATE = -7      /* call out of order (e.g. step before set_particles) */
} ecpic_status;

/* Arithmetic of the particle sweeps of Subsystem I. */
typedef enum {
    ECPIC_FP64 = 0,       /* every sweep in FP64 */
    ECPIC_FP32_MIXED = 1  /* FP32 gather/push/deposit sweeps with compensated (two-sum) cell
                             accumulation, then FP64 sweeps until the FP64 test passes; the
                             residual test, field update and diagnostics stay FP64 */
} ecpic_precision;

/* Initial Picard iterate of Subsystem I. */
typedef enum {
    ECPIC_WS_EXPLICIT = 0, /* delta^(0) = dt p / gamma(x^n, p^n), e^(0) = e_x^n */
    ECPIC_WS_PREVIOUS = 1, /* delta^(0) = the increment the previous Subsystem I substep committed
                              for the same particle (explicit after set_particles), e^(0) = e_x^n */
    ECPIC_WS_MLP = 2       /* delta^(0) from the learned predictor (see ecpic_ws_*) */
} ecpic_warmstart;

/* Ordering of the Picard map of Subsystem I.  Both converge to the same fixed
 * point of the scheme (Section 4.2, Subsystem I); they differ in which
 * increment feeds the current of a sweep. */
typedef enum {
    ECPIC_MAP_JACOBI = 0, /* current of sweep k from delta^(k); commit x^n + delta^(k),
                             the momentum of sweep k and e^(k+1) */
    ECPIC_MAP_SEIDEL = 1  /* current of sweep k from delta^(k+1), the increment the sweep
                             has just produced; commit x^n + delta^(k+1), e^(k+1) and the
                             momentum re-evaluated from both */
} ecpic_map;

/* Composition of the substeps into a time step. */
typedef enum {
    ECPIC_LIE_TROTTER = 0, /* Subsystem I over dt, then II over dt (Section 5; first order) */
    ECPIC_SYMMETRIC = 1    /* Subsystem I over dt/2, II over dt, then the adjoint of Subsystem I
                              over dt/2 (ecpic_substep_particles_adjoint): a map composed with
                              its adjoint around the symmetric Subsystem II, second order; each
                              substep conserves the discrete energy as in Section 4.1 */
} ecpic_splitting;

typedef struct {
    double L;                 /* domain length; grid x_j = j L/M (Section 3.1) */
    int32_t M;                /* cells = number of V0 and V1 coefficients; M >= degree + 3 */
    int32_t degree;           /* V0 spline degree p in [2, 5]; V1 has degree p - 1 */
    int64_t n_particles;      /* N >= 0 */
    double weight;            /* w_a for all particles; 0 => L / N (mean density 1) */
    double dt;                /* time step; must satisfy dt < L/M (at most one cell per step) */
    double picard_tol;        /* absolute max-norm tolerance on the increments (Section 5) */
    int32_t picard_max_iter;  /* sweeps per substep before ECPIC_ENOTCONV; 0 => 50 */
    int32_t precision;        /* ecpic_precision */
    int32_t warmstart;        /* ecpic_warmstart */
    int32_t map;              /* ecpic_map */
    int32_t device;           /* HIP device ordinal */
    void *stream;             /* hipStream_t to run on (e.g. torch's); NULL => library-owned */
    int32_t fp32_sweeps;      /* ECPIC_FP32_MIXED: FP32 sweeps that open every Subsystem I substep
                                 before the FP64 ones; 0 => 2.  Ignored for ECPIC_FP64. */
    int32_t sweep_guess;      /* sweeps / iterations enqueued per substep before the first status
                                 read of a step; later steps use what earlier ones needed; 0 => 4 */
    int32_t waves_per_item;   /* launch shape of the particle passes: 64-lane waves per work item
                                 (a cell or a slice of at most 2048 of its particles), 1..4;
                                 0 => chosen from the item count (about four waves per SIMD).
                                 Results do not depend on it beyond rounding order. */
    int32_t splitting;        /* ecpic_splitting */
    int32_t item_particles;   /* launch shape: at most this many particles of one cell per work item
                                 (a power of two in [2048, 16384]); 0 => twice the mean particles per
                                 cell, so that cells normally hold one item.  Results do not depend
                                 on it beyond rounding order. */
    int32_t spin;             /* 1: the particles carry spins s_a (Section 2.1; ecpic_set_spins) and
                                 a step is Subsystems I, II, III (symmetric: I(dt/2), III(dt/2),
                                 II(dt), III(dt/2), adjoint I(dt/2)); 0: no spin.  Spin runs the
                                 plain FP64 sweeps: ECPIC_FP32_MIXED and ECPIC_WS_MLP are EINVAL. */
    double hbar;              /* normalised Planck constant of the Zeeman energy
                                 hbar sum_a w (s_y dA_z/dx - s_z dA_y/dx)(x_a) (eq. discrete_H);
                                 must be 0 without spin.  With hbar = 0 the spins still precess
                                 (Subsystem III) but act on nothing. */
} ecpic_config;

typedef struct {
    int32_t sweeps;   /* Picard sweeps (Subsystem I) or iterations (Subsystem II) */
    int32_t fp32_sweeps; /* of which in FP32 (precision form) */
    double residual;  /* last max-norm increment (length / field units) */
    int32_t crossing_queue; /* Subsystem I: nonzero if some sweep redid the particles whose step
                               crosses a cell boundary through its per-wave queue (degree >= 4,
                               when some step crosses); 0 for Subsystem II */
    int32_t sweeps_adjoint; /* ecpic_step with ECPIC_SYMMETRIC, Subsystem I entries: sweeps of the
                               step's closing adjoint substep (sweeps is the opening one's); else 0 */
    double residual_hist[4];  /* Subsystem I: residuals of the substep's first four FP64 sweeps (the
                                 max-norm change each made to the iterate it started from,
                                 increments in length units or the field, whichever is larger;
                                 0 past the last sweep): how far each iterate was from the fixed
                                 point, to a factor 1 +- rho, rho the contraction of the map.
                                 Zero for Subsystem II. */
} ecpic_iter_stats;

typedef struct {
    double kinetic;   /* sum_a w (gamma_a - 1) */
    double e_long;    /* 1/2 e_x^T M1 e_x */
    double e_trans;   /* 1/2 (e_y^T M0 e_y + e_z^T M0 e_z) */
    double b_trans;   /* 1/2 (a_y^T K a_y + a_z^T K a_z), K = G^T M1 G */
    double total;     /* discrete Hamiltonian H (eq. discrete_H), the Zeeman term included */
    double zeeman;    /* hbar sum_a w (s_y dA_z/dx - s_z dA_y/dx)(x_a) (0 without spin) */
} ecpic_energy_parts;

/* Create a context on cfg->device; allocates every device buffer it needs for
 * N particles and M cells.  *out receives the context.  Errors: EINVAL for an
 * invalid config (degree outside [2,5], M < degree + 3, dt >= L/M, N < 0,
 * non-positive L or tol), EDEVICE when the device is missing or not gfx950,
 * ENOMEM. */
int ecpic_create(const ecpic_config *cfg, ecpic_ctx **out);

/* Release every resource of ctx (NULL is allowed). */
int ecpic_destroy(ecpic_ctx *ctx);

/* Particle state (f_h of eq. f_dirac).  x: positions, any real (wrapped into
 * [0, L)); p: momenta p_x; n must equal n_particles.  Host arrays, copied.  The
 * library keeps particles cell-sorted internally and remembers each particle's
 * index, so get_particles returns them in the order given here. */
int ecpic_set_particles(ecpic_ctx *ctx, const double *x, const double *p, int64_t n);
int ecpic_get_particles(ecpic_ctx *ctx, double *x, double *p, int64_t n);
/* Same, with device arrays of length n (float64). */
int ecpic_set_particles_dev(ecpic_ctx *ctx, const double *x, const double *p, int64_t n);
int ecpic_get_particles_dev(ecpic_ctx *ctx, double *x, double *p, int64_t n);

/* Spins s_a = (s_x, s_y, s_z) of the particles (eq. f_dirac; needs cfg.spin),
 * host arrays of n = n_particles entries each, in the order of set_particles
 * (copied).  set_particles sets every spin to zero.  get_spins returns them in
 * that order.  EINVAL without spin or if n differs; ESTATE before set_particles. */
int ecpic_set_spins(ecpic_ctx *ctx, const double *sx, const double *sy, const double *sz, int64_t n);
int ecpic_get_spins(ecpic_ctx *ctx, double *sx, double *sy, double *sz, int64_t n);

/* Field coefficients (eqs. fem_e, fem_a), host arrays of length M; a NULL input
 * sets that field to zero, a NULL output skips it. */
int ecpic_set_fields(ecpic_ctx *ctx, const double *ex, const double *ey, const double *ez,
                     const double *ay, const double *az);
int ecpic_get_fields(ecpic_ctx *ctx, double *ex, double *ey, double *ez, double *ay, double *az);

/* Set e_x to the solution of the discrete Poisson equation of the second remark
 * of Section 4.2, G^T M1 e_x = dx 1 - Lambda0(X)^T W 1, in the zero-mean gauge
 * (the right-hand side is taken minus its mean if the weights do not
 * neutralise the background exactly). */
int ecpic_solve_gauss(ecpic_ctx *ctx);

/* Subsystem I (Section 4.2): solve the implicit discrete-gradient update of
 * (x, p, e_x) over time step dt with a_perp frozen, by Picard sweeps to
 * picard_tol.  0 < dt < L/M (EINVAL otherwise); the configured dt is not
 * changed.  stats may be NULL.  ENOTCONV rolls back to the state before the
 * call; ENONFINITE / ECFL leave the state as before the call as well (nothing
 * is committed), but the caller should set it again before going on. */
int ecpic_substep_particles(ecpic_ctx *ctx, double dt, ecpic_iter_stats *stats);

/* The adjoint of the Subsystem I scheme over dt.  The scheme's discrete
 * gradient (Section 4.1, as used for Subsystem I in Section 4.2) varies x first,
 * at p^n, then p, at x^{n+1}; the adjoint varies p first, at x^n, then x, at
 * p^{n+1}:
 *   delta / dt = (p^n + p^{n+1}) / (gamma(x^n, p^n) + gamma(x^n, p^{n+1})),
 *   (p^{n+1} - p^n) / dt = lbar.ebar - (A(x^{n+1}) + A(x^n)).DA
 *                          / (gamma(x^n, p^{n+1}) + gamma(x^{n+1}, p^{n+1})),
 * with the same line means lbar, difference quotient DA and e_x equation.  It
 * is the scheme run backwards: ecpic_substep_particles over -dt would undo it.
 * Iterated on delta (p^{n+1} follows from delta in closed form) by FP64 sweeps
 * from delta^(0) = dt p / gamma, each depositing the current of the increment
 * it produces; it commits x^n + delta^(k+1), the momentum that increment stands
 * for, and e^(k+1), so Gauss's law holds exactly and energy to the tolerance.
 * Precision form, learned and previous-step starts do not apply; the increment
 * it commits is kept for a following ECPIC_WS_PREVIOUS start.  Errors as for
 * ecpic_substep_particles. */
int ecpic_substep_particles_adjoint(ecpic_ctx *ctx, double dt, ecpic_iter_stats *stats);

/* Subsystem II (Section 4.2): solve the update of (e_y, e_z, a_y, a_z) over time
 * step dt with the particles frozen, by fixed-point iteration on e_perp with the
 * matrix M0 + dt^2 K / 4 inverted exactly and the particle term lagged.  The
 * inverse for a dt not seen before is computed once (host DFT, O(M^2)) and kept.
 * 0 < dt < L/M.  ENOTCONV rolls back. */
int ecpic_substep_fields(ecpic_ctx *ctx, double dt, ecpic_iter_stats *stats);

/* Subsystem III over dt (Section 4.2, eq. spin_rodrigue; needs cfg.spin): every
 * spin turns about r_a = (0, dA_z/dx, -dA_y/dx)(x_a) by the exact rotation
 * exp(dt rhat_a); positions, momenta and fields do not change, and neither do
 * |s_a| nor the energy.  dt may be any real (negative undoes a positive one).
 * With hbar != 0, ecpic_substep_fields also applies the spin source of
 * Subsystem II, -/+ hbar G^T Lambda1(X)^T W S_{z/y}, and ecpic_substep_particles
 * the spin force. */
int ecpic_substep_spin(ecpic_ctx *ctx, double dt);

/* nsteps time steps composed as cfg.splitting says (with cfg.spin the
 * Subsystem III substeps too; without it Subsystem III is the identity).  per_step_I / per_step_II: arrays of nsteps entries
 * or NULL.  On ENOTCONV the failing step is rolled back and *steps_done (if
 * not NULL) tells how many steps completed.  Lie-Trotter steps are enqueued in
 * batches of up to 16, each gated on the device on the one before having
 * committed; a step that needs more sweeps than were enqueued is finished
 * alone and the batch resumes after it, so the result does not depend on the
 * batching.  Symmetric steps and steps with spin run their substeps one after
 * the other, with a status read after each. */
int ecpic_step(ecpic_ctx *ctx, int32_t nsteps, ecpic_iter_stats *per_step_I,
               ecpic_iter_stats *per_step_II, int32_t *steps_done);

/* Current of straight segments: J_j = w sum_a int_{x0_a}^{x1_a} Lambda1_j (the
 * time-averaged basis of the Subsystem I scheme times the displacement).  x0,
 * x1: host arrays of n unwrapped positions with |x1 - x0| < dx; J: host array
 * of length M, overwritten. */
int ecpic_deposit_current(ecpic_ctx *ctx, const double *x0, const double *x1, int64_t n,
                          double *J);

/* The current of ecpic_deposit_current for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  x0, x1: device arrays of n doubles, J: device array of M
 * doubles (overwritten), flags: device int32 or NULL, all on the context's
 * device.  The call only enqueues two kernels on the context's stream and
 * returns: it allocates nothing, copies nothing to the host and does not wait,
 * so J and *flags are ready when the stream reaches that point.  *flags gets 2
 * (the ECPIC_ECFL cause) if some segment ends outside the neighbour cells of its
 * start (that segment is left out), else 0.  Per-block partial currents live in
 * a fixed static device buffer of 64 x 16384 doubles (8 MiB per device, held
 * until the process ends), shared by every call on that device: calls that
 * overlap on one device race.  EINVAL if M > 16384 (the buffer's limit) or for a
 * bad argument; EDEVICE if the buffer could not be located on this device. */
int ecpic_deposit_current_noalloc(ecpic_ctx *ctx, const double *x0, const double *x1, int64_t n, double *J,
                                  int32_t *flags);

/* Charge rho = Lambda0(X)^T W 1 of the current particles (second remark of
 * Section 4.2); rho: host array of length M. */
int ecpic_deposit_charge(ecpic_ctx *ctx, double *rho);

/* Discrete Hamiltonian (eq. discrete_H), with the Zeeman term when cfg.spin is set
 * (its value also in out->zeeman). */
int ecpic_energy(ecpic_ctx *ctx, ecpic_energy_parts *out);

/* Gauss-law residual r = G^T M1 e_x + Lambda0(X)^T W 1 - dx 1 (second remark of
 * Section 4.2 with the background of the Poisson equation of Section 2.1);
 * *linf = max_j |r_j|; vec (length M) may be NULL. */
int ecpic_gauss_residual(ecpic_ctx *ctx, double *linf, double *vec);

/* ---- Learned warm start of Subsystem I ------------------------------------
 * The initial Picard iterate of Subsystem I (Section 4.2 leaves it open) can
 * come from a small network instead of the explicit predictor: an MLP
 * D -> 64 -> 64 -> 2, GELU (tanh form), D = 3 + 6 (degree + 1), fed the
 * particle's features
 *   [t - 1/2, p, gamma0 - 1, a_y[c-p..c+p+1], a_z[c-p..c+p+1], e_x[c-p..c+p+1]]
 * (t = x/dx - c in cell c, gamma0 = sqrt(1 + p^2 + |A_perp(x)|^2)) and trained
 * on the converged increments
 *   [(delta - dt p/gamma0)/dt^2, (p^{n+1} - p)/dt].
 * With the network enabled every Subsystem I substep starts with a predictor
 * pass: the network is evaluated per cell on an 8 x 8 grid of (t, p) nodes
 * (BF16 matrix cores, FP32 accumulation), each particle interpolates its cell's
 * table for delta^(1), and the current of delta^(1) gives a consistent e^(1);
 * the ordinary Picard sweeps follow to the same tolerance, so the network only
 * changes how many are needed.  Parameters are one flat float vector
 *   [W1 (64 x D) | b1 | W2 (64 x 64) | b2 | W3 (2 x 64) | b3 |
 *    mu (D + 2) | sd (D + 2) | p_lo, p_hi]
 * (normalisation of features and targets, momentum range of the table). */
typedef struct {
    int32_t steps;   /* Adam steps; 0 => 2000 */
    int32_t batch;   /* samples per step, a multiple of 32; 0 => 1024 */
    float lr;        /* Adam step size; 0 => 1e-3 */
    uint64_t seed;   /* initial weights and sample draws (counter-based) */
} ecpic_ws_train_config;

/* From the next step on, record one training pair per committed Subsystem I
 * substep for every particle with id % stride == (step count % stride), into a
 * device buffer of `capacity` pairs (reallocated if the capacity changes;
 * recording restarts from empty).  stride = 0 stops recording.  ENOMEM if the
 * buffer cannot be allocated. */
int ecpic_ws_record(ecpic_ctx *ctx, int32_t stride, int64_t capacity);
/* Number of pairs held (at most the capacity). */
int ecpic_ws_records(ecpic_ctx *ctx, int64_t *n);
/* Copy the first n pairs to host arrays feat (n x D) and targ (n x 2) (either may
 * be NULL); EINVAL if n exceeds the pairs held. */
int ecpic_ws_get_records(ecpic_ctx *ctx, float *feat, float *targ, int64_t n);
/* Train from scratch on the recorded pairs (FP32 forward/backward and Adam on
 * the GPU; normalisation from the pairs' mean and standard deviation).
 * *final_loss = mean squared error (normalised targets) of the last batch.
 * ESTATE without recorded pairs. */
int ecpic_ws_train(ecpic_ctx *ctx, const ecpic_ws_train_config *cfg, float *final_loss);
/* Length of the flat parameter vector. */
int ecpic_ws_n_params(ecpic_ctx *ctx, int64_t *n);
/* Copy the parameters out / in (host arrays of ecpic_ws_n_params floats). */
int ecpic_ws_get_weights(ecpic_ctx *ctx, float *w, int64_t n);
int ecpic_ws_set_weights(ecpic_ctx *ctx, const float *w, int64_t n);
/* Use (on != 0) or stop using the network for the following substeps; ESTATE
 * if it has neither been trained nor set. */
int ecpic_ws_enable(ecpic_ctx *ctx, int32_t on);
/* Gradient (length n_params minus the normalisation tail) and loss of the mean
 * squared error over n samples given already normalised: x (n x D), y (n x 2),
 * host arrays.  The computation is the training kernels'.  ESTATE without a
 * network. */
int ecpic_ws_grad(ecpic_ctx *ctx, const float *x, const float *y, int64_t n, float *grad, float *loss);
/* The per-cell tables of the increment target (physical units, [M][8 t][8 p],
 * t_i = i/7, p_j = p_lo + j (p_hi - p_lo)/7) for the current state; host array. */
int ecpic_ws_table(ecpic_ctx *ctx, float *table);

/* Per-kernel timing with HIP events on the context's stream.  enable != 0 starts
 * recording (and clears the totals); ecpic_kernel_time returns the accumulated
 * milliseconds and launch count of the named kernel family ("sweep_I",
 * "field_I", "commit_I", "sweep_II", "field_II", ...). */
int ecpic_profile_enable(ecpic_ctx *ctx, int32_t enable);
int ecpic_kernel_time(ecpic_ctx *ctx, const char *name, double *ms, int64_t *launches);

/* Bandwidth reference: times reps launches of a plain streaming copy kernel that
 * reads and writes `bytes` bytes each (buffers allocated for the call) and
 * returns the mean milliseconds per copy.  The same kernel is the calibration
 * reference for hardware fetch/write byte counters. */
int ecpic_bandwidth_probe(ecpic_ctx *ctx, int64_t bytes, int32_t reps, double *ms_per_copy);

/* Static description of the error code. */
const char *ecpic_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* ECPIC_H */
