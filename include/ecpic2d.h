/*
 * ecpic2d.h -- C-ABI of the MI355X (gfx950) library for the energy-conserving
 * particle-in-cell step of the reduced 2D relativistic Vlasov-Maxwell model
 * (Li, "Energy conserving particle-in-cell methods for relativistic
 * Vlasov-Maxwell equations of laser-plasma interaction", Sections 2.2, 3.2 and
 * 4.3), with or without the spin terms (hbar, the particles' spins s_a).
 *
 * State (Section 3.2): particle positions x_a = (x1, x2) and momenta
 * p_a = (p1, p2) with a common weight w; the fields on a periodic uniform grid of
 * M1 x M2 cells, as coefficients of tensor products of B-splines of degree p:
 *   a_z, e_z   in V0 (degree p in x1 and x2),
 *   e_xy       in V1: e1 (degree p-1 in x1, p in x2) and e2 (p in x1, p-1 in x2),
 *   b_z        in V2 (degree p-1 in both).
 * Every coefficient array has M1 M2 entries, row-major: entry i1 M2 + i2 is the
 * coefficient of the basis function N_{i1}(x1) N_{i2}(x2), N_j supported on
 * [j dx, (j + d + 1) dx).  Units are those of the reduced model (Section 2.2):
 * c = 1, plasma frequency 1 at density 1, ions a uniform neutralising
 * background.
 *
 * A Lie-Trotter step applies the four subsystems of the Section 4.3 splitting in
 * order: I (positions, momenta and e_xy by the discrete gradient, Picard
 * iteration), II (rotation of the momenta by B_z, and of the spins about B_h),
 * III (a_z and e_z, fixed point), IV (e_xy and b_z, Maxwell).
 *
 * With spin (cfg.spin = 1) the Hamiltonian carries the Zeeman term
 * hbar sum_a w s_a . B_h(x_a), B_h = (dA_z/dx2, -dA_z/dx1, B_z) (Section 2.2):
 * Subsystem I adds its force (the divided differences of s . B_h along the two
 * legs of the discrete gradient), II turns every spin about B_h(x_a) exactly,
 * and III and IV add the constant sources hbar G*^T Lambda1*(X)^T W S_xy and
 * hbar C^T Lambda2(X)^T W S_z.
 *
 * Every call returns an ecpic_status (ecpic.h).  Unless stated otherwise:
 *   - host arrays are read or written during the call only and never kept;
 *   - ECPIC_EINVAL leaves the state unchanged;
 *   - a context is bound to one device and one stream and is not thread-safe.
 * All computation runs in HIP kernels on the GPU; there is no CPU fallback, and
 * ecpic2d_create fails with ECPIC_EDEVICE when no gfx950 device is usable.
 * The deposits accumulate with floating-point atomics (LDS, then global), so two
 * runs from one state agree to rounding, not bit for bit.
 */
#ifndef ECPIC2D_H
#define ECPIC2D_H

#include <stdint.h>

#include "ecpic.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ecpic2d_ctx ecpic2d_ctx;

typedef struct {
    double L1, L2;            /* domain [0, L1) x [0, L2); grid x_{k,j} = j L_k / M_k (Section 3.2) */
    int32_t M1, M2;           /* cells per direction: powers of two in [8, 512] */
    int32_t degree;           /* V0 degree p in [2, 5] in both directions */
    int32_t picard_max_iter;  /* sweeps (I) and iterations (III) before ECPIC_ENOTCONV; 0 => 50, <= 64 */
    int64_t n_particles;      /* N >= 0 */
    double weight;            /* w_a for all particles; 0 => L1 L2 / N (mean density 1) */
    double dt;                /* time step of ecpic2d_step; 0 < dt < min(L1/M1, L2/M2) */
    double picard_tol;        /* absolute max-norm tolerance of the fixed points (> 0) */
    int32_t device;           /* HIP device ordinal */
    int32_t spin;             /* 1: the particles carry spins (ecpic2d_set_spins) and the hbar terms are
                                 on; 0: no spin */
    double hbar;              /* normalised Planck constant of the Zeeman term; must be 0 without spin.
                                 With hbar = 0 the spins still precess in Subsystem II but act on
                                 nothing. */
} ecpic2d_config;

typedef struct {
    int32_t sweeps;   /* Picard sweeps (Subsystem I) or fixed-point iterations (Subsystem III) */
    int32_t reserved;
    double residual;  /* max-norm increment of the last sweep (length and field units) */
} ecpic2d_iter_stats;

typedef struct {
    double kinetic;   /* sum_a w (gamma_a - 1), gamma = sqrt(1 + |p|^2 + A_z(x_a)^2) */
    double e_xy;      /* 1/2 e_xy^T M1 e_xy */
    double b_z;       /* 1/2 b_z^T M2 b_z */
    double e_z;       /* 1/2 e_z^T M0 e_z */
    double a_z;       /* 1/2 a_z^T K a_z, K = G^T M1 G (|grad A_z|^2 / 2) */
    double total;     /* the discrete Hamiltonian of Section 3.2 (the Zeeman term included) */
    double zeeman;    /* hbar sum_a w s_a . B_h(x_a) (0 without spin) */
} ecpic2d_energy_parts;

/* Create a context on cfg->device and allocate every device buffer for N
 * particles and M1 x M2 cells.  Errors: EINVAL for an invalid config, EDEVICE
 * when the device is missing or not gfx950, ENOMEM. */
int ecpic2d_create(const ecpic2d_config *cfg, ecpic2d_ctx **out);

/* Release every resource of ctx (NULL is allowed). */
int ecpic2d_destroy(ecpic2d_ctx *ctx);

/* Particle state: positions (any real, wrapped into the domain) and momenta, host
 * arrays of n = n_particles entries.  The library keeps the particles sorted by
 * cell and remembers each one's index, so get_particles returns them in the
 * order given to set_particles. */
int ecpic2d_set_particles(ecpic2d_ctx *ctx, const double *x1, const double *x2, const double *p1,
                          const double *p2, int64_t n);
int ecpic2d_get_particles(ecpic2d_ctx *ctx, double *x1, double *x2, double *p1, double *p2, int64_t n);

/* Spins s_a = (s_x, s_y, s_z) (Section 2.2; needs cfg.spin), host arrays of n =
 * n_particles entries in the order given to set_particles.  set_particles sets
 * every spin to zero; get_spins returns them in that order.  EINVAL without spin,
 * if n differs or a value is not finite; ESTATE before set_particles. */
int ecpic2d_set_spins(ecpic2d_ctx *ctx, const double *sx, const double *sy, const double *sz, int64_t n);
int ecpic2d_get_spins(ecpic2d_ctx *ctx, double *sx, double *sy, double *sz, int64_t n);

/* Field coefficients, host arrays of M1 M2 entries each (layout above).  A NULL
 * input sets that field to zero; a NULL output skips it. */
int ecpic2d_set_fields(ecpic2d_ctx *ctx, const double *e1, const double *e2, const double *bz,
                       const double *ez, const double *az);
int ecpic2d_get_fields(ecpic2d_ctx *ctx, double *e1, double *e2, double *bz, double *ez, double *az);

/* Correct e_xy so that the discrete Gauss law G^T M1 e_xy + Lambda0(X)^T W 1 =
 * dx1 dx2 1 holds: e_xy <- e_xy - G phi with K phi the residual (zero-mean phi).
 * A divergence-free part of the given e_xy is kept.  ESTATE before
 * set_particles. */
int ecpic2d_solve_gauss(ecpic2d_ctx *ctx);

/* Subsystem I of Section 4.3 over dt: the discrete-gradient update of
 * (x, p, e_xy) with a_z, e_z, b_z frozen, solved by Jacobi Picard sweeps in
 * (x^{n+1} - x^n, e_xy^{n+1}) to picard_tol.  0 < dt < min(dx1, dx2).  stats
 * may be NULL.  ENOTCONV and ENONFINITE leave the state as before the call. */
int ecpic2d_substep_I(ecpic2d_ctx *ctx, double dt, ecpic2d_iter_stats *stats);

/* Subsystem II: every momentum turned by the angle B_z(x_a) dt / gamma_a, and
 * with spin every spin turned about B_h(x_a) by the angle -|B_h(x_a)| dt
 * (ds/dt = s x B_h, Rodrigues' formula): the exact solution of the subsystem. */
int ecpic2d_substep_II(ecpic2d_ctx *ctx, double dt);

/* Subsystem III: (a_z, e_z) by the implicit midpoint scheme, fixed point on e_z
 * with the linear part (M0 + dt^2 K / 4) solved exactly; with spin the right-hand
 * side carries hbar dt G*^T Lambda1*(X)^T W S_xy.  ENOTCONV and ENONFINITE leave
 * the state as before the call. */
int ecpic2d_substep_III(ecpic2d_ctx *ctx, double dt, ecpic2d_iter_stats *stats);

/* Subsystem IV: (e_xy, b_z) by the implicit midpoint scheme, solved exactly; with
 * spin the b_z term of the e_xy equation carries hbar Lambda2(X)^T W S_z. */
int ecpic2d_substep_IV(ecpic2d_ctx *ctx, double dt);

/* nsteps Lie-Trotter steps I, II, III, IV with the configured dt.
 * sweeps_I / iters_III (nullable, nsteps entries) receive the per-step counts.
 * On an error the steps before the failing one stay applied. */
int ecpic2d_step(ecpic2d_ctx *ctx, int32_t nsteps, int32_t *sweeps_I, int32_t *iters_III);

/* Discrete Hamiltonian and its parts for the current state. */
int ecpic2d_energy(ecpic2d_ctx *ctx, ecpic2d_energy_parts *out);

/* Max-norm of the discrete Gauss-law residual r = G^T M1 e_xy + Lambda0(X)^T W 1
 * - dx1 dx2 1; vec (nullable, host, M1 M2) receives r. */
int ecpic2d_gauss_residual(ecpic2d_ctx *ctx, double *linf, double *vec);

/* Charge deposit rho = Lambda0(X)^T W 1 (host array of M1 M2 entries). */
int ecpic2d_deposit_charge(ecpic2d_ctx *ctx, double *rho);

/* Kernel timing with HIP events on the context's stream: while enabled, every
 * launch is bracketed and its time accumulated per kernel family ("sweep_I",
 * "commit_I", "sort", "solve_I", "rotate_II", "deposit_III", "solve_III",
 * "maxwell_IV", ...).  enable = 1 also clears the totals. */
int ecpic2d_profile_enable(ecpic2d_ctx *ctx, int32_t enable);
int ecpic2d_kernel_time(ecpic2d_ctx *ctx, const char *name, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* ECPIC2D_H */
