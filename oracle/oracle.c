/*
 * Plain FP64 CPU oracle for the energy-conserving PIC step of the reduced 1D
 * relativistic Vlasov-Maxwell model (Li, "Energy conserving particle-in-cell
 * methods for relativistic Vlasov-Maxwell equations of laser-plasma
 * interaction"), spin term off.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * code, header, table or helper with the HIP library; it is deliberately slow
 * and literal so that it can be checked against the paper by eye:
 *   - B-splines by the Cox-de Boor recursion on integer knots,
 *   - every integral (mass matrices, line integrals) by Gauss-Legendre
 *     quadrature that is exact for the polynomial degree involved,
 *   - stiffness applied as G^T M1 G by three sparse products,
 *   - linear solves by conjugate gradients plus iterative refinement,
 *   - particles kept in input order, absolute positions x in [0, L).
 *
 * Every function names the passage of the paper it follows.  Conventions
 * (Section 3.1): x_j = j dx, dx = L/M, Lambda0_j = N^p_j (support
 * [x_j, x_{j+p+1})), Lambda1_j = N^{p-1}_j, indices periodic mod M,
 * (G c)_i = (c_i - c_{i-1}) / dx so that d/dx Lambda0_j = (Lambda1_j -
 * Lambda1_{j+1}) / dx.
 *
 * Readings of the paper taken here (also listed in the design notes):
 *   - the divided difference (A(x1)-A(x0))/(x1-x0) of Subsystem I is
 *     evaluated through the exact identity sum_j (G a)_j lbar_j(x0,x1),
 *     where lbar is the line mean of Lambda1 along the step; this removes the
 *     0/0 that the paper's first remark approximates away;
 *   - the particle term of Subsystem II uses Lambda0 (A_perp lives in V0);
 *   - the discrete Gauss law carries the neutralising background:
 *     r = G^T M1 e_x + Lambda0(X)^T W 1 - dx 1;
 *   - the Picard map of Subsystem I is a Jacobi sweep in (delta, e_x) started
 *     from delta = dt p / gamma(x^n, p^n) and e = e_x^n, stopped on the max
 *     norm of both increments, committing x^n + delta^(k), p^(k+1) and
 *     e^(k+1), the triple whose deposit and position agree exactly;
 *   - optionally (seidel = 1) each sweep deposits the current of the increment
 *     it has just produced, delta^(k+1), instead of delta^(k); the fixed point is
 *     the same, the contraction per sweep is the square of Jacobi's, and the
 *     commit is x^n + delta^(k+1), e^(k+1) and the momentum re-evaluated from
 *     (delta^(k+1), e^(k+1));
 *   - optionally (warm_previous = 1) the iteration of a Subsystem I substep
 *     starts from the increments the previous substep of the run committed
 *     (explicit start on the first); the fixed point does not change;
 *   - the adjoint of the Subsystem I scheme (Section 4.1: the discrete gradient
 *     with the two coordinates varied in the opposite order, p first at x^n,
 *     then x at p^{n+1}) is iterated on the new momentum P: each sweep forms the
 *     increment of P, the new momentum, and the increment of the new momentum,
 *     deposits the current of that last increment and commits it together with
 *     the new momentum and e^(k+1);
 *   - optionally (splitting = 1) a step is the symmetric composition
 *     Subsystem I over dt/2, Subsystem II over dt, adjoint Subsystem I over dt/2
 *     (second order in dt); splitting = 0 is the Lie-Trotter step of Section 5.
 * With spin (the *_s functions; hbar = the normalised Planck constant):
 *   - the Zeeman energy of eq. discrete_H, hbar sum_a w (s_y dA_z/dx - s_z dA_y/dx)
 *     at x_a, enters Subsystem I through the divided difference of dA/dx along
 *     the step, evaluated as sum_j (G G a)_j times the line mean of the degree
 *     p-2 splines Lambda2_j (d/dx Lambda1_j = (Lambda2_j - Lambda2_{j+1}) / dx),
 *     the same 0/0-free identity one degree down; the sign is the one the
 *     gradient of that energy gives (the printed discrete gradient drops a sign
 *     and a weight), and it matches the printed momentum update;
 *   - Subsystem II gains the constant source -/+ hbar G^T Lambda1(X)^T W S_{z/y},
 *     multiplied by dt in the combined (M0 + dt^2 K/4) system (the M0^{-1}
 *     printed there is a slip: the e_y scheme multiplied by M0 has none);
 *   - Subsystem III rotates every spin exactly about r = (0, Z, -Y),
 *     Y = dA_y/dx(x_a), Z = dA_z/dx(x_a), by Rodrigues' formula;
 *   - a Lie-Trotter step with spin is I, II, III; the symmetric one
 *     I(dt/2), III(dt/2), II(dt), III(dt/2), adjoint I(dt/2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double L;
    int32_t M;
    int32_t p;                  /* degree of V0; V1 has degree p - 1 */
    int64_t n;                  /* particle count */
    double w;                   /* particle weight omega_a (all equal) */
    double dt;
    double tol;                 /* absolute max-norm Picard tolerance */
    int32_t kmax;               /* Picard iteration cap */
    int32_t commit_unconverged; /* test hook: commit after kmax sweeps anyway */
    int32_t seidel;             /* 0: Jacobi map, 1: current from the fresh increment */
    int32_t splitting;          /* 0: Lie-Trotter (I then II), 1: I(dt/2), II(dt), adjoint I(dt/2) */
    int32_t warm_previous;      /* 1: Subsystem I starts from the last committed increments */
    double hbar;                /* spin coupling (the *_s functions) */
} orc_cfg;

enum { ORC_OK = 0, ORC_ENOTCONV = -3, ORC_ENOMEM = -2 };

/* ------------------------------------------------------------------ */
/* Quadrature: 6-point Gauss-Legendre on [-1, 1], exact to degree 11.   */
/* ------------------------------------------------------------------ */
static const double GL_X[6] = {-0.9324695142031521, -0.6612093864662645, -0.2386191860831969,
                               0.2386191860831969,  0.6612093864662645,  0.9324695142031521};
static const double GL_W[6] = {0.1713244923791704, 0.3607615730481386, 0.4679139345726910,
                               0.4679139345726910, 0.3607615730481386, 0.1713244923791704};

static double dx_of(const orc_cfg *c) { return c->L / (double)c->M; }
static long imod(long j, long M) { long r = j % M; return r < 0 ? r + M : r; }

/* ------------------------------------------------------------------ */
/* Section 3.1: B-spline bases.                                         */
/* ------------------------------------------------------------------ */

/* Cardinal B-spline of degree d on the integer knots 0..d+1 (Cox-de Boor). */
double orc_bspline(int d, double u)
{
    if (d == 0) return (u >= 0.0 && u < 1.0) ? 1.0 : 0.0;
    return (u * orc_bspline(d - 1, u) + ((double)d + 1.0 - u) * orc_bspline(d - 1, u - 1.0)) /
           (double)d;
}

/* Lambda0_j(x) = B_p((x - x_j)/dx) and Lambda1_j(x) = B_{p-1}((x - x_j)/dx); j is an
 * unwrapped index and x an unwrapped position, so no periodic image is taken here. */
double orc_lambda0(const orc_cfg *c, long j, double x) { return orc_bspline(c->p, x / dx_of(c) - (double)j); }
double orc_lambda1(const orc_cfg *c, long j, double x) { return orc_bspline(c->p - 1, x / dx_of(c) - (double)j); }

static long cell_of(const orc_cfg *c, double x) { return (long)floor(x / dx_of(c)); }

/* Field of the V0 expansion (eq. fem_a): sum_j c_j Lambda0_j(x), over the p+1
 * splines that do not vanish on x's cell; x may lie slightly outside [0, L). */
double orc_field0(const orc_cfg *c, const double *coef, double x)
{
    long i = cell_of(c, x);
    double s = 0.0;
    for (long j = i - c->p; j <= i; ++j) s += coef[imod(j, c->M)] * orc_lambda0(c, j, x);
    return s;
}

/* Field of the V1 expansion (eq. fem_e): sum_j c_j Lambda1_j(x). */
double orc_field1(const orc_cfg *c, const double *coef, double x)
{
    long i = cell_of(c, x);
    double s = 0.0;
    for (long j = i - c->p + 1; j <= i; ++j) s += coef[imod(j, c->M)] * orc_lambda1(c, j, x);
    return s;
}

/* ------------------------------------------------------------------ */
/* Section 3.1: mass matrices M0, M1, derivative matrix G, K=G^T M1 G.  */
/* ------------------------------------------------------------------ */

/* Row of the mass matrix of degree-d splines with dx = 1: row[k + d] =
 * int B_d(u) B_d(u - k) du for k = -d..d, integrated cell by cell. */
void orc_mass_row(int d, double *row)
{
    for (int k = -d; k <= d; ++k) {
        double s = 0.0;
        for (int cell = 0; cell <= d; ++cell) {
            for (int q = 0; q < 6; ++q) {
                double u = cell + 0.5 + 0.5 * GL_X[q];
                s += 0.5 * GL_W[q] * orc_bspline(d, u) * orc_bspline(d, u - k);
            }
        }
        row[k + d] = s;
    }
}

/* y = M x for the circulant with the given row (half band b), scaled by dx. */
static void circ_apply(int M, int b, const double *row, double scale, const double *x, double *y)
{
    for (int i = 0; i < M; ++i) {
        double s = 0.0;
        for (int k = -b; k <= b; ++k) s += row[k + b] * x[imod(i + k, M)];
        y[i] = scale * s;
    }
}

void orc_apply_M0(const orc_cfg *c, const double *x, double *y)
{
    double row[32];
    orc_mass_row(c->p, row);
    circ_apply(c->M, c->p, row, dx_of(c), x, y);
}

void orc_apply_M1(const orc_cfg *c, const double *x, double *y)
{
    double row[32];
    orc_mass_row(c->p - 1, row);
    circ_apply(c->M, c->p - 1, row, dx_of(c), x, y);
}

/* (G c)_i = (c_i - c_{i-1}) / dx (Section 3.1, derivative relation). */
void orc_apply_G(const orc_cfg *c, const double *x, double *y)
{
    double dx = dx_of(c);
    for (int i = 0; i < c->M; ++i) y[i] = (x[i] - x[imod(i - 1, c->M)]) / dx;
}

/* (G^T u)_j = (u_j - u_{j+1}) / dx. */
void orc_apply_GT(const orc_cfg *c, const double *x, double *y)
{
    double dx = dx_of(c);
    for (int j = 0; j < c->M; ++j) y[j] = (x[j] - x[imod(j + 1, c->M)]) / dx;
}

/* K x = G^T M1 G x (stiffness, eq. discrete_H). */
void orc_apply_K(const orc_cfg *c, const double *x, double *y)
{
    double *t1 = malloc(sizeof(double) * c->M), *t2 = malloc(sizeof(double) * c->M);
    orc_apply_G(c, x, t1);
    orc_apply_M1(c, t1, t2);
    orc_apply_GT(c, t2, y);
    free(t1); free(t2);
}

/* (M0 + dt^2/4 K) x and (M0 - dt^2/4 K) x (Subsystem II linear system). */
static void apply_cn(const orc_cfg *c, const double *x, double *y, double sign)
{
    double *t = malloc(sizeof(double) * c->M);
    orc_apply_M0(c, x, y);
    orc_apply_K(c, x, t);
    for (int i = 0; i < c->M; ++i) y[i] += sign * 0.25 * c->dt * c->dt * t[i];
    free(t);
}
void orc_apply_cn_plus(const orc_cfg *c, const double *x, double *y) { apply_cn(c, x, y, +1.0); }
void orc_apply_cn_minus(const orc_cfg *c, const double *x, double *y) { apply_cn(c, x, y, -1.0); }

/* ------------------------------------------------------------------ */
/* Linear solves: conjugate gradients with two refinement passes.       */
/* ------------------------------------------------------------------ */
typedef void (*orc_op)(const orc_cfg *, const double *, double *);

static double dotv(int M, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < M; ++i) s += a[i] * b[i];
    return s;
}

static void cg_core(const orc_cfg *c, orc_op A, const double *b, double *x)
{
    int M = c->M;
    double *r = malloc(sizeof(double) * M), *d = malloc(sizeof(double) * M),
           *Ad = malloc(sizeof(double) * M), *best = malloc(sizeof(double) * M);
    memset(x, 0, sizeof(double) * M);
    memcpy(r, b, sizeof(double) * M);
    memcpy(d, b, sizeof(double) * M);
    memset(best, 0, sizeof(double) * M);
    double rr = dotv(M, r, r), bb = rr, best_rr = rr;
    int stall = 0;
    if (bb > 0.0) {
        for (int it = 0; it < 20 * M + 200; ++it) {
            A(c, d, Ad);
            double alpha = rr / dotv(M, d, Ad);
            for (int i = 0; i < M; ++i) { x[i] += alpha * d[i]; r[i] -= alpha * Ad[i]; }
            double rn = dotv(M, r, r);
            if (rn < best_rr) { best_rr = rn; stall = 0; memcpy(best, x, sizeof(double) * M); }
            else ++stall;
            if (rn <= 1e-36 * bb || stall >= 8) break;
            double beta = rn / rr;
            for (int i = 0; i < M; ++i) d[i] = r[i] + beta * d[i];
            rr = rn;
        }
        memcpy(x, best, sizeof(double) * M);
    }
    free(r); free(d); free(Ad); free(best);
}

static void solve(const orc_cfg *c, orc_op A, const double *b, double *x)
{
    int M = c->M;
    double *r = malloc(sizeof(double) * M), *dx = malloc(sizeof(double) * M);
    cg_core(c, A, b, x);
    for (int pass = 0; pass < 2; ++pass) {
        A(c, x, r);
        for (int i = 0; i < M; ++i) r[i] = b[i] - r[i];
        cg_core(c, A, r, dx);
        for (int i = 0; i < M; ++i) x[i] += dx[i];
    }
    free(r); free(dx);
}

void orc_solve_M1(const orc_cfg *c, const double *b, double *x) { solve(c, orc_apply_M1, b, x); }
void orc_solve_M0(const orc_cfg *c, const double *b, double *x) { solve(c, orc_apply_M0, b, x); }
void orc_solve_cn(const orc_cfg *c, const double *b, double *x) { solve(c, orc_apply_cn_plus, b, x); }

/* ------------------------------------------------------------------ */
/* Line integrals along the straight trajectory (Subsystem I scheme).    */
/* ------------------------------------------------------------------ */

/* Mean of the degree-d splines B_d((x - x_j)/dx) over the segment between x0 and
 * x1 (unwrapped positions): (1/(x1-x0)) int_{x0}^{x1} B_d((x - x_j)/dx) dx.  The
 * segment is cut at the knots and each piece integrated by Gauss-Legendre
 * (exact for degree d <= 11); piece means are combined with weights len/total,
 * so no 0/0 arises; for x1 == x0 the mean is the value at x0.  Returns the
 * number of entries written to vals for the unwrapped indices *jlo, *jlo+1, ... */
static int line_mean_deg(const orc_cfg *c, int d, double x0, double x1, long *jlo, double *vals)
{
    double dx = dx_of(c);
    double lo = x0 < x1 ? x0 : x1, hi = x0 < x1 ? x1 : x0;
    long ilo = cell_of(c, lo), ihi = cell_of(c, hi);
    long j0 = ilo - d;
    int nj = (int)(ihi - ilo) + d + 1;
    *jlo = j0;
    for (int k = 0; k < nj; ++k) vals[k] = 0.0;
    if (hi == lo) {
        for (long j = j0; j <= ihi; ++j) vals[j - j0] = orc_bspline(d, lo / dx - (double)j);
        return nj;
    }
    double total = hi - lo;
    for (long cell = ilo; cell <= ihi; ++cell) {
        double s = lo > cell * dx ? lo : cell * dx;
        double e = hi < (cell + 1) * dx ? hi : (cell + 1) * dx;
        if (!(e > s)) continue;
        double frac = (e - s) / total;
        for (int q = 0; q < 6; ++q) {
            double xq = 0.5 * (s + e) + 0.5 * (e - s) * GL_X[q];
            for (long j = cell - d; j <= cell; ++j)
                vals[j - j0] += frac * 0.5 * GL_W[q] * orc_bspline(d, xq / dx - (double)j);
        }
    }
    return nj;
}

/* Mean of Lambda1_j over the segment (the time average of the basis along the
 * straight trajectory of the Subsystem I scheme): lbar_j = (1/dt) int
 * Lambda1_j(x(tau)) dtau = (1/(x1-x0)) int_{x0}^{x1} Lambda1_j. */
int orc_line_mean(const orc_cfg *c, double x0, double x1, long *jlo, double *vals)
{
    return line_mean_deg(c, c->p - 1, x0, x1, jlo, vals);
}

/* Mean of Lambda2_j = B_{p-2}((x - x_j)/dx) over the segment: the divided
 * difference of a V1 field phi = sum c_j Lambda1_j along the step is
 * sum_j (G c)_j times these means (spin force of Subsystem I). */
int orc_line_mean2(const orc_cfg *c, double x0, double x1, long *jlo, double *vals)
{
    return line_mean_deg(c, c->p - 2, x0, x1, jlo, vals);
}

/* Current deposit J_j = sum_a w int_{x0_a}^{x1_a} Lambda1_j (length units), the
 * quantity that drives e_x in Subsystem I. */
void orc_deposit_current(const orc_cfg *c, const double *x0, const double *x1, int64_t n, double *J)
{
    long jlo;
    double vals[16];
    memset(J, 0, sizeof(double) * c->M);
    for (int64_t a = 0; a < n; ++a) {
        int nj = orc_line_mean(c, x0[a], x1[a], &jlo, vals);
        for (int k = 0; k < nj; ++k) J[imod(jlo + k, c->M)] += c->w * (x1[a] - x0[a]) * vals[k];
    }
}

/* Charge deposit rho = Lambda0(X)^T W 1 (Remark 2). */
void orc_deposit_charge(const orc_cfg *c, const double *x, double *rho)
{
    memset(rho, 0, sizeof(double) * c->M);
    for (int64_t a = 0; a < c->n; ++a) {
        long i = cell_of(c, x[a]);
        for (long j = i - c->p; j <= i; ++j) rho[imod(j, c->M)] += c->w * orc_lambda0(c, j, x[a]);
    }
}

/* ------------------------------------------------------------------ */
/* Diagnostics: discrete Hamiltonian (eq. discrete_H) and Gauss law.    */
/* ------------------------------------------------------------------ */

/* parts = {kinetic, 1/2 ex^T M1 ex, 1/2 sum e_c^T M0 e_c, 1/2 sum a_c^T K a_c, H}.
 * gamma - 1 is written (p^2 + |A|^2)/(gamma + 1), the same number without the
 * cancellation of gamma - 1 near gamma = 1. */
void orc_energy(const orc_cfg *c, const double *x, const double *p, const double *ex,
                const double *ey, const double *ez, const double *ay, const double *az,
                double *parts)
{
    int M = c->M;
    double *t = malloc(sizeof(double) * M);
    double kin = 0.0;
    for (int64_t a = 0; a < c->n; ++a) {
        double Ay = orc_field0(c, ay, x[a]), Az = orc_field0(c, az, x[a]);
        double q = p[a] * p[a] + Ay * Ay + Az * Az;
        double g = sqrt(1.0 + q);
        kin += c->w * q / (g + 1.0);
    }
    orc_apply_M1(c, ex, t);
    double el = 0.5 * dotv(M, ex, t);
    orc_apply_M0(c, ey, t);
    double et = 0.5 * dotv(M, ey, t);
    orc_apply_M0(c, ez, t);
    et += 0.5 * dotv(M, ez, t);
    orc_apply_K(c, ay, t);
    double bt = 0.5 * dotv(M, ay, t);
    orc_apply_K(c, az, t);
    bt += 0.5 * dotv(M, az, t);
    parts[0] = kin; parts[1] = el; parts[2] = et; parts[3] = bt; parts[4] = kin + el + et + bt;
    free(t);
}

/* r = G^T M1 e_x + Lambda0(X)^T W 1 - dx 1; returns max |r_j|, writes r if non-null. */
double orc_gauss_residual(const orc_cfg *c, const double *x, const double *ex, double *r_out)
{
    int M = c->M;
    double *t = malloc(sizeof(double) * M), *r = malloc(sizeof(double) * M), *rho = malloc(sizeof(double) * M);
    orc_apply_M1(c, ex, t);
    orc_apply_GT(c, t, r);
    orc_deposit_charge(c, x, rho);
    double m = 0.0, dx = dx_of(c);
    for (int j = 0; j < M; ++j) {
        r[j] += rho[j] - dx;
        if (fabs(r[j]) > m) m = fabs(r[j]);
    }
    if (r_out) memcpy(r_out, r, sizeof(double) * M);
    free(t); free(r); free(rho);
    return m;
}

/* Initial e_x from the discrete Poisson equation G^T M1 e_x = dx 1 - rho in the
 * zero-mean gauge: u = M1 e_x solves G^T u = rhs, i.e. u_{j+1} = u_j - dx rhs_j
 * (a running sum), shifted to zero mean, then e_x = M1^{-1} u.  If the weights
 * do not neutralise the background exactly, rhs is taken minus its mean. */
void orc_solve_gauss(const orc_cfg *c, const double *x, double *ex)
{
    int M = c->M;
    double dx = dx_of(c);
    double *rho = malloc(sizeof(double) * M), *u = malloc(sizeof(double) * M);
    orc_deposit_charge(c, x, rho);
    double mean = 0.0;
    for (int j = 0; j < M; ++j) { rho[j] = dx - rho[j]; mean += rho[j]; }
    mean /= M;
    for (int j = 0; j < M; ++j) rho[j] -= mean;
    u[0] = 0.0;
    for (int j = 0; j + 1 < M; ++j) u[j + 1] = u[j] - dx * rho[j];
    double um = 0.0;
    for (int j = 0; j < M; ++j) um += u[j];
    um /= M;
    for (int j = 0; j < M; ++j) u[j] -= um;
    orc_solve_M1(c, u, ex);
    free(rho); free(u);
}

/* ------------------------------------------------------------------ */
/* Subsystem I (Section 4.2): implicit update of (x, p, e_x).            */
/* ------------------------------------------------------------------ */

static double wrap(const orc_cfg *c, double x)
{
    if (x < 0.0) x += c->L;
    else if (x >= c->L) x -= c->L;
    if (x >= c->L) x = 0.0;
    return x;
}

/* Spin force of the Subsystem I scheme on one particle stepping from x0 to x1:
 * hbar [s_z (dA_y/dx(x1) - dA_y/dx(x0)) - s_y (dA_z/dx(x1) - dA_z/dx(x0))] / (x1 - x0),
 * the divided differences taken as sum_j (G G a)_j mean_j(Lambda2) (hy = G G a_y,
 * hz = G G a_z). */
static double spin_force(const orc_cfg *c, double x0, double x1, double sy, double sz, const double *hy,
                         const double *hz)
{
    long jlo;
    double m2[16];
    int nj = orc_line_mean2(c, x0, x1, &jlo, m2);
    double DDy = 0.0, DDz = 0.0;
    for (int k = 0; k < nj; ++k) {
        long j = imod(jlo + k, c->M);
        DDy += m2[k] * hy[j];
        DDz += m2[k] * hz[j];
    }
    return c->hbar * (sz * DDy - sy * DDz);
}

/* One particle of one Picard sweep.  Inputs: start x0, p0, iterate delta, field
 * coefficients a_y, a_z, gy = G a_y, gz = G a_z and ebar = (e^n + e^(k))/2; with
 * spin also the particle's s_y, s_z and hy = G G a_y, hz = G G a_z (NULL: no
 * spin term).  Outputs: p1 (the momentum update), the next delta and the
 * line-mean vector (for the current).  The discrete gradients are those of the
 * Subsystem I scheme:
 *   p1 = p0 + dt [ lbar.ebar - (A0 + A1).DA / (g(p0,A0) + g(p0,A1)) + spin force ],
 *   delta' = dt (p0 + p1) / (g(p0,A1) + g(p1,A1)),
 * with DA = (A1 - A0)/(x1 - x0) = sum_j (G a)_j lbar_j. */
static void particle_map_s(const orc_cfg *c, double x0, double p0, double delta, double sy, double sz,
                           const double *ay, const double *az, const double *gy, const double *gz,
                           const double *hy, const double *hz, const double *ebar, double *p1_out,
                           double *delta_out, long *jlo, int *nj, double *lbar)
{
    double x1 = x0 + delta;
    double A0y = orc_field0(c, ay, x0), A0z = orc_field0(c, az, x0);
    double A1y = orc_field0(c, ay, x1), A1z = orc_field0(c, az, x1);
    double g00 = sqrt(1.0 + p0 * p0 + A0y * A0y + A0z * A0z);
    double g01 = sqrt(1.0 + p0 * p0 + A1y * A1y + A1z * A1z);
    *nj = orc_line_mean(c, x0, x1, jlo, lbar);
    double LE = 0.0, LGy = 0.0, LGz = 0.0;
    for (int k = 0; k < *nj; ++k) {
        long j = imod(*jlo + k, c->M);
        LE += lbar[k] * ebar[j];
        LGy += lbar[k] * gy[j];
        LGz += lbar[k] * gz[j];
    }
    double F = LE - ((A0y + A1y) * LGy + (A0z + A1z) * LGz) / (g00 + g01);
    if (hy) F += spin_force(c, x0, x1, sy, sz, hy, hz);
    double p1 = p0 + c->dt * F;
    double g11 = sqrt(1.0 + p1 * p1 + A1y * A1y + A1z * A1z);
    *p1_out = p1;
    *delta_out = c->dt * (p0 + p1) / (g01 + g11);
}

void orc_particle_map(const orc_cfg *c, double x0, double p0, double delta,
                      const double *ay, const double *az, const double *gy, const double *gz,
                      const double *ebar, double *p1_out, double *delta_out,
                      long *jlo, int *nj, double *lbar)
{
    particle_map_s(c, x0, p0, delta, 0.0, 0.0, ay, az, gy, gz, NULL, NULL, ebar, p1_out, delta_out, jlo, nj,
                   lbar);
}

/* The same with the spin term (hy = G G a_y, hz = G G a_z). */
void orc_particle_map_spin(const orc_cfg *c, double x0, double p0, double delta, double sy, double sz,
                           const double *ay, const double *az, const double *gy, const double *gz,
                           const double *hy, const double *hz, const double *ebar, double *p1_out,
                           double *delta_out)
{
    long jlo;
    int nj;
    double lbar[16];
    particle_map_s(c, x0, p0, delta, sy, sz, ay, az, gy, gz, hy, hz, ebar, p1_out, delta_out, &jlo, &nj, lbar);
}

/* Solve Subsystem I over the time step h by Picard iteration; on success x, p, ex
 * hold the new state.  dstart (nullable): initial increments instead of the
 * explicit h p / gamma; dcommit (nullable): receives the committed increments. */
int orc_substep_I_hs(const orc_cfg *cfg, double h, double *x, double *p, double *ex, const double *ay,
                     const double *az, const double *sy, const double *sz, const double *dstart,
                     double *dcommit, int32_t *sweeps, double *res)
{
    orc_cfg ch = *cfg;
    ch.dt = h;
    const orc_cfg *c = &ch;
    int M = c->M;
    int64_t n = c->n;
    double *d = malloc(sizeof(double) * n), *dn = malloc(sizeof(double) * n),
           *p1 = malloc(sizeof(double) * n);
    double *ek = malloc(sizeof(double) * M), *enew = malloc(sizeof(double) * M),
           *ebar = malloc(sizeof(double) * M), *J = malloc(sizeof(double) * M),
           *MJ = malloc(sizeof(double) * M), *gy = malloc(sizeof(double) * M),
           *gz = malloc(sizeof(double) * M);
    if (!d || !dn || !p1 || !ek || !enew || !ebar || !J || !MJ || !gy || !gz) return ORC_ENOMEM;
    orc_apply_G(c, ay, gy);
    orc_apply_G(c, az, gz);
    /* spin: second differences G G a for the divided differences of dA/dx */
    const int spin = sy != NULL;
    double *hy = spin ? malloc(sizeof(double) * M) : NULL, *hz = spin ? malloc(sizeof(double) * M) : NULL;
    if (spin) {
        orc_apply_G(c, gy, hy);
        orc_apply_G(c, gz, hz);
    }
    for (int64_t a = 0; a < n; ++a) {
        double Ay = orc_field0(c, ay, x[a]), Az = orc_field0(c, az, x[a]);
        d[a] = dstart ? dstart[a] : c->dt * p[a] / sqrt(1.0 + p[a] * p[a] + Ay * Ay + Az * Az);
    }
    memcpy(ek, ex, sizeof(double) * M);
    int status = ORC_ENOTCONV;
    double r = 0.0;
    int k;
    for (k = 0; k < c->kmax; ++k) {
        for (int j = 0; j < M; ++j) ebar[j] = 0.5 * (ex[j] + ek[j]);
        memset(J, 0, sizeof(double) * M);
        double rx = 0.0;
        for (int64_t a = 0; a < n; ++a) {
            long jlo;
            int nj;
            double lbar[16];
            particle_map_s(c, x[a], p[a], d[a], spin ? sy[a] : 0.0, spin ? sz[a] : 0.0, ay, az, gy, gz, hy, hz,
                           ebar, &p1[a], &dn[a], &jlo, &nj, lbar);
            double step = c->seidel ? dn[a] : d[a];
            if (c->seidel) nj = orc_line_mean(c, x[a], x[a] + step, &jlo, lbar);
            double inc = (x[a] + step) - x[a];
            for (int q = 0; q < nj; ++q) J[imod(jlo + q, M)] += c->w * inc * lbar[q];
            double dd = fabs(dn[a] - d[a]);
            if (dd > rx) rx = dd;
        }
        /* e^(k+1) = e^n - dt M1^{-1} (J/dt) */
        orc_solve_M1(c, J, MJ);
        double re = 0.0;
        for (int j = 0; j < M; ++j) {
            enew[j] = ex[j] - MJ[j];
            double de = fabs(enew[j] - ek[j]);
            if (de > re) re = de;
        }
        r = rx > re ? rx : re;
        int last = (k == c->kmax - 1);
        if (r <= c->tol || (last && c->commit_unconverged)) {
            if (c->seidel) {
                for (int j = 0; j < M; ++j) ebar[j] = 0.5 * (ex[j] + enew[j]);
                for (int64_t a = 0; a < n; ++a) {
                    long jlo;
                    int nj;
                    double lbar[16], pc, dc;
                    particle_map_s(c, x[a], p[a], dn[a], spin ? sy[a] : 0.0, spin ? sz[a] : 0.0, ay, az, gy, gz,
                                   hy, hz, ebar, &pc, &dc, &jlo, &nj, lbar);
                    if (dcommit) dcommit[a] = dn[a];
                    x[a] = wrap(c, x[a] + dn[a]);
                    p[a] = pc;
                }
            } else {
                for (int64_t a = 0; a < n; ++a) {
                    if (dcommit) dcommit[a] = d[a];
                    x[a] = wrap(c, x[a] + d[a]);
                    p[a] = p1[a];
                }
            }
            memcpy(ex, enew, sizeof(double) * M);
            status = (r <= c->tol) ? ORC_OK : ORC_ENOTCONV;
            ++k;
            break;
        }
        double *t = d; d = dn; dn = t;
        memcpy(ek, enew, sizeof(double) * M);
    }
    if (sweeps) *sweeps = k;
    if (res) *res = r;
    free(d); free(dn); free(p1); free(ek); free(enew); free(ebar); free(J); free(MJ); free(gy); free(gz);
    free(hy); free(hz);
    return status;
}

/* Subsystem I over the time step h without spin. */
int orc_substep_I_h(const orc_cfg *cfg, double h, double *x, double *p, double *ex, const double *ay,
                    const double *az, const double *dstart, double *dcommit, int32_t *sweeps, double *res)
{
    return orc_substep_I_hs(cfg, h, x, p, ex, ay, az, NULL, NULL, dstart, dcommit, sweeps, res);
}

/* Subsystem I over the configured step, explicit start. */
int orc_substep_I(const orc_cfg *c, double *x, double *p, double *ex, const double *ay,
                  const double *az, int32_t *sweeps, double *res)
{
    return orc_substep_I_h(c, c->dt, x, p, ex, ay, az, NULL, NULL, sweeps, res);
}

/* ------------------------------------------------------------------ */
/* The adjoint of the Subsystem I scheme (Section 4.1 discrete gradient  */
/* with the coordinates taken in the other order).                       */
/* ------------------------------------------------------------------ */

/* The Subsystem I scheme varies x first (at p^n) and then p (at x^{n+1}).  Its
 * adjoint varies p first, at x^n, then x, at p^{n+1}:
 *   grad_p H = (gamma(x^n, p^{n+1}) - gamma(x^n, p^n)) / (p^{n+1} - p^n)
 *            = (p^n + p^{n+1}) / (gamma(x^n, p^n) + gamma(x^n, p^{n+1})),
 *   grad_x H = (gamma(x^{n+1}, p^{n+1}) - gamma(x^n, p^{n+1})) / (x^{n+1} - x^n)
 *            = (A(x^{n+1}) + A(x^n)).(A(x^{n+1}) - A(x^n)) / (x^{n+1} - x^n)
 *              / (gamma(x^n, p^{n+1}) + gamma(x^{n+1}, p^{n+1})),
 * and the step is delta / h = grad_p H, (p^{n+1} - p^n) / h = lbar.ebar - grad_x H,
 * with the same line means and field equation as the scheme.  Both gradients
 * still satisfy the discrete-gradient identity, so energy is conserved exactly
 * at the fixed point.  Given the iterate P of p^{n+1}, the increment follows
 * explicitly from the first equation; this evaluates the map once:
 *   delta = h (p0 + P) / (g(x0, p0) + g(x0, P)),  x1 = x0 + delta,
 *   P'    = p0 + h [lbar(x0, x1).ebar - (A0 + A1).DA / (g(x0, P) + g(x1, P))],
 *   delta' = h (p0 + P') / (g(x0, p0) + g(x0, P')),
 * where DA = (A1 - A0)/(x1 - x0) = sum_j (G a)_j lbar_j. */
static void adjoint_map_s(const orc_cfg *c, double x0, double p0, double P, double sy, double sz,
                          const double *ay, const double *az, const double *gy, const double *gz,
                          const double *hy, const double *hz, const double *ebar, double *delta_out,
                          double *P_out, double *delta_next)
{
    double A0y = orc_field0(c, ay, x0), A0z = orc_field0(c, az, x0);
    double qa0 = A0y * A0y + A0z * A0z;
    double g00 = sqrt(1.0 + p0 * p0 + qa0);
    double g10 = sqrt(1.0 + P * P + qa0);
    double delta = c->dt * (p0 + P) / (g00 + g10);
    double x1 = x0 + delta;
    double A1y = orc_field0(c, ay, x1), A1z = orc_field0(c, az, x1);
    double g11 = sqrt(1.0 + P * P + A1y * A1y + A1z * A1z);
    long jlo;
    double lbar[16];
    int nj = orc_line_mean(c, x0, x1, &jlo, lbar);
    double LE = 0.0, LGy = 0.0, LGz = 0.0;
    for (int k = 0; k < nj; ++k) {
        long j = imod(jlo + k, c->M);
        LE += lbar[k] * ebar[j];
        LGy += lbar[k] * gy[j];
        LGz += lbar[k] * gz[j];
    }
    double F = LE - ((A0y + A1y) * LGy + (A0z + A1z) * LGz) / (g10 + g11);
    if (hy) F += spin_force(c, x0, x1, sy, sz, hy, hz);   /* independent of p: the same in both orders */
    double Pn = p0 + c->dt * F;
    double g10n = sqrt(1.0 + Pn * Pn + qa0);
    *delta_out = delta;
    *P_out = Pn;
    *delta_next = c->dt * (p0 + Pn) / (g00 + g10n);
}

void orc_particle_map_adjoint(const orc_cfg *c, double x0, double p0, double P,
                              const double *ay, const double *az, const double *gy, const double *gz,
                              const double *ebar, double *delta_out, double *P_out, double *delta_next)
{
    adjoint_map_s(c, x0, p0, P, 0.0, 0.0, ay, az, gy, gz, NULL, NULL, ebar, delta_out, P_out, delta_next);
}

/* The adjoint Subsystem I scheme over the time step h, by Picard iteration on
 * (P, e_x) from P = p^n, e = e_x^n.  Sweep k forms P^(k+1) from (P^(k), e^(k)),
 * the increment delta^(k+1) of P^(k+1), and deposits the current of
 * delta^(k+1); e^(k+1) = e_x^n - M1^{-1} J.  The test is the max norm of the
 * change of the increment and of e; the commit is x^n + delta^(k+1), P^(k+1),
 * e^(k+1) (position and deposit from one increment: Gauss's law holds
 * exactly).  dcommit (nullable) receives the committed increments. */
int orc_substep_I_adjoint_s(const orc_cfg *cfg, double h, double *x, double *p, double *ex, const double *ay,
                            const double *az, const double *sy, const double *sz, double *dcommit,
                            int32_t *sweeps, double *res)
{
    orc_cfg ch = *cfg;
    ch.dt = h;
    const orc_cfg *c = &ch;
    int M = c->M;
    int64_t n = c->n;
    double *P = malloc(sizeof(double) * (n > 0 ? n : 1)), *Pn = malloc(sizeof(double) * (n > 0 ? n : 1)),
           *dn = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *ek = malloc(sizeof(double) * M), *enew = malloc(sizeof(double) * M),
           *ebar = malloc(sizeof(double) * M), *J = malloc(sizeof(double) * M),
           *MJ = malloc(sizeof(double) * M), *gy = malloc(sizeof(double) * M),
           *gz = malloc(sizeof(double) * M);
    if (!P || !Pn || !dn || !ek || !enew || !ebar || !J || !MJ || !gy || !gz) return ORC_ENOMEM;
    orc_apply_G(c, ay, gy);
    orc_apply_G(c, az, gz);
    const int spin = sy != NULL;
    double *hy = spin ? malloc(sizeof(double) * M) : NULL, *hz = spin ? malloc(sizeof(double) * M) : NULL;
    if (spin) {
        orc_apply_G(c, gy, hy);
        orc_apply_G(c, gz, hz);
    }
    for (int64_t a = 0; a < n; ++a) P[a] = p[a];
    memcpy(ek, ex, sizeof(double) * M);
    int status = ORC_ENOTCONV;
    double r = 0.0;
    int k;
    for (k = 0; k < c->kmax; ++k) {
        for (int j = 0; j < M; ++j) ebar[j] = 0.5 * (ex[j] + ek[j]);
        memset(J, 0, sizeof(double) * M);
        double rx = 0.0;
        for (int64_t a = 0; a < n; ++a) {
            double dk;
            adjoint_map_s(c, x[a], p[a], P[a], spin ? sy[a] : 0.0, spin ? sz[a] : 0.0, ay, az, gy, gz, hy, hz,
                          ebar, &dk, &Pn[a], &dn[a]);
            long jlo;
            double lbar[16];
            int nj = orc_line_mean(c, x[a], x[a] + dn[a], &jlo, lbar);
            double inc = (x[a] + dn[a]) - x[a];
            for (int q = 0; q < nj; ++q) J[imod(jlo + q, M)] += c->w * inc * lbar[q];
            double dd = fabs(dn[a] - dk);
            if (dd > rx) rx = dd;
        }
        orc_solve_M1(c, J, MJ);
        double re = 0.0;
        for (int j = 0; j < M; ++j) {
            enew[j] = ex[j] - MJ[j];
            double de = fabs(enew[j] - ek[j]);
            if (de > re) re = de;
        }
        r = rx > re ? rx : re;
        int last = (k == c->kmax - 1);
        if (r <= c->tol || (last && c->commit_unconverged)) {
            for (int64_t a = 0; a < n; ++a) {
                if (dcommit) dcommit[a] = dn[a];
                x[a] = wrap(c, x[a] + dn[a]);
                p[a] = Pn[a];
            }
            memcpy(ex, enew, sizeof(double) * M);
            status = (r <= c->tol) ? ORC_OK : ORC_ENOTCONV;
            ++k;
            break;
        }
        double *t = P; P = Pn; Pn = t;
        memcpy(ek, enew, sizeof(double) * M);
    }
    if (sweeps) *sweeps = k;
    if (res) *res = r;
    free(P); free(Pn); free(dn); free(ek); free(enew); free(ebar); free(J); free(MJ); free(gy); free(gz);
    free(hy); free(hz);
    return status;
}

int orc_substep_I_adjoint(const orc_cfg *cfg, double h, double *x, double *p, double *ex, const double *ay,
                          const double *az, double *dcommit, int32_t *sweeps, double *res)
{
    return orc_substep_I_adjoint_s(cfg, h, x, p, ex, ay, az, NULL, NULL, dcommit, sweeps, res);
}

/* ------------------------------------------------------------------ */
/* Subsystem II (Section 4.2): (e_y, e_z, a_y, a_z) with particles fixed. */
/* ------------------------------------------------------------------ */

/* Fixed point on e_perp^{n+1} of
 *   (M0 + dt^2 K/4) e^{n+1} = (M0 - dt^2 K/4) e^n + dt K a^n + dt b,
 *   b = sum_a w (A^{n+1}(x_a) + A^n(x_a)) Lambda0(x_a) / (g^n_a + g^{n+1}_a),
 *   a^{n+1} = a^n - dt/2 (e^n + e^{n+1}),
 * with the particle term lagged one iteration and the matrix inverted exactly. */
/* V1 deposit of the spins, u_j = sum_a w s_a Lambda1_j(x_a) (the vector
 * Lambda1(X)^T W S of the Subsystem II spin source). */
static void deposit_spin_v1(const orc_cfg *c, const double *x, const double *s, double *u)
{
    memset(u, 0, sizeof(double) * c->M);
    for (int64_t a = 0; a < c->n; ++a) {
        long i = cell_of(c, x[a]);
        for (long j = i - c->p + 1; j <= i; ++j) u[imod(j, c->M)] += c->w * s[a] * orc_lambda1(c, j, x[a]);
    }
}

int orc_substep_II_hs(const orc_cfg *cfg, double h, const double *x, const double *p, const double *sy,
                      const double *sz, double *ey, double *ez, double *ay, double *az, int32_t *iters,
                      double *res)
{
    orc_cfg ch = *cfg;
    ch.dt = h;
    const orc_cfg *c = &ch;
    int M = c->M;
    int64_t n = c->n;
    double *Any = malloc(sizeof(double) * n), *Anz = malloc(sizeof(double) * n),
           *gn = malloc(sizeof(double) * n);
    double *rhs_y = malloc(sizeof(double) * M), *rhs_z = malloc(sizeof(double) * M),
           *t = malloc(sizeof(double) * M), *eky = malloc(sizeof(double) * M),
           *ekz = malloc(sizeof(double) * M), *aky = malloc(sizeof(double) * M),
           *akz = malloc(sizeof(double) * M), *by = malloc(sizeof(double) * M),
           *bz = malloc(sizeof(double) * M), *eny = malloc(sizeof(double) * M),
           *enz = malloc(sizeof(double) * M);
    for (int64_t a = 0; a < n; ++a) {
        Any[a] = orc_field0(c, ay, x[a]);
        Anz[a] = orc_field0(c, az, x[a]);
        gn[a] = sqrt(1.0 + p[a] * p[a] + Any[a] * Any[a] + Anz[a] * Anz[a]);
    }
    /* constant part of the right-hand side */
    orc_apply_cn_minus(c, ey, rhs_y);
    orc_apply_K(c, ay, t);
    for (int j = 0; j < M; ++j) rhs_y[j] += c->dt * t[j];
    orc_apply_cn_minus(c, ez, rhs_z);
    orc_apply_K(c, az, t);
    for (int j = 0; j < M; ++j) rhs_z[j] += c->dt * t[j];
    if (sy) {
        /* spin source: e_y gains -hbar G^T Lambda1^T W S_z, e_z gains +hbar G^T Lambda1^T W S_y */
        double *u = malloc(sizeof(double) * M);
        deposit_spin_v1(c, x, sz, u);
        orc_apply_GT(c, u, t);
        for (int j = 0; j < M; ++j) rhs_y[j] -= c->dt * c->hbar * t[j];
        deposit_spin_v1(c, x, sy, u);
        orc_apply_GT(c, u, t);
        for (int j = 0; j < M; ++j) rhs_z[j] += c->dt * c->hbar * t[j];
        free(u);
    }

    memcpy(eky, ey, sizeof(double) * M);
    memcpy(ekz, ez, sizeof(double) * M);
    int status = ORC_ENOTCONV, k;
    double r = 0.0;
    for (k = 0; k < c->kmax; ++k) {
        for (int j = 0; j < M; ++j) {
            aky[j] = ay[j] - 0.5 * c->dt * (ey[j] + eky[j]);
            akz[j] = az[j] - 0.5 * c->dt * (ez[j] + ekz[j]);
        }
        memset(by, 0, sizeof(double) * M);
        memset(bz, 0, sizeof(double) * M);
        for (int64_t a = 0; a < n; ++a) {
            double Aky = orc_field0(c, aky, x[a]), Akz = orc_field0(c, akz, x[a]);
            double gk = sqrt(1.0 + p[a] * p[a] + Aky * Aky + Akz * Akz);
            double cy = c->w * (Aky + Any[a]) / (gn[a] + gk);
            double cz = c->w * (Akz + Anz[a]) / (gn[a] + gk);
            long i = cell_of(c, x[a]);
            for (long j = i - c->p; j <= i; ++j) {
                double l0 = orc_lambda0(c, j, x[a]);
                by[imod(j, M)] += cy * l0;
                bz[imod(j, M)] += cz * l0;
            }
        }
        for (int j = 0; j < M; ++j) { by[j] = rhs_y[j] + c->dt * by[j]; bz[j] = rhs_z[j] + c->dt * bz[j]; }
        orc_solve_cn(c, by, eny);
        orc_solve_cn(c, bz, enz);
        r = 0.0;
        for (int j = 0; j < M; ++j) {
            double dy = fabs(eny[j] - eky[j]), dz = fabs(enz[j] - ekz[j]);
            if (dy > r) r = dy;
            if (dz > r) r = dz;
        }
        memcpy(eky, eny, sizeof(double) * M);
        memcpy(ekz, enz, sizeof(double) * M);
        int last = (k == c->kmax - 1);
        if (r <= c->tol || (last && c->commit_unconverged)) {
            for (int j = 0; j < M; ++j) {
                ay[j] = ay[j] - 0.5 * c->dt * (ey[j] + eny[j]);
                az[j] = az[j] - 0.5 * c->dt * (ez[j] + enz[j]);
            }
            memcpy(ey, eny, sizeof(double) * M);
            memcpy(ez, enz, sizeof(double) * M);
            status = (r <= c->tol) ? ORC_OK : ORC_ENOTCONV;
            ++k;
            break;
        }
    }
    if (iters) *iters = k;
    if (res) *res = r;
    free(Any); free(Anz); free(gn); free(rhs_y); free(rhs_z); free(t); free(eky); free(ekz);
    free(aky); free(akz); free(by); free(bz); free(eny); free(enz);
    return status;
}

int orc_substep_II_h(const orc_cfg *cfg, double h, const double *x, const double *p, double *ey, double *ez,
                     double *ay, double *az, int32_t *iters, double *res)
{
    return orc_substep_II_hs(cfg, h, x, p, NULL, NULL, ey, ez, ay, az, iters, res);
}

/* Subsystem II over the configured step. */
int orc_substep_II(const orc_cfg *c, const double *x, const double *p, double *ey, double *ez,
                   double *ay, double *az, int32_t *iters, double *res)
{
    return orc_substep_II_h(c, c->dt, x, p, ey, ez, ay, az, iters, res);
}

/* ------------------------------------------------------------------ */
/* Subsystem III (Section 4.2): the spins, everything else fixed.        */
/* ------------------------------------------------------------------ */

/* Each spin obeys ds/dt = rhat s with
 *   rhat = [[0, Y, Z], [-Y, 0, 0], [-Z, 0, 0]],  Y = dA_y/dx(x_a), Z = dA_z/dx(x_a),
 * a constant matrix over the substep (x and a_perp are fixed), i.e. ds/dt =
 * r x s with r = (0, Z, -Y).  The exact solution over h is the rotation of
 * eq. spin_rodrigue:
 *   s^{n+1} = (I + sin(h|r|)/|r| rhat + 1/2 (sin(h|r|/2)/(|r|/2))^2 rhat^2) s^n,
 * written here with the matrix rhat and its square as printed (|r| = 0: the
 * identity). */
void orc_substep_III_h(const orc_cfg *c, double h, const double *x, const double *ay, const double *az,
                       double *sx, double *sy, double *sz)
{
    int M = c->M;
    double *gy = malloc(sizeof(double) * M), *gz = malloc(sizeof(double) * M);
    orc_apply_G(c, ay, gy);
    orc_apply_G(c, az, gz);
    for (int64_t a = 0; a < c->n; ++a) {
        double Y = orc_field1(c, gy, x[a]), Z = orc_field1(c, gz, x[a]);
        double R[3][3] = {{0.0, Y, Z}, {-Y, 0.0, 0.0}, {-Z, 0.0, 0.0}};
        double R2[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                R2[i][j] = 0.0;
                for (int k = 0; k < 3; ++k) R2[i][j] += R[i][k] * R[k][j];
            }
        double nr = sqrt(Y * Y + Z * Z);
        if (nr == 0.0) continue;
        double c1 = sin(h * nr) / nr;
        double hs = sin(0.5 * h * nr) / (0.5 * nr);
        double c2 = 0.5 * hs * hs;
        double s0[3] = {sx[a], sy[a], sz[a]}, s1[3];
        for (int i = 0; i < 3; ++i) {
            s1[i] = s0[i];
            for (int j = 0; j < 3; ++j) s1[i] += (c1 * R[i][j] + c2 * R2[i][j]) * s0[j];
        }
        sx[a] = s1[0]; sy[a] = s1[1]; sz[a] = s1[2];
    }
    free(gy); free(gz);
}

/* Discrete Hamiltonian with the Zeeman term of eq. discrete_H:
 * parts = {kinetic, 1/2 ex^T M1 ex, 1/2 sum e_c^T M0 e_c, 1/2 sum a_c^T K a_c,
 *          hbar sum_a w (s_y dA_z/dx - s_z dA_y/dx)(x_a), H}. */
void orc_energy_s(const orc_cfg *c, const double *x, const double *p, const double *sy, const double *sz,
                  const double *ex, const double *ey, const double *ez, const double *ay, const double *az,
                  double *parts)
{
    double five[5];
    orc_energy(c, x, p, ex, ey, ez, ay, az, five);
    int M = c->M;
    double *gy = malloc(sizeof(double) * M), *gz = malloc(sizeof(double) * M);
    orc_apply_G(c, ay, gy);
    orc_apply_G(c, az, gz);
    double zee = 0.0;
    for (int64_t a = 0; a < c->n; ++a)
        zee += c->w * (sy[a] * orc_field1(c, gz, x[a]) - sz[a] * orc_field1(c, gy, x[a]));
    zee *= c->hbar;
    for (int i = 0; i < 4; ++i) parts[i] = five[i];
    parts[4] = zee;
    parts[5] = five[4] + zee;
    free(gy); free(gz);
}

/* Steps with spin.  splitting = 0: Lie-Trotter I, II, III.  splitting = 1: the
 * symmetric composition I(dt/2), III(dt/2), II(dt), III(dt/2), adjoint I(dt/2)
 * (Subsystems II and III are self-adjoint: the discrete gradient of II is
 * symmetric in the two time levels, III is an exact flow).  On failure the state
 * (spins included) is restored to the start of the failing step.  energy rows
 * hold the six parts of orc_energy_s. */
int orc_step_s(const orc_cfg *c, int32_t nsteps, double *x, double *p, double *sx, double *sy, double *sz,
               double *ex, double *ey, double *ez, double *ay, double *az, int32_t *sweeps_I,
               int32_t *iters_II, int32_t *sweeps_I2, double *energy_per_step /* nsteps+1 x 6, nullable */)
{
    int M = c->M;
    int64_t n = c->n;
    size_t nb = sizeof(double) * (n > 0 ? n : 1);
    double *save = malloc(nb * 5), *sf = malloc(sizeof(double) * 5 * M);
    double *dprev = c->warm_previous ? malloc(nb) : NULL;
    int have_prev = 0;
    int status = ORC_OK;
    double h = c->splitting ? 0.5 * c->dt : c->dt;
    if (energy_per_step) orc_energy_s(c, x, p, sy, sz, ex, ey, ez, ay, az, energy_per_step);
    for (int s = 0; s < nsteps; ++s) {
        memcpy(save, x, sizeof(double) * n); memcpy(save + n, p, sizeof(double) * n);
        memcpy(save + 2 * n, sx, sizeof(double) * n); memcpy(save + 3 * n, sy, sizeof(double) * n);
        memcpy(save + 4 * n, sz, sizeof(double) * n);
        memcpy(sf, ex, sizeof(double) * M); memcpy(sf + M, ey, sizeof(double) * M);
        memcpy(sf + 2 * M, ez, sizeof(double) * M); memcpy(sf + 3 * M, ay, sizeof(double) * M);
        memcpy(sf + 4 * M, az, sizeof(double) * M);
        int32_t k1 = 0, k2 = 0, k3 = 0;
        int st = orc_substep_I_hs(c, h, x, p, ex, ay, az, sy, sz, have_prev ? dprev : NULL, dprev, &k1, NULL);
        if (st == ORC_OK) {
            if (c->splitting) orc_substep_III_h(c, h, x, ay, az, sx, sy, sz);
            st = orc_substep_II_hs(c, c->dt, x, p, sy, sz, ey, ez, ay, az, &k2, NULL);
        }
        if (st == ORC_OK) orc_substep_III_h(c, h, x, ay, az, sx, sy, sz);
        if (st == ORC_OK && c->splitting)
            st = orc_substep_I_adjoint_s(c, h, x, p, ex, ay, az, sy, sz, dprev, &k3, NULL);
        if (sweeps_I) sweeps_I[s] = k1;
        if (iters_II) iters_II[s] = k2;
        if (sweeps_I2) sweeps_I2[s] = k3;
        if (st != ORC_OK) {
            memcpy(x, save, sizeof(double) * n); memcpy(p, save + n, sizeof(double) * n);
            memcpy(sx, save + 2 * n, sizeof(double) * n); memcpy(sy, save + 3 * n, sizeof(double) * n);
            memcpy(sz, save + 4 * n, sizeof(double) * n);
            memcpy(ex, sf, sizeof(double) * M); memcpy(ey, sf + M, sizeof(double) * M);
            memcpy(ez, sf + 2 * M, sizeof(double) * M); memcpy(ay, sf + 3 * M, sizeof(double) * M);
            memcpy(az, sf + 4 * M, sizeof(double) * M);
            status = st;
            break;
        }
        have_prev = dprev != NULL;
        if (energy_per_step) orc_energy_s(c, x, p, sy, sz, ex, ey, ez, ay, az, energy_per_step + 6 * (s + 1));
    }
    free(save); free(sf); free(dprev);
    return status;
}

/* ------------------------------------------------------------------ */
/* One time step.  splitting = 0: the Lie-Trotter composition of        */
/* Section 5, Subsystem I then II.  splitting = 1: the symmetric        */
/* composition Subsystem I over dt/2, II over dt, adjoint I over dt/2.  */
/* Subsystem III is the identity without spin.  On failure the state   */
/* is restored to the start of the failing step.  sweeps_I2 (nullable)  */
/* receives the sweeps of the adjoint substep.                          */
/* ------------------------------------------------------------------ */
int orc_step(const orc_cfg *c, int32_t nsteps, double *x, double *p, double *ex, double *ey,
             double *ez, double *ay, double *az, int32_t *sweeps_I, int32_t *iters_II,
             int32_t *sweeps_I2, double *energy_per_step /* nsteps+1 x 5, nullable */)
{
    int M = c->M;
    int64_t n = c->n;
    double *sx = malloc(sizeof(double) * (n > 0 ? n : 1)), *sp = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *sf = malloc(sizeof(double) * 5 * M);
    double *dprev = c->warm_previous ? malloc(sizeof(double) * (n > 0 ? n : 1)) : NULL;
    int have_prev = 0;
    int status = ORC_OK;
    double h = c->splitting ? 0.5 * c->dt : c->dt;
    if (energy_per_step) orc_energy(c, x, p, ex, ey, ez, ay, az, energy_per_step);
    for (int s = 0; s < nsteps; ++s) {
        memcpy(sx, x, sizeof(double) * n);
        memcpy(sp, p, sizeof(double) * n);
        memcpy(sf, ex, sizeof(double) * M); memcpy(sf + M, ey, sizeof(double) * M);
        memcpy(sf + 2 * M, ez, sizeof(double) * M); memcpy(sf + 3 * M, ay, sizeof(double) * M);
        memcpy(sf + 4 * M, az, sizeof(double) * M);
        int32_t k1 = 0, k2 = 0, k3 = 0;
        int st = orc_substep_I_h(c, h, x, p, ex, ay, az, have_prev ? dprev : NULL, dprev, &k1, NULL);
        if (st == ORC_OK) st = orc_substep_II_h(c, c->dt, x, p, ey, ez, ay, az, &k2, NULL);
        if (st == ORC_OK && c->splitting) st = orc_substep_I_adjoint(c, h, x, p, ex, ay, az, dprev, &k3, NULL);
        if (sweeps_I) sweeps_I[s] = k1;
        if (iters_II) iters_II[s] = k2;
        if (sweeps_I2) sweeps_I2[s] = k3;
        if (st != ORC_OK) {
            memcpy(x, sx, sizeof(double) * n);
            memcpy(p, sp, sizeof(double) * n);
            memcpy(ex, sf, sizeof(double) * M); memcpy(ey, sf + M, sizeof(double) * M);
            memcpy(ez, sf + 2 * M, sizeof(double) * M); memcpy(ay, sf + 3 * M, sizeof(double) * M);
            memcpy(az, sf + 4 * M, sizeof(double) * M);
            status = st;
            break;
        }
        have_prev = dprev != NULL;
        if (energy_per_step) orc_energy(c, x, p, ex, ey, ez, ay, az, energy_per_step + 5 * (s + 1));
    }
    free(sx); free(sp); free(sf); free(dprev);
    return status;
}
