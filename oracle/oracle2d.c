/*
 * Plain FP64 CPU oracle of the reduced 2D model (Sections 2.2, 3.2 and 4.3 of Li,
 * "Energy conserving particle-in-cell methods for relativistic Vlasov-Maxwell
 * equations of laser-plasma interaction"), without spin (the plain functions) and with
 * the spin terms (the _s functions, hbar != 0).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * code, header, table or helper with the HIP library.  It uses the 1D oracle's
 * B-spline (Cox-de Boor) and mass-matrix row (Gauss-Legendre) from oracle.c;
 * everything else is written out here, slowly and literally.
 *
 * Conventions (Section 3.2: tensor products of the 1D bases of Section 3.1, the
 * same degree p in both directions):
 *   - grid x_{1,j} = j dx1, x_{2,j} = j dx2; coefficient index i = i1 M2 + i2,
 *     both indices periodic; N^d_j(x) = B_d(x/dx - j), support [x_j, x_{j+d+1});
 *   - V0 (a_z, e_z): N^p_{i1}(x1) N^p_{i2}(x2);
 *     V1 (e_xy = (e1, e2)): (N^{p-1}_{i1} N^p_{i2}, 0) and (0, N^p_{i1} N^{p-1}_{i2});
 *     V2 (b_z): N^{p-1}_{i1} N^{p-1}_{i2};
 *   - (G a)_1 = (a_{i1,i2} - a_{i1-1,i2}) / dx1, (G a)_2 = (a_{i1,i2} - a_{i1,i2-1}) / dx2
 *     (grad of a V0 field, exactly, in V1);
 *     (C e)_i = (e2_{i1,i2} - e2_{i1-1,i2}) / dx1 - (e1_{i1,i2} - e1_{i1,i2-1}) / dx2
 *     (curl of a V1 field, exactly, in V2); C G = 0;
 *   - mass matrices are tensor products of the 1D circulant mass matrices;
 *     the stiffness of a_z in the Hamiltonian, G*^T M1* G*, equals K = G^T M1 G
 *     because |grad^T A_z| = |grad A_z|.
 * Readings of the paper taken here (also listed in the design notes):
 *   - discrete Gauss law r = G^T M1 e_xy + Lambda0(X)^T W 1 - dx1 dx2 1, as in 1D;
 *     the initial e_xy is the given field plus -G phi with K phi chosen so r = 0;
 *   - Subsystem I: the field in the momentum update is (e^n + e^{n+1})/2 (the
 *     printed scheme leaves the time level off; the midpoint is the one that
 *     conserves the discrete energy);
 *   - Subsystem I: the two divided differences of A_z along the path (x2 varied
 *     first at x1^n, then x1 at x2^{n+1}) are evaluated as the means of dA_z/dx2
 *     and dA_z/dx1 along those two straight legs (0/0-free, exact identity);
 *   - Subsystem I: Jacobi Picard map in (delta, e_xy), started from
 *     delta = dt p^n / gamma(x^n, p^n), e = e^n, stopped on the max norm of both
 *     increments, committing x^n + delta^(k), p^(k+1), e^(k+1) (the triple whose
 *     position and deposited current agree exactly);
 *   - Subsystem III: fixed point in e_z with the linear part (M0 + dt^2 K/4)
 *     solved exactly, stopped on the max norm of the e_z increment; the printed
 *     iteration preconditioned by M0 converges to the same solution;
 *   - Subsystem IV: the linear system for e_xy solved exactly, then b_z;
 *   - Lie-Trotter step: I, II, III, IV in the order the splitting numbers them.
 * With spin (Section 2.2's Zeeman term hbar sum_a w s_a . B_h(x_a), Section 4.3):
 *   - B_h = (dA_z/dx2, -dA_z/dx1, B_z); dA_z/dx2 has the coefficients (G a)_2 on the
 *     degrees (p, p-1) and dA_z/dx1 the coefficients (G a)_1 on (p-1, p), so
 *     G* a = ((G a)_2, -(G a)_1) and Lambda1* pairs (p, p-1) with s_x and (p-1, p)
 *     with s_y;
 *   - Subsystem I: the divided differences of dA_z/dx2, dA_z/dx1 and B_z along the
 *     same two legs as A_z's are the means of their derivatives along the legs (the
 *     derivative coefficients are again backward differences); the momentum
 *     update subtracts dt hbar (s_x DD(dA_z/dx2) - s_y DD(dA_z/dx1) + s_z DD(B_z));
 *   - Subsystem II: ds/dt = s x B_h(x) with B_h fixed, so s turns about B_h by the
 *     angle -|B_h| dt (Rodrigues' formula), and p turns by B_z as without spin;
 *   - Subsystem III: the right-hand side gains hbar dt G*^T Lambda1*(X^n)^T W S_xy;
 *   - Subsystem IV: it gains hbar dt C^T Lambda2(X^n)^T W S_z.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double L1, L2;
    int32_t M1, M2;
    int32_t p;        /* degree of V0 in both directions */
    int32_t kmax;     /* Picard iteration cap (Subsystems I and III) */
    int64_t n;        /* particles */
    double w;         /* weight omega_a (all equal) */
    double dt;
    double tol;       /* absolute max-norm tolerance of the fixed points */
} orc2_cfg;

enum { ORC2_OK = 0, ORC2_ENOTCONV = -3, ORC2_ENOMEM = -2 };

double orc_bspline(int d, double u);   /* oracle.c: cardinal B-spline, Cox-de Boor */
void orc_mass_row(int d, double *row); /* oracle.c: row of the 1D mass matrix, dx = 1 */

static const double GX[6] = {-0.9324695142031521, -0.6612093864662645, -0.2386191860831969,
                             0.2386191860831969,  0.6612093864662645,  0.9324695142031521};
static const double GW[6] = {0.1713244923791704, 0.3607615730481386, 0.4679139345726910,
                             0.4679139345726910, 0.3607615730481386, 0.1713244923791704};

static long imod2(long j, long M) { long r = j % M; return r < 0 ? r + M : r; }
static double h1(const orc2_cfg *c) { return c->L1 / (double)c->M1; }
static double h2(const orc2_cfg *c) { return c->L2 / (double)c->M2; }
static long nodes(const orc2_cfg *c) { return (long)c->M1 * (long)c->M2; }
static long at(const orc2_cfg *c, long i1, long i2) { return imod2(i1, c->M1) * c->M2 + imod2(i2, c->M2); }

/* ------------------------------------------------------------------ */
/* Section 3.2: tensor-product fields and point deposits.               */
/* ------------------------------------------------------------------ */

/* The (d+1) splines of degree d that do not vanish at u = x/dx: vals[k] is
 * N^d_{j0+k}(x), j0 = floor(u) - d. */
static long spl(int d, double u, double *vals)
{
    long c = (long)floor(u);
    for (int k = 0; k <= d; ++k) vals[k] = orc_bspline(d, u - (double)(c - d + k));
    return c - d;
}

/* sum_{i1,i2} coef_i N^{d1}_{i1}(x1) N^{d2}_{i2}(x2) at an unwrapped point. */
double orc2_eval(const orc2_cfg *c, const double *coef, int d1, int d2, double x1, double x2)
{
    double v1[8], v2[8];
    long j1 = spl(d1, x1 / h1(c), v1), j2 = spl(d2, x2 / h2(c), v2);
    double s = 0.0;
    for (int a = 0; a <= d1; ++a)
        for (int b = 0; b <= d2; ++b) s += coef[at(c, j1 + a, j2 + b)] * v1[a] * v2[b];
    return s;
}

/* grid_i += q N^{d1}_{i1}(x1) N^{d2}_{i2}(x2). */
static void deposit_point(const orc2_cfg *c, double *grid, int d1, int d2, double x1, double x2, double q)
{
    double v1[8], v2[8];
    long j1 = spl(d1, x1 / h1(c), v1), j2 = spl(d2, x2 / h2(c), v2);
    for (int a = 0; a <= d1; ++a)
        for (int b = 0; b <= d2; ++b) grid[at(c, j1 + a, j2 + b)] += q * v1[a] * v2[b];
}

/* ------------------------------------------------------------------ */
/* Means along a straight segment (the trajectory of Subsystem I).      */
/* ------------------------------------------------------------------ */

static int cmp_dbl(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Breakpoints in [0, 1] of the segment a -> b (physical units): the parameters s
 * at which a coordinate crosses a grid line, plus 0 and 1, sorted.  Between two
 * breakpoints both coordinates stay in one cell, so a tensor-product spline is a
 * polynomial of degree d1 + d2 in s there. */
static int breaks(const orc2_cfg *c, double a1, double a2, double b1, double b2, double **out)
{
    double u[2] = {a1 / h1(c), a2 / h2(c)}, v[2] = {b1 / h1(c), b2 / h2(c)};
    long cnt = 2;
    for (int d = 0; d < 2; ++d) cnt += labs((long)floor(v[d]) - (long)floor(u[d])) + 1;
    double *s = malloc(sizeof(double) * (size_t)cnt);
    int n = 0;
    s[n++] = 0.0;
    s[n++] = 1.0;
    for (int d = 0; d < 2; ++d) {
        if (v[d] == u[d]) continue;
        double lo = u[d] < v[d] ? u[d] : v[d], hi = u[d] < v[d] ? v[d] : u[d];
        for (long k = (long)floor(lo) + 1; (double)k < hi; ++k) {
            double t = ((double)k - u[d]) / (v[d] - u[d]);
            if (t > 0.0 && t < 1.0) s[n++] = t;
        }
    }
    qsort(s, (size_t)n, sizeof(double), cmp_dbl);
    *out = s;
    return n;
}

/* int_0^1 F(a + s (b - a)) ds of the tensor-product field coef of degrees (d1, d2):
 * the mean of the field along the segment, exact (6-point Gauss-Legendre on each
 * piece, exact to degree 11 >= d1 + d2). */
double orc2_line_mean(const orc2_cfg *c, const double *coef, int d1, int d2, double a1, double a2, double b1,
                      double b2)
{
    double *s;
    int n = breaks(c, a1, a2, b1, b2, &s);
    double acc = 0.0;
    for (int k = 0; k + 1 < n; ++k) {
        double s0 = s[k], s1 = s[k + 1];
        if (!(s1 > s0)) continue;
        for (int q = 0; q < 6; ++q) {
            double t = 0.5 * (s0 + s1) + 0.5 * (s1 - s0) * GX[q];
            acc += 0.5 * (s1 - s0) * GW[q] *
                   orc2_eval(c, coef, d1, d2, a1 + t * (b1 - a1), a2 + t * (b2 - a2));
        }
    }
    free(s);
    return acc;
}

/* grid_i += q int_0^1 Lambda_i(a + s (b - a)) ds for the basis of degrees (d1, d2). */
void orc2_line_deposit(const orc2_cfg *c, double *grid, int d1, int d2, double a1, double a2, double b1,
                       double b2, double q)
{
    double *s;
    int n = breaks(c, a1, a2, b1, b2, &s);
    for (int k = 0; k + 1 < n; ++k) {
        double s0 = s[k], s1 = s[k + 1];
        if (!(s1 > s0)) continue;
        for (int g = 0; g < 6; ++g) {
            double t = 0.5 * (s0 + s1) + 0.5 * (s1 - s0) * GX[g];
            deposit_point(c, grid, d1, d2, a1 + t * (b1 - a1), a2 + t * (b2 - a2), q * 0.5 * (s1 - s0) * GW[g]);
        }
    }
    free(s);
}

/* ------------------------------------------------------------------ */
/* Section 3.2: mass matrices, G, C, K and their transposes.            */
/* ------------------------------------------------------------------ */

/* y = (Mass_{d1} (x) Mass_{d2}) x: y_i = dx1 dx2 sum_{k1,k2} r1_{k1} r2_{k2} x_{i1+k1, i2+k2}. */
static void apply_mass(const orc2_cfg *c, int d1, int d2, const double *x, double *y)
{
    double r1[16], r2[16];
    orc_mass_row(d1, r1);
    orc_mass_row(d2, r2);
    double s = h1(c) * h2(c);
    for (long i1 = 0; i1 < c->M1; ++i1)
        for (long i2 = 0; i2 < c->M2; ++i2) {
            double acc = 0.0;
            for (int k1 = -d1; k1 <= d1; ++k1)
                for (int k2 = -d2; k2 <= d2; ++k2) acc += r1[k1 + d1] * r2[k2 + d2] * x[at(c, i1 + k1, i2 + k2)];
            y[i1 * c->M2 + i2] = s * acc;
        }
}

void orc2_apply_M0(const orc2_cfg *c, const double *x, double *y) { apply_mass(c, c->p, c->p, x, y); }
void orc2_apply_M2(const orc2_cfg *c, const double *x, double *y) { apply_mass(c, c->p - 1, c->p - 1, x, y); }
/* V1 vectors are (e1, e2) back to back, each M1 M2 long. */
void orc2_apply_M1(const orc2_cfg *c, const double *x, double *y)
{
    apply_mass(c, c->p - 1, c->p, x, y);
    apply_mass(c, c->p, c->p - 1, x + nodes(c), y + nodes(c));
}

void orc2_apply_G(const orc2_cfg *c, const double *a, double *g)
{
    long N = nodes(c);
    for (long i1 = 0; i1 < c->M1; ++i1)
        for (long i2 = 0; i2 < c->M2; ++i2) {
            long i = i1 * c->M2 + i2;
            g[i] = (a[i] - a[at(c, i1 - 1, i2)]) / h1(c);
            g[N + i] = (a[i] - a[at(c, i1, i2 - 1)]) / h2(c);
        }
}

void orc2_apply_GT(const orc2_cfg *c, const double *u, double *y)
{
    long N = nodes(c);
    for (long i1 = 0; i1 < c->M1; ++i1)
        for (long i2 = 0; i2 < c->M2; ++i2) {
            long i = i1 * c->M2 + i2;
            y[i] = (u[i] - u[at(c, i1 + 1, i2)]) / h1(c) + (u[N + i] - u[N + at(c, i1, i2 + 1)]) / h2(c);
        }
}

void orc2_apply_C(const orc2_cfg *c, const double *e, double *b)
{
    long N = nodes(c);
    for (long i1 = 0; i1 < c->M1; ++i1)
        for (long i2 = 0; i2 < c->M2; ++i2) {
            long i = i1 * c->M2 + i2;
            b[i] = (e[N + i] - e[N + at(c, i1 - 1, i2)]) / h1(c) - (e[i] - e[at(c, i1, i2 - 1)]) / h2(c);
        }
}

void orc2_apply_CT(const orc2_cfg *c, const double *b, double *e)
{
    long N = nodes(c);
    for (long i1 = 0; i1 < c->M1; ++i1)
        for (long i2 = 0; i2 < c->M2; ++i2) {
            long i = i1 * c->M2 + i2;
            e[i] = -(b[i] - b[at(c, i1, i2 + 1)]) / h2(c);
            e[N + i] = (b[i] - b[at(c, i1 + 1, i2)]) / h1(c);
        }
}

/* K a = G^T M1 G a. */
void orc2_apply_K(const orc2_cfg *c, const double *a, double *y)
{
    long N = nodes(c);
    double *g = malloc(sizeof(double) * 2 * N), *mg = malloc(sizeof(double) * 2 * N);
    orc2_apply_G(c, a, g);
    orc2_apply_M1(c, g, mg);
    orc2_apply_GT(c, mg, y);
    free(g); free(mg);
}

/* C^T M2 C e (V1 -> V1). */
static void apply_CtM2C(const orc2_cfg *c, const double *e, double *y)
{
    long N = nodes(c);
    double *b = malloc(sizeof(double) * N), *mb = malloc(sizeof(double) * N);
    orc2_apply_C(c, e, b);
    orc2_apply_M2(c, b, mb);
    orc2_apply_CT(c, mb, y);
    free(b); free(mb);
}

/* ------------------------------------------------------------------ */
/* Linear solves: conjugate gradients with two refinement passes.       */
/* ------------------------------------------------------------------ */
typedef void (*orc2_op)(const orc2_cfg *, double, const double *, double *);

static double dot2(long n, const double *a, const double *b)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void cg2_core(const orc2_cfg *c, orc2_op A, double prm, long n, int zero_mean, const double *b, double *x)
{
    double *r = malloc(sizeof(double) * n), *d = malloc(sizeof(double) * n), *Ad = malloc(sizeof(double) * n),
           *best = malloc(sizeof(double) * n);
    memset(x, 0, sizeof(double) * n);
    memcpy(r, b, sizeof(double) * n);
    if (zero_mean) {   /* singular K: solve on the complement of the constants */
        double m = 0.0;
        for (long i = 0; i < n; ++i) m += r[i];
        m /= (double)n;
        for (long i = 0; i < n; ++i) r[i] -= m;
    }
    memcpy(d, r, sizeof(double) * n);
    memset(best, 0, sizeof(double) * n);
    double rr = dot2(n, r, r), bb = rr, best_rr = rr;
    int stall = 0;
    if (bb > 0.0) {
        for (long it = 0; it < 20 * n + 200; ++it) {
            A(c, prm, d, Ad);
            double alpha = rr / dot2(n, d, Ad);
            for (long i = 0; i < n; ++i) { x[i] += alpha * d[i]; r[i] -= alpha * Ad[i]; }
            double rn = dot2(n, r, r);
            if (rn < best_rr) { best_rr = rn; stall = 0; memcpy(best, x, sizeof(double) * n); }
            else ++stall;
            /* the residual norm of CG is not monotone on ill-conditioned systems (the
             * quintic mass matrices): allow a full 2n iterations without a new best */
            if (rn <= 1e-36 * bb || stall >= 2 * n + 50) break;
            double beta = rn / rr;
            for (long i = 0; i < n; ++i) d[i] = r[i] + beta * d[i];
            rr = rn;
        }
        memcpy(x, best, sizeof(double) * n);
    }
    if (zero_mean) {
        double m = 0.0;
        for (long i = 0; i < n; ++i) m += x[i];
        m /= (double)n;
        for (long i = 0; i < n; ++i) x[i] -= m;
    }
    free(r); free(d); free(Ad); free(best);
}

static void solve2(const orc2_cfg *c, orc2_op A, double prm, long n, int zero_mean, const double *b, double *x)
{
    double *r = malloc(sizeof(double) * n), *dx = malloc(sizeof(double) * n);
    cg2_core(c, A, prm, n, zero_mean, b, x);
    for (int pass = 0; pass < 2; ++pass) {
        A(c, prm, x, r);
        for (long i = 0; i < n; ++i) r[i] = b[i] - r[i];
        cg2_core(c, A, prm, n, zero_mean, r, dx);
        for (long i = 0; i < n; ++i) x[i] += dx[i];
    }
    free(r); free(dx);
}

static void op_M1(const orc2_cfg *c, double prm, const double *x, double *y) { (void)prm; orc2_apply_M1(c, x, y); }
static void op_K(const orc2_cfg *c, double prm, const double *x, double *y) { (void)prm; orc2_apply_K(c, x, y); }
/* M0 + prm K (Subsystem III with prm = dt^2/4). */
static void op_M0K(const orc2_cfg *c, double prm, const double *x, double *y)
{
    long N = nodes(c);
    double *t = malloc(sizeof(double) * N);
    orc2_apply_M0(c, x, y);
    orc2_apply_K(c, x, t);
    for (long i = 0; i < N; ++i) y[i] += prm * t[i];
    free(t);
}
/* M1 + prm C^T M2 C (Subsystem IV with prm = dt^2/4). */
static void op_M1C(const orc2_cfg *c, double prm, const double *x, double *y)
{
    long N2 = 2 * nodes(c);
    double *t = malloc(sizeof(double) * N2);
    orc2_apply_M1(c, x, y);
    apply_CtM2C(c, x, t);
    for (long i = 0; i < N2; ++i) y[i] += prm * t[i];
    free(t);
}

void orc2_solve_M1(const orc2_cfg *c, const double *b, double *x) { solve2(c, op_M1, 0.0, 2 * nodes(c), 0, b, x); }

/* ------------------------------------------------------------------ */
/* Discrete Gauss law, initial field, energy.                           */
/* ------------------------------------------------------------------ */

void orc2_deposit_charge(const orc2_cfg *c, const double *x1, const double *x2, double *rho)
{
    memset(rho, 0, sizeof(double) * nodes(c));
    for (int64_t a = 0; a < c->n; ++a) deposit_point(c, rho, c->p, c->p, x1[a], x2[a], c->w);
}

/* r = G^T M1 e + Lambda0(X)^T W 1 - dx1 dx2 1; returns max |r_i|. */
double orc2_gauss_residual(const orc2_cfg *c, const double *x1, const double *x2, const double *e, double *r_out)
{
    long N = nodes(c);
    double *me = malloc(sizeof(double) * 2 * N), *r = malloc(sizeof(double) * N), *rho = malloc(sizeof(double) * N);
    orc2_apply_M1(c, e, me);
    orc2_apply_GT(c, me, r);
    orc2_deposit_charge(c, x1, x2, rho);
    double m = 0.0;
    for (long i = 0; i < N; ++i) {
        r[i] += rho[i] - h1(c) * h2(c);
        if (fabs(r[i]) > m) m = fabs(r[i]);
    }
    if (r_out) memcpy(r_out, r, sizeof(double) * N);
    free(me); free(r); free(rho);
    return m;
}

/* e <- e - G phi with K phi = G^T M1 e + rho - dx1 dx2 (zero-mean phi): the
 * given e_xy corrected so that the discrete Gauss law holds. */
void orc2_solve_gauss(const orc2_cfg *c, const double *x1, const double *x2, double *e)
{
    long N = nodes(c);
    double *r = malloc(sizeof(double) * N), *phi = malloc(sizeof(double) * N), *g = malloc(sizeof(double) * 2 * N);
    orc2_gauss_residual(c, x1, x2, e, r);
    solve2(c, op_K, 0.0, N, 1, r, phi);
    orc2_apply_G(c, phi, g);
    for (long i = 0; i < 2 * N; ++i) e[i] -= g[i];
    free(r); free(phi); free(g);
}

static double gam(double p1, double p2, double A) { return sqrt(1.0 + p1 * p1 + p2 * p2 + A * A); }

/* Discrete Hamiltonian (eq. discrete_H2d, hbar = 0): out = {kinetic, 1/2 e^T M1 e,
 * 1/2 b^T M2 b, 1/2 e_z^T M0 e_z, 1/2 a^T K a, total}. */
void orc2_energy(const orc2_cfg *c, const double *x1, const double *x2, const double *p1, const double *p2,
                 const double *e, const double *bz, const double *ez, const double *az, double *out)
{
    long N = nodes(c);
    double kin = 0.0;
    for (int64_t a = 0; a < c->n; ++a) {
        double A = orc2_eval(c, az, c->p, c->p, x1[a], x2[a]);
        kin += c->w * (gam(p1[a], p2[a], A) - 1.0);
    }
    double *t = malloc(sizeof(double) * 2 * N);
    orc2_apply_M1(c, e, t);
    double ee = 0.5 * dot2(2 * N, e, t);
    orc2_apply_M2(c, bz, t);
    double bb = 0.5 * dot2(N, bz, t);
    orc2_apply_M0(c, ez, t);
    double zz = 0.5 * dot2(N, ez, t);
    orc2_apply_K(c, az, t);
    double aa = 0.5 * dot2(N, az, t);
    free(t);
    out[0] = kin; out[1] = ee; out[2] = bb; out[3] = zz; out[4] = aa;
    out[5] = kin + ee + bb + zz + aa;
}

static double wrapL(double x, double L)
{
    double y = fmod(x, L);
    if (y < 0.0) y += L;
    if (y >= L) y -= L;
    return y;
}

/* ------------------------------------------------------------------ */
/* Section 4.3, Subsystem I: x, p, e_xy by the discrete gradient.       */
/* ------------------------------------------------------------------ */

/* One application of the momentum and position updates of the Subsystem I scheme
 * for one particle, given the increment d = x^{n+1} - x^n and the mean field
 * ebar = (e^n + e^{n+1})/2:
 *   Ebar = mean of Lambda1^T ebar along the straight path x^n -> x^n + d,
 *   F = -(A(x^n) + A(x^n+d)) (D1, D2) / (gamma(p^n, A(x^n)) + gamma(p^n, A(x^n+d))),
 *   D2 = mean of dA/dx2 along (x1^n, x2^n) -> (x1^n, x2^n + d2),
 *   D1 = mean of dA/dx1 along (x1^n, x2^n + d2) -> (x1^n + d1, x2^n + d2),
 *   p^{n+1} = p^n + dt (Ebar + F),
 *   d' = dt (p^n + p^{n+1}) / (gamma(p^n, A(x^n+d)) + gamma(p^{n+1}, A(x^n+d))). */
void orc2_particle_map(const orc2_cfg *c, double x1, double x2, double p1, double p2, double d1, double d2,
                       const double *ebar, const double *az, const double *ga, double *pn, double *dn)
{
    long N = nodes(c);
    int p = c->p;
    double b1 = x1 + d1, b2 = x2 + d2;
    double E1 = orc2_line_mean(c, ebar, p - 1, p, x1, x2, b1, b2);
    double E2 = orc2_line_mean(c, ebar + N, p, p - 1, x1, x2, b1, b2);
    double Aa = orc2_eval(c, az, p, p, x1, x2), Ab = orc2_eval(c, az, p, p, b1, b2);
    double D2 = orc2_line_mean(c, ga + N, p, p - 1, x1, x2, x1, b2);
    double D1 = orc2_line_mean(c, ga, p - 1, p, x1, b2, b1, b2);
    double ga_ = gam(p1, p2, Aa), gb = gam(p1, p2, Ab);
    double f = -(Aa + Ab) / (ga_ + gb);
    double q1 = p1 + c->dt * (E1 + f * D1), q2 = p2 + c->dt * (E2 + f * D2);
    double gc = gam(q1, q2, Ab);
    pn[0] = q1;
    pn[1] = q2;
    dn[0] = c->dt * (p1 + q1) / (gb + gc);
    dn[1] = c->dt * (p2 + q2) / (gb + gc);
}

int orc2_substep_I(const orc2_cfg *cfg, double h, double *x1, double *x2, double *p1, double *p2, double *e,
                   const double *az, int32_t *sweeps, double *res)
{
    orc2_cfg ch = *cfg;
    ch.dt = h;
    const orc2_cfg *c = &ch;
    long N = nodes(c), N2 = 2 * N;
    int64_t n = c->n;
    int p = c->p;
    double *d = malloc(sizeof(double) * 2 * n), *dn = malloc(sizeof(double) * 2 * n),
           *pk = malloc(sizeof(double) * 2 * n);
    double *ek = malloc(sizeof(double) * N2), *enew = malloc(sizeof(double) * N2),
           *ebar = malloc(sizeof(double) * N2), *J = malloc(sizeof(double) * N2),
           *MJ = malloc(sizeof(double) * N2), *ga = malloc(sizeof(double) * N2);
    if (!d || !dn || !pk || !ek || !enew || !ebar || !J || !MJ || !ga) return ORC2_ENOMEM;
    orc2_apply_G(c, az, ga);
    for (int64_t a = 0; a < n; ++a) {
        double g = gam(p1[a], p2[a], orc2_eval(c, az, p, p, x1[a], x2[a]));
        d[2 * a] = c->dt * p1[a] / g;
        d[2 * a + 1] = c->dt * p2[a] / g;
    }
    memcpy(ek, e, sizeof(double) * N2);
    int status = ORC2_ENOTCONV, k;
    double r = 0.0;
    for (k = 0; k < c->kmax; ++k) {
        for (long i = 0; i < N2; ++i) ebar[i] = 0.5 * (e[i] + ek[i]);
        memset(J, 0, sizeof(double) * N2);
        double rx = 0.0;
        for (int64_t a = 0; a < n; ++a) {
            orc2_particle_map(c, x1[a], x2[a], p1[a], p2[a], d[2 * a], d[2 * a + 1], ebar, az, ga, &pk[2 * a],
                              &dn[2 * a]);
            /* current of the increment d^(k): w times the path mean of Lambda1 times d */
            double b1 = x1[a] + d[2 * a], b2 = x2[a] + d[2 * a + 1];
            orc2_line_deposit(c, J, p - 1, p, x1[a], x2[a], b1, b2, c->w * d[2 * a]);
            orc2_line_deposit(c, J + N, p, p - 1, x1[a], x2[a], b1, b2, c->w * d[2 * a + 1]);
            for (int q = 0; q < 2; ++q) {
                double dd = fabs(dn[2 * a + q] - d[2 * a + q]);
                if (dd > rx) rx = dd;
            }
        }
        orc2_solve_M1(c, J, MJ);
        double re = 0.0;
        for (long i = 0; i < N2; ++i) {
            enew[i] = e[i] - MJ[i];
            double de = fabs(enew[i] - ek[i]);
            if (de > re) re = de;
        }
        r = rx > re ? rx : re;
        if (r <= c->tol) {
            for (int64_t a = 0; a < n; ++a) {
                x1[a] = wrapL(x1[a] + d[2 * a], c->L1);
                x2[a] = wrapL(x2[a] + d[2 * a + 1], c->L2);
                p1[a] = pk[2 * a];
                p2[a] = pk[2 * a + 1];
            }
            memcpy(e, enew, sizeof(double) * N2);
            status = ORC2_OK;
            ++k;
            break;
        }
        double *t = d; d = dn; dn = t;
        memcpy(ek, enew, sizeof(double) * N2);
    }
    if (sweeps) *sweeps = k;
    if (res) *res = r;
    free(d); free(dn); free(pk); free(ek); free(enew); free(ebar); free(J); free(MJ); free(ga);
    return status;
}

/* ------------------------------------------------------------------ */
/* Section 4.3, Subsystem II: rotation of p by B_z (the S^p block).      */
/* ------------------------------------------------------------------ */

/* dp/dt = (p2, -p1) B_z(x) / gamma with gamma = sqrt(1 + |p|^2 + A_z(x)^2) constant
 * (|p| and x do not change): p turns clockwise by the angle B_z dt / gamma. */
void orc2_substep_II(const orc2_cfg *c, double h, const double *x1, const double *x2, double *p1, double *p2,
                     const double *bz, const double *az)
{
    int p = c->p;
    for (int64_t a = 0; a < c->n; ++a) {
        double B = orc2_eval(c, bz, p - 1, p - 1, x1[a], x2[a]);
        double A = orc2_eval(c, az, p, p, x1[a], x2[a]);
        double th = B * h / gam(p1[a], p2[a], A);
        double q1 = p1[a] * cos(th) + p2[a] * sin(th);
        double q2 = -p1[a] * sin(th) + p2[a] * cos(th);
        p1[a] = q1;
        p2[a] = q2;
    }
}

/* ------------------------------------------------------------------ */
/* Section 4.3, Subsystem III: a_z, e_z.                                */
/* ------------------------------------------------------------------ */

/* (M0 + h^2 K/4) e^{n+1} = (M0 - h^2 K/4) e^n + h K a^n
 *     + h sum_a w (A^n(x_a) + A^{n+1}(x_a)) Lambda0(x_a) / (gamma(p_a, A^n) + gamma(p_a, A^{n+1})),
 * a^{n+1} = a^n - h (e^n + e^{n+1})/2, iterated on e_z from e^n. */
int orc2_substep_III(const orc2_cfg *cfg, double h, const double *x1, const double *x2, const double *p1,
                     const double *p2, double *ez, double *az, int32_t *iters, double *res)
{
    orc2_cfg ch = *cfg;
    ch.dt = h;
    const orc2_cfg *c = &ch;
    long N = nodes(c);
    int64_t n = c->n;
    int p = c->p;
    double *An = malloc(sizeof(double) * n), *gn = malloc(sizeof(double) * n);
    double *rhs = malloc(sizeof(double) * N), *t = malloc(sizeof(double) * N), *ek = malloc(sizeof(double) * N),
           *ak = malloc(sizeof(double) * N), *S = malloc(sizeof(double) * N), *en = malloc(sizeof(double) * N);
    for (int64_t a = 0; a < n; ++a) {
        An[a] = orc2_eval(c, az, p, p, x1[a], x2[a]);
        gn[a] = gam(p1[a], p2[a], An[a]);
    }
    op_M0K(c, -0.25 * h * h, ez, rhs);
    orc2_apply_K(c, az, t);
    for (long i = 0; i < N; ++i) rhs[i] += h * t[i];
    memcpy(ek, ez, sizeof(double) * N);
    int status = ORC2_ENOTCONV, k;
    double r = 0.0;
    for (k = 0; k < c->kmax; ++k) {
        for (long i = 0; i < N; ++i) ak[i] = az[i] - 0.5 * h * (ez[i] + ek[i]);
        memset(S, 0, sizeof(double) * N);
        for (int64_t a = 0; a < n; ++a) {
            double Ak = orc2_eval(c, ak, p, p, x1[a], x2[a]);
            double q = c->w * (An[a] + Ak) / (gn[a] + gam(p1[a], p2[a], Ak));
            deposit_point(c, S, p, p, x1[a], x2[a], q);
        }
        for (long i = 0; i < N; ++i) S[i] = rhs[i] + h * S[i];
        solve2(c, op_M0K, 0.25 * h * h, N, 0, S, en);
        r = 0.0;
        for (long i = 0; i < N; ++i) {
            double de = fabs(en[i] - ek[i]);
            if (de > r) r = de;
        }
        memcpy(ek, en, sizeof(double) * N);
        if (r <= c->tol) {
            for (long i = 0; i < N; ++i) az[i] = az[i] - 0.5 * h * (ez[i] + en[i]);
            memcpy(ez, en, sizeof(double) * N);
            status = ORC2_OK;
            ++k;
            break;
        }
    }
    if (iters) *iters = k;
    if (res) *res = r;
    free(An); free(gn); free(rhs); free(t); free(ek); free(ak); free(S); free(en);
    return status;
}

/* ------------------------------------------------------------------ */
/* Section 4.3, Subsystem IV: e_xy, b_z (Maxwell, implicit midpoint).   */
/* ------------------------------------------------------------------ */

/* (M1 + h^2 C^T M2 C/4) e^{n+1} = (M1 - h^2 C^T M2 C/4) e^n + h C^T M2 b^n,
 * b^{n+1} = b^n - h C (e^n + e^{n+1})/2. */
void orc2_substep_IV(const orc2_cfg *c, double h, double *e, double *bz)
{
    long N = nodes(c), N2 = 2 * N;
    double *rhs = malloc(sizeof(double) * N2), *t = malloc(sizeof(double) * N2), *en = malloc(sizeof(double) * N2),
           *mb = malloc(sizeof(double) * N), *cb = malloc(sizeof(double) * N);
    op_M1C(c, -0.25 * h * h, e, rhs);
    orc2_apply_M2(c, bz, mb);
    orc2_apply_CT(c, mb, t);
    for (long i = 0; i < N2; ++i) rhs[i] += h * t[i];
    solve2(c, op_M1C, 0.25 * h * h, N2, 0, rhs, en);
    for (long i = 0; i < N2; ++i) t[i] = 0.5 * (e[i] + en[i]);
    orc2_apply_C(c, t, cb);
    for (long i = 0; i < N; ++i) bz[i] -= h * cb[i];
    memcpy(e, en, sizeof(double) * N2);
    free(rhs); free(t); free(en); free(mb); free(cb);
}

/* ------------------------------------------------------------------ */
/* Spin terms (hbar != 0): Zeeman energy and the four substeps.         */
/* ------------------------------------------------------------------ */

/* B_h(x) = (dA_z/dx2, -dA_z/dx1, B_z) from ga = G a_z and b_z. */
void orc2_bfield(const orc2_cfg *c, const double *ga, const double *bz, double x1, double x2, double *B)
{
    long N = nodes(c);
    int p = c->p;
    B[0] = orc2_eval(c, ga + N, p, p - 1, x1, x2);
    B[1] = -orc2_eval(c, ga, p - 1, p, x1, x2);
    B[2] = orc2_eval(c, bz, p - 1, p - 1, x1, x2);
}

/* The Hamiltonian with the Zeeman term: out = {kinetic, 1/2 e^T M1 e, 1/2 b^T M2 b,
 * 1/2 e_z^T M0 e_z, 1/2 a^T K a, hbar sum_a w s_a . B_h(x_a), total}. */
void orc2_energy_s(const orc2_cfg *c, double hbar, const double *x1, const double *x2, const double *p1,
                   const double *p2, const double *sx, const double *sy, const double *sz, const double *e,
                   const double *bz, const double *ez, const double *az, double *out)
{
    long N = nodes(c);
    orc2_energy(c, x1, x2, p1, p2, e, bz, ez, az, out);
    double *ga = malloc(sizeof(double) * 2 * N);
    orc2_apply_G(c, az, ga);
    double zee = 0.0;
    for (int64_t a = 0; a < c->n; ++a) {
        double B[3];
        orc2_bfield(c, ga, bz, x1[a], x2[a], B);
        zee += c->w * (sx[a] * B[0] + sy[a] * B[1] + sz[a] * B[2]);
    }
    free(ga);
    out[6] = out[5] + hbar * zee;
    out[5] = hbar * zee;
}

/* Derivative coefficients of the fields in B_h (backward differences, any degree):
 * gg2 = G (G a)_2 (d/dx1, d/dx2 of dA_z/dx2), gg1 = G (G a)_1, gb = G b_z. */
typedef struct {
    double hbar;
    const double *sx, *sy, *sz;
    double *gg1, *gg2, *gb;
} orc2_spin;

static void spin_derivs(const orc2_cfg *c, const double *ga, const double *bz, orc2_spin *sp)
{
    long N = nodes(c);
    sp->gg1 = malloc(sizeof(double) * 2 * N);
    sp->gg2 = malloc(sizeof(double) * 2 * N);
    sp->gb = malloc(sizeof(double) * 2 * N);
    orc2_apply_G(c, ga, sp->gg1);
    orc2_apply_G(c, ga + N, sp->gg2);
    orc2_apply_G(c, bz, sp->gb);
}

static void spin_free(orc2_spin *sp) { free(sp->gg1); free(sp->gg2); free(sp->gb); }

/* The spin part of (1/w) times the discrete gradient of H in x for particle a with
 * increment d, divided by hbar:
 *   s_x DD(dA_z/dx2) - s_y DD(dA_z/dx1) + s_z DD(B_z),
 * DD(F) = (mean of dF/dx1 along (x1, x2 + d2) -> (x1 + d1, x2 + d2),
 *          mean of dF/dx2 along (x1, x2) -> (x1, x2 + d2)). */
static void spin_force(const orc2_cfg *c, const orc2_spin *sp, int64_t a, double x1, double x2, double d1,
                       double d2, double *F)
{
    long N = nodes(c);
    int p = c->p;
    double b1 = x1 + d1, b2 = x2 + d2;
    /* dA_z/dx2 on (p, p-1): d/dx1 on (p-1, p-1), d/dx2 on (p, p-2) */
    double Dy1 = orc2_line_mean(c, sp->gg2, p - 1, p - 1, x1, b2, b1, b2);
    double Dy2 = orc2_line_mean(c, sp->gg2 + N, p, p - 2, x1, x2, x1, b2);
    /* dA_z/dx1 on (p-1, p): d/dx1 on (p-2, p), d/dx2 on (p-1, p-1) */
    double Dx1 = orc2_line_mean(c, sp->gg1, p - 2, p, x1, b2, b1, b2);
    double Dx2 = orc2_line_mean(c, sp->gg1 + N, p - 1, p - 1, x1, x2, x1, b2);
    /* B_z on (p-1, p-1): d/dx1 on (p-2, p-1), d/dx2 on (p-1, p-2) */
    double Db1 = orc2_line_mean(c, sp->gb, p - 2, p - 1, x1, b2, b1, b2);
    double Db2 = orc2_line_mean(c, sp->gb + N, p - 1, p - 2, x1, x2, x1, b2);
    F[0] = sp->sx[a] * Dy1 - sp->sy[a] * Dx1 + sp->sz[a] * Db1;
    F[1] = sp->sx[a] * Dy2 - sp->sy[a] * Dx2 + sp->sz[a] * Db2;
}

/* Subsystem I with spin: the map of orc2_particle_map with the momentum update
 * p^{n+1} = p^n + dt (Ebar + F - hbar spin_force). */
static void particle_map_s(const orc2_cfg *c, const orc2_spin *sp, int64_t a, double x1, double x2, double p1,
                           double p2, double d1, double d2, const double *ebar, const double *az, const double *ga,
                           double *pn, double *dn)
{
    long N = nodes(c);
    int p = c->p;
    double b1 = x1 + d1, b2 = x2 + d2;
    double E1 = orc2_line_mean(c, ebar, p - 1, p, x1, x2, b1, b2);
    double E2 = orc2_line_mean(c, ebar + N, p, p - 1, x1, x2, b1, b2);
    double Aa = orc2_eval(c, az, p, p, x1, x2), Ab = orc2_eval(c, az, p, p, b1, b2);
    double D2 = orc2_line_mean(c, ga + N, p, p - 1, x1, x2, x1, b2);
    double D1 = orc2_line_mean(c, ga, p - 1, p, x1, b2, b1, b2);
    double Fs[2];
    spin_force(c, sp, a, x1, x2, d1, d2, Fs);
    double ga_ = gam(p1, p2, Aa), gb = gam(p1, p2, Ab);
    double f = -(Aa + Ab) / (ga_ + gb);
    double q1 = p1 + c->dt * (E1 + f * D1 - sp->hbar * Fs[0]);
    double q2 = p2 + c->dt * (E2 + f * D2 - sp->hbar * Fs[1]);
    double gc = gam(q1, q2, Ab);
    pn[0] = q1;
    pn[1] = q2;
    dn[0] = c->dt * (p1 + q1) / (gb + gc);
    dn[1] = c->dt * (p2 + q2) / (gb + gc);
}

/* One evaluation of the Subsystem I map with spin for particle a (tests). */
void orc2_particle_map_s(const orc2_cfg *c, double hbar, const double *sx, const double *sy, const double *sz,
                         int64_t a, double x1, double x2, double p1, double p2, double d1, double d2,
                         const double *ebar, const double *az, const double *bz, double *pn, double *dn)
{
    long N = nodes(c);
    double *ga = malloc(sizeof(double) * 2 * N);
    orc2_apply_G(c, az, ga);
    orc2_spin sp = {hbar, sx, sy, sz, NULL, NULL, NULL};
    spin_derivs(c, ga, bz, &sp);
    particle_map_s(c, &sp, a, x1, x2, p1, p2, d1, d2, ebar, az, ga, pn, dn);
    spin_free(&sp);
    free(ga);
}

int orc2_substep_I_s(const orc2_cfg *cfg, double h, double hbar, double *x1, double *x2, double *p1, double *p2,
                     const double *sx, const double *sy, const double *sz, double *e, const double *az,
                     const double *bz, int32_t *sweeps, double *res)
{
    orc2_cfg ch = *cfg;
    ch.dt = h;
    const orc2_cfg *c = &ch;
    long N = nodes(c), N2 = 2 * N;
    int64_t n = c->n;
    int p = c->p;
    double *d = malloc(sizeof(double) * 2 * n), *dn = malloc(sizeof(double) * 2 * n),
           *pk = malloc(sizeof(double) * 2 * n);
    double *ek = malloc(sizeof(double) * N2), *enew = malloc(sizeof(double) * N2),
           *ebar = malloc(sizeof(double) * N2), *J = malloc(sizeof(double) * N2),
           *MJ = malloc(sizeof(double) * N2), *ga = malloc(sizeof(double) * N2);
    if (!d || !dn || !pk || !ek || !enew || !ebar || !J || !MJ || !ga) return ORC2_ENOMEM;
    orc2_apply_G(c, az, ga);
    orc2_spin sp = {hbar, sx, sy, sz, NULL, NULL, NULL};
    spin_derivs(c, ga, bz, &sp);
    for (int64_t a = 0; a < n; ++a) {
        double g = gam(p1[a], p2[a], orc2_eval(c, az, p, p, x1[a], x2[a]));
        d[2 * a] = c->dt * p1[a] / g;
        d[2 * a + 1] = c->dt * p2[a] / g;
    }
    memcpy(ek, e, sizeof(double) * N2);
    int status = ORC2_ENOTCONV, k;
    double r = 0.0;
    for (k = 0; k < c->kmax; ++k) {
        for (long i = 0; i < N2; ++i) ebar[i] = 0.5 * (e[i] + ek[i]);
        memset(J, 0, sizeof(double) * N2);
        double rx = 0.0;
        for (int64_t a = 0; a < n; ++a) {
            particle_map_s(c, &sp, a, x1[a], x2[a], p1[a], p2[a], d[2 * a], d[2 * a + 1], ebar, az, ga, &pk[2 * a],
                           &dn[2 * a]);
            double b1 = x1[a] + d[2 * a], b2 = x2[a] + d[2 * a + 1];
            orc2_line_deposit(c, J, p - 1, p, x1[a], x2[a], b1, b2, c->w * d[2 * a]);
            orc2_line_deposit(c, J + N, p, p - 1, x1[a], x2[a], b1, b2, c->w * d[2 * a + 1]);
            for (int q = 0; q < 2; ++q) {
                double dd = fabs(dn[2 * a + q] - d[2 * a + q]);
                if (dd > rx) rx = dd;
            }
        }
        orc2_solve_M1(c, J, MJ);
        double re = 0.0;
        for (long i = 0; i < N2; ++i) {
            enew[i] = e[i] - MJ[i];
            double de = fabs(enew[i] - ek[i]);
            if (de > re) re = de;
        }
        r = rx > re ? rx : re;
        if (r <= c->tol) {
            for (int64_t a = 0; a < n; ++a) {
                x1[a] = wrapL(x1[a] + d[2 * a], c->L1);
                x2[a] = wrapL(x2[a] + d[2 * a + 1], c->L2);
                p1[a] = pk[2 * a];
                p2[a] = pk[2 * a + 1];
            }
            memcpy(e, enew, sizeof(double) * N2);
            status = ORC2_OK;
            ++k;
            break;
        }
        double *t = d; d = dn; dn = t;
        memcpy(ek, enew, sizeof(double) * N2);
    }
    if (sweeps) *sweeps = k;
    if (res) *res = r;
    spin_free(&sp);
    free(d); free(dn); free(pk); free(ek); free(enew); free(ebar); free(J); free(MJ); free(ga);
    return status;
}

/* Subsystem II with spin: p as without spin; ds/dt = s x B_h(x) with B_h fixed
 * turns s about k = B_h/|B_h| by the angle -|B_h| h:
 * s' = s cos(th) - (k x s) sin(th) + k (k . s)(1 - cos(th)), th = |B_h| h. */
void orc2_substep_II_s(const orc2_cfg *c, double h, const double *x1, const double *x2, double *p1, double *p2,
                       double *sx, double *sy, double *sz, const double *bz, const double *az)
{
    long N = nodes(c);
    double *ga = malloc(sizeof(double) * 2 * N);
    orc2_apply_G(c, az, ga);
    for (int64_t a = 0; a < c->n; ++a) {
        double B[3];
        orc2_bfield(c, ga, bz, x1[a], x2[a], B);
        double nb = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
        if (nb == 0.0) continue;
        double k0 = B[0] / nb, k1 = B[1] / nb, k2 = B[2] / nb, th = nb * h;
        double s0 = sx[a], s1 = sy[a], s2 = sz[a];
        double kx0 = k1 * s2 - k2 * s1, kx1 = k2 * s0 - k0 * s2, kx2 = k0 * s1 - k1 * s0;
        double ks = k0 * s0 + k1 * s1 + k2 * s2, cs = cos(th), sn = sin(th);
        sx[a] = s0 * cs - kx0 * sn + k0 * ks * (1.0 - cs);
        sy[a] = s1 * cs - kx1 * sn + k1 * ks * (1.0 - cs);
        sz[a] = s2 * cs - kx2 * sn + k2 * ks * (1.0 - cs);
    }
    free(ga);
    orc2_substep_II(c, h, x1, x2, p1, p2, bz, az);
}

/* The spin sources at the particles: sxy = G*^T (Lambda1*(X)^T W S_xy), i.e.
 * G2^T D_x - G1^T D_y with D_x = sum w s_x N^p N^{p-1}, D_y = sum w s_y N^{p-1} N^p;
 * dz = Lambda2(X)^T W S_z = sum w s_z N^{p-1} N^{p-1}. */
void orc2_spin_sources(const orc2_cfg *c, const double *x1, const double *x2, const double *sx, const double *sy,
                       const double *sz, double *sxy, double *dz)
{
    long N = nodes(c);
    int p = c->p;
    double *u = calloc((size_t)(2 * N), sizeof(double));
    if (dz) memset(dz, 0, sizeof(double) * N);
    for (int64_t a = 0; a < c->n; ++a) {
        if (sxy) {
            deposit_point(c, u, p - 1, p, x1[a], x2[a], -c->w * sy[a]);   /* slot of (G a)_1 */
            deposit_point(c, u + N, p, p - 1, x1[a], x2[a], c->w * sx[a]); /* slot of (G a)_2 */
        }
        if (dz) deposit_point(c, dz, p - 1, p - 1, x1[a], x2[a], c->w * sz[a]);
    }
    if (sxy) orc2_apply_GT(c, u, sxy);
    free(u);
}

/* Subsystem III with spin: the right-hand side of orc2_substep_III plus
 * hbar h G*^T Lambda1*(X^n)^T W S_xy^n. */
int orc2_substep_III_s(const orc2_cfg *cfg, double h, double hbar, const double *x1, const double *x2,
                       const double *p1, const double *p2, const double *sx, const double *sy, double *ez,
                       double *az, int32_t *iters, double *res)
{
    orc2_cfg ch = *cfg;
    ch.dt = h;
    const orc2_cfg *c = &ch;
    long N = nodes(c);
    int64_t n = c->n;
    int p = c->p;
    double *An = malloc(sizeof(double) * n), *gn = malloc(sizeof(double) * n);
    double *rhs = malloc(sizeof(double) * N), *t = malloc(sizeof(double) * N), *ek = malloc(sizeof(double) * N),
           *ak = malloc(sizeof(double) * N), *S = malloc(sizeof(double) * N), *en = malloc(sizeof(double) * N),
           *src = malloc(sizeof(double) * N);
    for (int64_t a = 0; a < n; ++a) {
        An[a] = orc2_eval(c, az, p, p, x1[a], x2[a]);
        gn[a] = gam(p1[a], p2[a], An[a]);
    }
    orc2_spin_sources(c, x1, x2, sx, sy, NULL, src, NULL);
    op_M0K(c, -0.25 * h * h, ez, rhs);
    orc2_apply_K(c, az, t);
    for (long i = 0; i < N; ++i) rhs[i] += h * t[i] + hbar * h * src[i];
    memcpy(ek, ez, sizeof(double) * N);
    int status = ORC2_ENOTCONV, k;
    double r = 0.0;
    for (k = 0; k < c->kmax; ++k) {
        for (long i = 0; i < N; ++i) ak[i] = az[i] - 0.5 * h * (ez[i] + ek[i]);
        memset(S, 0, sizeof(double) * N);
        for (int64_t a = 0; a < n; ++a) {
            double Ak = orc2_eval(c, ak, p, p, x1[a], x2[a]);
            double q = c->w * (An[a] + Ak) / (gn[a] + gam(p1[a], p2[a], Ak));
            deposit_point(c, S, p, p, x1[a], x2[a], q);
        }
        for (long i = 0; i < N; ++i) S[i] = rhs[i] + h * S[i];
        solve2(c, op_M0K, 0.25 * h * h, N, 0, S, en);
        r = 0.0;
        for (long i = 0; i < N; ++i) {
            double de = fabs(en[i] - ek[i]);
            if (de > r) r = de;
        }
        memcpy(ek, en, sizeof(double) * N);
        if (r <= c->tol) {
            for (long i = 0; i < N; ++i) az[i] = az[i] - 0.5 * h * (ez[i] + en[i]);
            memcpy(ez, en, sizeof(double) * N);
            status = ORC2_OK;
            ++k;
            break;
        }
    }
    if (iters) *iters = k;
    if (res) *res = r;
    free(An); free(gn); free(rhs); free(t); free(ek); free(ak); free(S); free(en); free(src);
    return status;
}

/* Subsystem IV with spin: (M1 + h^2 C^T M2 C/4) e^{n+1} = (M1 - h^2 C^T M2 C/4) e^n
 * + h C^T M2 b^n + hbar h C^T Lambda2(X^n)^T W S_z^n, b^{n+1} = b^n - h C (e^n + e^{n+1})/2. */
void orc2_substep_IV_s(const orc2_cfg *c, double h, double hbar, const double *x1, const double *x2,
                       const double *sz, double *e, double *bz)
{
    long N = nodes(c), N2 = 2 * N;
    double *rhs = malloc(sizeof(double) * N2), *t = malloc(sizeof(double) * N2), *en = malloc(sizeof(double) * N2),
           *mb = malloc(sizeof(double) * N), *cb = malloc(sizeof(double) * N), *dz = malloc(sizeof(double) * N);
    orc2_spin_sources(c, x1, x2, NULL, NULL, sz, NULL, dz);
    op_M1C(c, -0.25 * h * h, e, rhs);
    orc2_apply_M2(c, bz, mb);
    for (long i = 0; i < N; ++i) mb[i] += hbar * dz[i];
    orc2_apply_CT(c, mb, t);
    for (long i = 0; i < N2; ++i) rhs[i] += h * t[i];
    solve2(c, op_M1C, 0.25 * h * h, N2, 0, rhs, en);
    for (long i = 0; i < N2; ++i) t[i] = 0.5 * (e[i] + en[i]);
    orc2_apply_C(c, t, cb);
    for (long i = 0; i < N; ++i) bz[i] -= h * cb[i];
    memcpy(e, en, sizeof(double) * N2);
    free(rhs); free(t); free(en); free(mb); free(cb); free(dz);
}

/* Lie-Trotter step with spin: I, II, III, IV over dt each. */
int orc2_step_s(const orc2_cfg *c, double hbar, int32_t nsteps, double *x1, double *x2, double *p1, double *p2,
                double *sx, double *sy, double *sz, double *e, double *bz, double *ez, double *az,
                int32_t *sweeps_I, int32_t *iters_III)
{
    for (int32_t s = 0; s < nsteps; ++s) {
        int st = orc2_substep_I_s(c, c->dt, hbar, x1, x2, p1, p2, sx, sy, sz, e, az, bz,
                                  sweeps_I ? &sweeps_I[s] : NULL, NULL);
        if (st) return st;
        orc2_substep_II_s(c, c->dt, x1, x2, p1, p2, sx, sy, sz, bz, az);
        st = orc2_substep_III_s(c, c->dt, hbar, x1, x2, p1, p2, sx, sy, ez, az, iters_III ? &iters_III[s] : NULL,
                                NULL);
        if (st) return st;
        orc2_substep_IV_s(c, c->dt, hbar, x1, x2, sz, e, bz);
    }
    return ORC2_OK;
}

/* ------------------------------------------------------------------ */
/* Lie-Trotter step: I, II, III, IV over dt each.                        */
/* ------------------------------------------------------------------ */
int orc2_step(const orc2_cfg *c, int32_t nsteps, double *x1, double *x2, double *p1, double *p2, double *e,
              double *bz, double *ez, double *az, int32_t *sweeps_I, int32_t *iters_III)
{
    for (int32_t s = 0; s < nsteps; ++s) {
        int st = orc2_substep_I(c, c->dt, x1, x2, p1, p2, e, az, sweeps_I ? &sweeps_I[s] : NULL, NULL);
        if (st) return st;
        orc2_substep_II(c, c->dt, x1, x2, p1, p2, bz, az);
        st = orc2_substep_III(c, c->dt, x1, x2, p1, p2, ez, az, iters_III ? &iters_III[s] : NULL, NULL);
        if (st) return st;
        orc2_substep_IV(c, c->dt, e, bz);
    }
    return ORC2_OK;
}
