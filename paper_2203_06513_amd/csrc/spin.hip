// The spin terms of the reduced model (hbar != 0; Sections 2.1 and 4.2).
//
// The Zeeman energy of the discrete Hamiltonian,
//     hbar sum_a w (s_y dA_z/dx - s_z dA_y/dx)(x_a),
// couples the spins to the particles and to the transverse potential:
// * Subsystem I: the force of that energy (in the sweep and the commit,
//   sub1.hip, compiled with SPIN);
// * Subsystem II: the constant source -hbar G^T Lambda1(X)^T W S_z (e_y) and
//   +hbar G^T Lambda1(X)^T W S_y (e_z), added to the right-hand side once per
//   substep (here: a deposit pass, the G^T stencil, and the (M0 + dt^2 K/4)
//   inverse of that source added to the iteration's constant part E0);
// * Subsystem III: every spin turns about r = (0, dA_z/dx, -dA_y/dx) by the
//   exact rotation of eq. spin_rodrigue (one pass);
// * the Zeeman part of the energy diagnostic.
//
// dA/dx at a particle of cell c with local coordinate t: the V1 expansion
// sum_j (G a)_j Lambda1_j(x), (G a)_j = (a_j - a_{j-1})/dx, over the P splines
// Lambda1_{c-m}(x) = B_{P-1}(t + m), m = 0..P-1, alive on the cell.  A block
// owns one work item (one cell), so it forms the P differences once.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "spline.hpp"

namespace ecpic {

// The block's item, its cell and the P values (G a)_{c-m}, m = 0..P-1, of both
// components.
template <int P>
struct CellDiff {
    int c, beg, end;
    double gy[P], gz[P];
};

template <int P>
__device__ __forceinline__ bool cell_diff(const SpinArgs &a, int item, int M, CellDiff<P> &d) {
    if (item >= a.items.n_items[0]) return false;
    d.c = a.items.cell[item];
    d.beg = a.items.begin[item];
    d.end = a.items.begin[item + 1];
    const double *ay = a.ay + HALO, *az = a.az + HALO;   // padded: indices -HALO .. M+HALO-1
#pragma unroll
    for (int m = 0; m < P; ++m) {
        const int j = d.c - m;   // >= -P, and j - 1 >= -P - 1 > -HALO
        d.gy[m] = (ay[j] - ay[j - 1]) * a.inv_dx;
        d.gz[m] = (az[j] - az[j - 1]) * a.inv_dx;
    }
    return true;
}

// dA_y/dx and dA_z/dx at local coordinate t of the cell.
template <int P>
__device__ __forceinline__ void dadx(const CellDiff<P> &d, double t, double &Y, double &Z) {
    double B[P];
    basis_values<P - 1, double>(t, B);
    Y = 0.0;
    Z = 0.0;
#pragma unroll
    for (int m = 0; m < P; ++m) {
        Y = fma(d.gy[m], B[m], Y);
        Z = fma(d.gz[m], B[m], Z);
    }
}

__device__ __forceinline__ double local_t(double xi, int c) { return fmin(fmax(xi - (double)c, 0.0), 1.0); }

// Subsystem III over h: s <- exp(h rhat) s, rhat s = r x s, r = (0, Z, -Y), by
// Rodrigues' formula s + c1 (r x s) + c2 r x (r x s) with c1 = sin(h|r|)/|r| and
// c2 = 2 sin^2(h|r|/2)/|r|^2 (the limits h and h^2/2 at r = 0).
template <int P>
__global__ void __launch_bounds__(256) k_spin_rotate(SpinArgs a, int M) {
    CellDiff<P> d;
    if (!cell_diff<P>(a, blockIdx.x, M, d)) return;
#pragma unroll 2
    for (int i = d.beg + (int)threadIdx.x; i < d.end; i += blockDim.x) {
        const double t = local_t(a.xi[i], d.c);
        double Y, Z;
        dadx<P>(d, t, Y, Z);
        const double sx = a.sx[i], sy = a.sy[i], sz = a.sz[i];
        const double nr2 = fma(Y, Y, Z * Z);
        double c1 = a.h, c2 = 0.5 * a.h * a.h;
        if (nr2 > 0.0) {   // sin(h|r|) = 2 sin(h|r|/2) cos(h|r|/2): one sincos
            const double nr = sqrt(nr2);
            double sh, ch;
            sincos(0.5 * a.h * nr, &sh, &ch);
            c1 = 2.0 * sh * ch / nr;
            c2 = 2.0 * sh * sh / nr2;
        }
        // u = rhat s, v = rhat u (rhat = [[0, Y, Z], [-Y, 0, 0], [-Z, 0, 0]])
        const double ux = fma(Y, sy, Z * sz), uy = -Y * sx, uz = -Z * sx;
        const double vx = fma(Y, uy, Z * uz), vy = -Y * ux, vz = -Z * ux;
        a.sx[i] = fma(c2, vx, fma(c1, ux, sx));
        a.sy[i] = fma(c2, vy, fma(c1, uy, sy));
        a.sz[i] = fma(c2, vz, fma(c1, uz, sz));
    }
}

// Per item: sum over its particles of s_y B_{P-1}(t + m) and s_z B_{P-1}(t + m),
// m = 0..P-1 (the item's share of Lambda1(X)^T S_y, S_z on V1 indices c - m),
// in a fixed order (lanes, then waves).
template <int P>
__global__ void __launch_bounds__(256) k_spin_deposit(SpinArgs a, int M) {
    __shared__ double lds[MAX_WAVES][2 * P];
    CellDiff<P> d;
    if (!cell_diff<P>(a, blockIdx.x, M, d)) return;
    double vy[P], vz[P];
#pragma unroll
    for (int m = 0; m < P; ++m) { vy[m] = 0.0; vz[m] = 0.0; }
#pragma unroll 4
    for (int i = d.beg + (int)threadIdx.x; i < d.end; i += blockDim.x) {
        double B[P];
        basis_values<P - 1, double>(local_t(a.xi[i], d.c), B);
        const double sy = a.sy[i], sz = a.sz[i];
#pragma unroll
        for (int m = 0; m < P; ++m) {
            vy[m] = fma(sy, B[m], vy[m]);
            vz[m] = fma(sz, B[m], vz[m]);
        }
    }
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
#pragma unroll
    for (int m = 0; m < P; ++m) {
        const double ty = wave_sum_dpp(vy[m]), tz = wave_sum_dpp(vz[m]);
        if (lane == 0) { lds[wid][m] = ty; lds[wid][P + m] = tz; }
    }
    __syncthreads();
    if (threadIdx.x < 2 * P) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) t += lds[w][threadIdx.x];
        a.spart[(size_t)blockIdx.x * 2 * P + threadIdx.x] = t;
    }
}

// The source of Subsystem II, times dt, added to the iteration's constant part
// E0 through the matrix inverse (E0 += taps * b, the taps of (M0 + dt^2 K/4)
// scaled by dx), one block per 256 outputs with its window of u and b in LDS:
//   u_k = w sum over items of cells c = k .. k+P-1 of their (V1 index c - m = k) sums,
//   b_y,k = -hbar dt (u^z_k - u^z_{k+1}) / dx,   b_z,k = +hbar dt (u^y_k - u^y_{k+1}) / dx
// (coef = hbar dt w / dx^2 takes the w, the 1/dx of G^T and that of the taps).
template <int P>
__global__ void __launch_bounds__(256) k_spin_source(const double *spart, ItemList items, int M, double coef,
                                                     const double *taps, int ntaps, int mlo, double *E0y,
                                                     double *E0z) {
    extern __shared__ double sh[];
    const int len = blockDim.x + ntaps - 1;            // b indices lo .. lo + len - 1
    const int j0 = blockIdx.x * blockDim.x;
    const int lo = j0 - mlo - (ntaps - 1);
    double *uy = sh, *uz = uy + (len + 1), *by = uz + (len + 1), *bz = by + len;
    const int one_each = items.n_items[1];
    for (int q = threadIdx.x; q < len + 1; q += blockDim.x) {
        double vy = 0.0, vz = 0.0;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int c = imod(lo + q + m, M);
            const int i0 = one_each ? c : items.cell_first[c];
            const int i1 = one_each ? c + 1 : items.cell_first[c + 1];
            for (int it = i0; it < i1; ++it) {
                vy += spart[(size_t)it * 2 * P + m];
                vz += spart[(size_t)it * 2 * P + P + m];
            }
        }
        uy[q] = vy;
        uz[q] = vz;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < len; q += blockDim.x) {
        by[q] = -coef * (uz[q] - uz[q + 1]);
        bz[q] = coef * (uy[q] - uy[q + 1]);
    }
    __syncthreads();
    const int j = j0 + threadIdx.x;
    if (j >= M) return;
    double sy = 0.0, sz = 0.0;
    for (int i = 0; i < ntaps; ++i) {   // b index j - mlo - i, at q = threadIdx.x + ntaps - 1 - i
        const int q = threadIdx.x + ntaps - 1 - i;
        sy = fma(taps[i], by[q], sy);
        sz = fma(taps[i], bz[q], sz);
    }
    E0y[j] += sy;
    E0z[j] += sz;
}

// Per item: sum over its particles of s_y dA_z/dx - s_z dA_y/dx (the Zeeman
// energy without hbar w), lanes then waves in a fixed order.
template <int P>
__global__ void __launch_bounds__(256) k_spin_energy(SpinArgs a, int M) {
    __shared__ double lds[MAX_WAVES];
    CellDiff<P> d;
    if (!cell_diff<P>(a, blockIdx.x, M, d)) return;
    double e = 0.0;
    for (int i = d.beg + (int)threadIdx.x; i < d.end; i += blockDim.x) {
        double Y, Z;
        dadx<P>(d, local_t(a.xi[i], d.c), Y, Z);
        e = fma(a.sy[i], Z, fma(-a.sz[i], Y, e));
    }
    const double t = wave_sum_dpp(e);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    if (lane == 0) lds[wid] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) s += lds[w];
        a.epart[blockIdx.x] = s;
    }
}

// Spins of a new particle order from arrays indexed by particle id, and back.
__global__ void __launch_bounds__(256) k_spin_in(const double *ix, const double *iy, const double *iz,
                                                 const int32_t *id, int64_t n, double *sx, double *sy, double *sz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t k = id[i];
    sx[i] = ix[k];
    sy[i] = iy[k];
    sz[i] = iz[k];
}

__global__ void __launch_bounds__(256) k_spin_out(const double *sx, const double *sy, const double *sz,
                                                  const int32_t *id, int64_t n, double *ox, double *oy, double *oz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t k = id[i];
    ox[k] = sx[i];
    oy[k] = sy[i];
    oz[k] = sz[i];
}

// ---- launchers ------------------------------------------------------------
#define ECPIC_SPIN_P(K, ...)                                                        \
    switch (P) {                                                                    \
        case 2: launch_k((K<2>), __VA_ARGS__); break;                               \
        case 3: launch_k((K<3>), __VA_ARGS__); break;                               \
        case 4: launch_k((K<4>), __VA_ARGS__); break;                               \
        case 5: launch_k((K<5>), __VA_ARGS__); break;                               \
    }

void launch_spin_rotate(int P, int grid, hipStream_t s, const SpinArgs &a, int M) {
    ECPIC_SPIN_P(k_spin_rotate, dim3(grid), dim3(256), 0, s, a, M)
}

void launch_spin_deposit(int P, int grid, hipStream_t s, const SpinArgs &a, int M) {
    ECPIC_SPIN_P(k_spin_deposit, dim3(grid), dim3(256), 0, s, a, M)
}

void launch_spin_source(int P, hipStream_t s, const double *spart, const ItemList &items, int M, double coef,
                        const double *taps, int ntaps, int mlo, double *E0y, double *E0z) {
    const size_t lds = sizeof(double) * (4 * (size_t)(256 + ntaps - 1) + 2);
    ECPIC_SPIN_P(k_spin_source, dim3((M + 255) / 256), dim3(256), lds, s, spart, items, M, coef, taps, ntaps, mlo,
                 E0y, E0z)
}

void launch_spin_energy(int P, int grid, hipStream_t s, const SpinArgs &a, int M) {
    ECPIC_SPIN_P(k_spin_energy, dim3(grid), dim3(256), 0, s, a, M)
}

void launch_spin_in(hipStream_t s, const double *ix, const double *iy, const double *iz, const int32_t *id,
                    int64_t n, double *sx, double *sy, double *sz) {
    if (n > 0)
        launch_k(k_spin_in, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ix, iy, iz, id, n, sx, sy, sz);
}

void launch_spin_out(hipStream_t s, const double *sx, const double *sy, const double *sz, const int32_t *id,
                     int64_t n, double *ox, double *oy, double *oz) {
    if (n > 0)
        launch_k(k_spin_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sx, sy, sz, id, n, ox, oy, oz);
}

}  // namespace ecpic
