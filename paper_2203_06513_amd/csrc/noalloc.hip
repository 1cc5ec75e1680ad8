// Current of straight segments for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc): the segment integrals of ecpic_deposit_current, with the
// per-block partial currents in a fixed file-scope device array instead of
// buffers the call allocates, and the call asynchronous on the context's stream.
//
// Layout of `scratch` (one copy per device, held until the process ends):
//   [NOALLOC_BLOCKS][NOALLOC_MAX_M]  partial current of each block (doubles)
//   [NOALLOC_BLOCKS]                 flag word of each block (one int per double slot)
// Every call on a device shares that device's copy; calls that overlap on one
// device race.  Each call clears what it reads: a block zeroes its partial
// before accumulating and writes its flag word.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/ecpic.h"
#include "common.hpp"
#include "spline.hpp"

namespace ecpic {

constexpr int NOALLOC_MAX_M = 16384;   // cells the partials have room for
constexpr int NOALLOC_BLOCKS = 64;     // blocks of the partial pass (one partial each)

static __device__ __align__(256) double scratch[NOALLOC_BLOCKS * NOALLOC_MAX_M + NOALLOC_BLOCKS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_scratch[MAX_DEVICES] = {};   // device address of `scratch` on each device
}  // namespace

int noalloc_max_cells() { return NOALLOC_MAX_M; }

// Device address of this device's `scratch`, taken once per device with that
// device current (ecpic_create calls it).  The array's name in host code is a
// host-side stand-in; only this address may be handed to kernels.
int noalloc_init(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return ECPIC_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[dev]) return ECPIC_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        std::fprintf(stderr, "ecpic: hipGetSymbolAddress of the deposit scratch failed on device %d: %s\n", dev,
                     hipGetErrorString(e));
        return ECPIC_EDEVICE;
    }
    g_scratch[dev] = static_cast<double *>(ptr);
    return ECPIC_OK;
}

double *noalloc_scratch(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_scratch[dev];
}

// Block b zeroes its partial, then adds w dx int Lambda1_j along segments
// b*256 + t, b*256 + t + G*256, ... (G blocks); a segment whose end leaves the
// neighbour cells of its start is skipped and flagged.
template <int P>
__global__ void __launch_bounds__(256) k_deposit_partial(const double *x0, const double *x1, int64_t n,
                                                         double inv_dx, double dx, double w, int M, double *part,
                                                         int *bflags) {
    __shared__ int fl;
    double *mine = part + (size_t)blockIdx.x * M;
    for (int j = threadIdx.x; j < M; j += blockDim.x) mine[j] = 0.0;
    if (threadIdx.x == 0) fl = 0;
    __syncthreads();   // the zeros are in place before any addition
    int f = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xi0 = x0[i] * inv_dx;
        const double cf = floor(xi0);
        const double t0 = xi0 - cf;
        const double t1 = x1[i] * inv_dx - cf;
        if (!(t1 > -1.0 && t1 < 2.0) || !(fabs(cf) < 1.0e9)) {
            f |= FLAG_CFL;
            continue;
        }
        const int c = (int)cf;
        const int s = t1 >= 1.0 ? 1 : (t1 < 0.0 ? -1 : 0);
        double I[P + 2];
        segment_integrals<P>(t0, t1, s, I);
#pragma unroll
        for (int q = 0; q < P + 2; ++q) atomicAdd(&mine[imod(c - P + q, M)], w * dx * I[q]);
    }
    if (f) atomicOr(&fl, f);
    __syncthreads();
    if (threadIdx.x == 0) bflags[blockIdx.x] = fl;
}

// J_j = sum over the nb partials in block order; flags = OR of their flag words.
__global__ void __launch_bounds__(256) k_deposit_reduce(const double *part, const int *bflags, int nb, int M,
                                                        double *J, int32_t *flags) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < M) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[(size_t)b * M + j];
        J[j] = s;
    }
    if (flags && blockIdx.x == 0 && threadIdx.x == 0) {
        int f = 0;
        for (int b = 0; b < nb; ++b) f |= bflags[b];
        *flags = f;
    }
}

// scr: the device address from noalloc_scratch; M <= NOALLOC_MAX_M (checked by the caller).
void launch_deposit_noalloc(int P, hipStream_t s, const double *x0, const double *x1, int64_t n, double inv_dx,
                            double dx, double w, int M, double *scr, double *J, int32_t *flags) {
    const int64_t want = (n + 255) / 256;
    const int nb = (int)(want < 1 ? 1 : (want > NOALLOC_BLOCKS ? NOALLOC_BLOCKS : want));
    int *bflags = reinterpret_cast<int *>(scr + (size_t)NOALLOC_BLOCKS * NOALLOC_MAX_M);
#define CALL(PP) \
    launch_k((k_deposit_partial<PP>), dim3(nb), dim3(256), 0, s, x0, x1, n, inv_dx, dx, w, M, scr, bflags)
    ECPIC_DISPATCH(P, CALL)
#undef CALL
    launch_k(k_deposit_reduce, dim3((M + 255) / 256), dim3(256), 0, s, (const double *)scr, (const int *)bflags, nb,
             M, J, flags);
}

}  // namespace ecpic
