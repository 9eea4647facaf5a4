// Deterministic FP64 reductions over the moment planes of one instance (the integral
// diagnostics of lbm_reduce): per-block partials, then one block folds them in a fixed
// order, so the result does not depend on timing.
#include "lbm_device.h"

#include <math.h>

namespace lbm {

// ------------------------------------------------------------------ reductions
// Per-block partials over the FP64 moment planes of one instance, then one block folds
// the partials in a fixed order: the result does not depend on timing.
constexpr int NRED = REDUCE_SLOTS;
enum {
    R_SPHI, R_SRHO, R_KIN, R_MAXU2, R_MINRHO, R_MINPHI, R_MAXPHI, R_PIN_S, R_PIN_N, R_POUT_S,
    R_POUT_N, R_CROSS, R_NONFIN
};

__device__ __forceinline__ void red_init(double (&a)[NRED]) {
#pragma unroll
    for (int k = 0; k < NRED; ++k) a[k] = 0.0;
    a[R_MINRHO] = INFINITY;
    a[R_MINPHI] = INFINITY;
    a[R_MAXPHI] = -INFINITY;
}

__device__ __forceinline__ void red_join(double (&a)[NRED], const double* b) {
    a[R_SPHI] += b[R_SPHI];
    a[R_SRHO] += b[R_SRHO];
    a[R_KIN] += b[R_KIN];
    a[R_MAXU2] = fmax(a[R_MAXU2], b[R_MAXU2]);
    a[R_MINRHO] = fmin(a[R_MINRHO], b[R_MINRHO]);
    a[R_MINPHI] = fmin(a[R_MINPHI], b[R_MINPHI]);
    a[R_MAXPHI] = fmax(a[R_MAXPHI], b[R_MAXPHI]);
    a[R_PIN_S] += b[R_PIN_S];
    a[R_PIN_N] += b[R_PIN_N];
    a[R_POUT_S] += b[R_POUT_S];
    a[R_POUT_N] += b[R_POUT_N];
    a[R_CROSS] += b[R_CROSS];
    a[R_NONFIN] += b[R_NONFIN];
}

// Wavefront reduction: a fixed-shape tree over the 64 lanes with cross-lane shuffles
// (lane l takes lane l + s for s = 32, 16, ..., 1), then lane 0 of each of the block's 4
// wavefronts leaves its result in LDS and thread 0 folds the 4 in wavefront order.  The
// shape never depends on timing, so the result is deterministic.  Thread 0 ends with the
// block's result.
constexpr int WAVE = 64;
__device__ __forceinline__ void block_fold(double (&acc)[NRED], double* sh) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int s = WAVE / 2; s > 0; s >>= 1) {
        double other[NRED];
#pragma unroll
        for (int k = 0; k < NRED; ++k) other[k] = __shfl_down(acc[k], s, WAVE);
        red_join(acc, other);   // lanes >= 64 - s fold in values they do not use
    }
    const int wave = tid / WAVE;
    if ((tid & (WAVE - 1)) == 0) {
#pragma unroll
        for (int k = 0; k < NRED; ++k) sh[wave * NRED + k] = acc[k];
    }
    __syncthreads();
    if (tid == 0) {
        for (int wv = 1; wv < BLOCK / WAVE; ++wv) red_join(acc, sh + wv * NRED);
    }
}

__global__ __launch_bounds__(BLOCK) void k_reduce_partial(const double* __restrict__ mom, int nx,
                                                          int ny, int periodic_y, double xc,
                                                          double yc, double r_in, double r_out,
                                                          double* __restrict__ partials) {
    __shared__ double sh[NRED * (BLOCK / WAVE)];
    double acc[NRED];
    red_init(acc);
    const int64_t n = (int64_t)nx * ny;
    const double* phi = mom;
    const double* rho = mom + n;
    const double* p = mom + 2 * n;
    const double* ux = mom + 3 * n;
    const double* uy = mom + 4 * n;
    for (int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * BLOCK) {
        const int y = (int)(c / nx), x = (int)(c - (int64_t)y * nx);
        const double ph = phi[c], r = rho[c], pr = p[c], u = ux[c], v = uy[c];
        const bool fin = isfinite(ph) && isfinite(r) && isfinite(pr) && isfinite(u) && isfinite(v);
        if (!fin) {
            acc[R_NONFIN] += 1.0;
            continue;
        }
        const double u2 = u * u + v * v;
        acc[R_SPHI] += ph;
        acc[R_SRHO] += r;
        acc[R_KIN] += 0.5 * r * u2;
        acc[R_MAXU2] = fmax(acc[R_MAXU2], u2);
        acc[R_MINRHO] = fmin(acc[R_MINRHO], r);
        acc[R_MINPHI] = fmin(acc[R_MINPHI], ph);
        acc[R_MAXPHI] = fmax(acc[R_MAXPHI], ph);
        double dx = fabs(x + 0.5 - xc);
        dx = fmin(dx, nx - dx);
        double dy = fabs(y + 0.5 - yc);
        if (periodic_y) dy = fmin(dy, ny - dy);
        const double d = sqrt(dx * dx + dy * dy);
        if (d < r_in) {
            acc[R_PIN_S] += pr;
            acc[R_PIN_N] += 1.0;
        }
        if (d > r_out) {
            acc[R_POUT_S] += pr;
            acc[R_POUT_N] += 1.0;
        }
        // crossings of phi = 0.5 with the right neighbour (periodic) and the upper one
        const bool liq = ph >= 0.5;
        const int xr = x + 1 == nx ? 0 : x + 1;
        if ((phi[(int64_t)y * nx + xr] >= 0.5) != liq) acc[R_CROSS] += 1.0;
        if (y + 1 < ny || periodic_y) {
            const int yu = y + 1 == ny ? 0 : y + 1;
            if ((phi[(int64_t)yu * nx + x] >= 0.5) != liq) acc[R_CROSS] += 1.0;
        }
    }
    block_fold(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NRED; ++k) partials[(int64_t)blockIdx.x * NRED + k] = acc[k];
    }
}

// out = {sum_phi, sum_rho, kinetic, max_u, min_rho, min_phi, max_phi, p_in, p_out,
//        crossings, spread_radius, nonfinite}
__global__ __launch_bounds__(BLOCK) void k_reduce_final(const double* __restrict__ partials,
                                                        int nblocks,
                                                        const double* __restrict__ mom, int nx,
                                                        int ny, double xc, int y_row,
                                                        double* __restrict__ out) {
    __shared__ double sh[NRED * (BLOCK / WAVE)];
    double acc[NRED];
    red_init(acc);
    for (int b = threadIdx.x; b < nblocks; b += BLOCK) red_join(acc, partials + (int64_t)b * NRED);
    block_fold(acc, sh);
    // spreading radius on row y_row (interpolated crossings between x and x + 1)
    __shared__ double rmax[BLOCK];
    double best = 0.0;
    if (y_row >= 0 && y_row < ny) {
        const double* row = mom + (int64_t)y_row * nx;
        for (int x = threadIdx.x; x < nx - 1; x += BLOCK) {
            const double a = row[x] - 0.5, b = row[x + 1] - 0.5;
            if ((a >= 0.0) != (b >= 0.0)) {
                const double xs = x + 0.5 + a / (a - b);
                best = fmax(best, fabs(xs - xc));
            }
        }
    }
    rmax[threadIdx.x] = best;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = acc[R_SPHI];
        out[1] = acc[R_SRHO];
        out[2] = acc[R_KIN];
        out[3] = sqrt(acc[R_MAXU2]);
        out[4] = acc[R_MINRHO];
        out[5] = acc[R_MINPHI];
        out[6] = acc[R_MAXPHI];
        out[7] = acc[R_PIN_N] > 0 ? acc[R_PIN_S] / acc[R_PIN_N] : 0.0;
        out[8] = acc[R_POUT_N] > 0 ? acc[R_POUT_S] / acc[R_POUT_N] : 0.0;
        out[9] = acc[R_CROSS];
        out[10] = rmax[0];
        out[11] = acc[R_NONFIN];
    }
}

int reduce_blocks(int64_t n) {
    int64_t b = (n + BLOCK - 1) / BLOCK;
    return (int)(b < REDUCE_MAX_BLOCKS ? (b < 1 ? 1 : b) : REDUCE_MAX_BLOCKS);
}

hipError_t launch_reduce(const double* mom, int nx, int ny, int periodic_y, const double* mask,
                         double* partials, double* out, hipStream_t st) {
    const int nb = reduce_blocks((int64_t)nx * ny);
    k_reduce_partial<<<nb, BLOCK, 0, st>>>(mom, nx, ny, periodic_y, mask[0], mask[1], mask[2],
                                           mask[3], partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_reduce_final<<<1, BLOCK, 0, st>>>(partials, nb, mom, nx, ny, mask[0],
                                        mask[4] < 0 ? -1 : (int)mask[4], out);
    return hipGetLastError();
}

}  // namespace lbm
