// HIP kernels (gfx950) of the phase-field lattice Boltzmann step of Liang et al.,
// arXiv:1710.09541: the conservative Allen-Cahn lattice f (Sec. 2.2) and the
// Navier-Stokes lattice g with the forcing distribution G_i (Sec. 2.3).
//
// State between steps (after the first): post-collision distributions in SoA planes
// [plane i][y][pitch], x fastest.  A step pulls f_i(x - c_i), g_i(x - c_i) (streaming with
// the boundary rules), recomputes phi on the tile and a one-node halo into LDS, evaluates
// the isotropic stencils (Eqs. 27-28), the local closure (Eqs. 2-3, 5-7, 13, 19, 23-26),
// the FP64 moments u then p (Eq. 22), the backward difference of phi u (Eq. 11), collides
// both lattices (Eqs. 8-9, 11, 15-17, 20) and writes the result at the node itself into the
// other buffer.  The very first step reads the initial (already streamed) distributions
// in place instead of pulling.
//
// Boundary rules in pull form (y only; x is periodic):
//   periodic   the source row wraps
//   wall       half-way bounce-back: a population that would come from across the wall is
//              the node's own outgoing opposite population, f_i(x) = f*_opp(i)(x)
//   open       zero gradient: an incoming population of the edge row equals the streamed
//              value of the row inside it, i.e. f*_i(x - c_ix, edge row)
// The stencil's ghost rows at walls and open sides mirror the edge row.
#include "lbm_device.h"

#include <math.h>

namespace lbm {

// ------------------------------------------------------------------ lattice (Eq. 10)
// i = 0 rest; 1..4 = (1,0), (0,1), (-1,0), (0,-1); 5..8 = (1,1), (-1,1), (-1,-1), (1,-1)
__device__ constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

template <typename C>
__device__ __forceinline__ C wgt(int i) {
    return i == 0 ? C(4.0 / 9.0) : (i < 5 ? C(1.0 / 9.0) : C(1.0 / 36.0));
}

// ------------------------------------------------------------------ storage codecs
template <typename S>
struct Store;
template <>
struct Store<double> {
    using C = double;
    static __device__ __forceinline__ double get(const double* p, int o) { return p[o]; }
    static __device__ __forceinline__ void put(double* p, int o, double v) { p[o] = v; }
};
template <>
struct Store<float> {
    using C = float;
    static __device__ __forceinline__ float get(const float* p, int o) { return p[o]; }
    static __device__ __forceinline__ void put(float* p, int o, float v) { p[o] = v; }
};
template <>
struct Store<_Float16> {
    using C = float;
    static __device__ __forceinline__ float get(const _Float16* p, int o) { return (float)p[o]; }
    static __device__ __forceinline__ void put(_Float16* p, int o, float v) { p[o] = (_Float16)v; }
};

// ------------------------------------------------------------------ streaming offsets
// Element offsets (relative to the instance's plane 0) of the 9 populations arriving at
// node (x, y).  PULL = false reads the node's own slots (the initial state is already in
// streamed form).
template <bool PULL>
__device__ __forceinline__ void pull_offsets(const InstDev& I, int x, int y, int o[9]) {
    const int pitch = I.pitch;
    const int plane = (int)I.plane;
    const int self = y * pitch + x;
    if (!PULL) {
#pragma unroll
        for (int i = 0; i < 9; ++i) o[i] = i * plane + self;
        return;
    }
    const int nx = I.nx, ny = I.ny;
    const int xm = x == 0 ? nx - 1 : x - 1;
    const int xp = x == nx - 1 ? 0 : x + 1;
    const bool at_lo = y == 0, at_hi = y == ny - 1;
    const int ym = at_lo ? (I.bc_lo == BC_PERIODIC ? ny - 1 : 0) : y - 1;
    const int yp = at_hi ? (I.bc_hi == BC_PERIODIC ? 0 : ny - 1) : y + 1;
    const bool bl = at_lo && I.bc_lo == BC_WALL;
    const bool bh = at_hi && I.bc_hi == BC_WALL;
    const int rc = y * pitch, rm = ym * pitch, rp = yp * pitch;
    o[0] = self;
    o[1] = plane + rc + xm;
    o[3] = 3 * plane + rc + xp;
    o[2] = bl ? 4 * plane + self : 2 * plane + rm + x;
    o[5] = bl ? 7 * plane + self : 5 * plane + rm + xm;
    o[6] = bl ? 8 * plane + self : 6 * plane + rm + xp;
    o[4] = bh ? 2 * plane + self : 4 * plane + rp + x;
    o[7] = bh ? 5 * plane + self : 7 * plane + rp + xp;
    o[8] = bh ? 6 * plane + self : 8 * plane + rp + xm;
}

// phi of the arriving f populations at (x, y): phi_ref + sum of the stored deviations
template <typename S, bool PULL>
__device__ __forceinline__ typename Store<S>::C pulled_phi(const InstDev& I, const S* fb, int x,
                                                           int y) {
    using C = typename Store<S>::C;
    int o[9];
    pull_offsets<PULL>(I, x, y, o);
    C v[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] = Store<S>::get(fb, o[i]);
    C s = v[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) s += v[i];
    return C(I.phi_ref) + s * C(I.inv_scale_f);
}

// row of the stencil's ghost node: wrap if periodic, else mirror the edge row
__device__ __forceinline__ int ghost_row(const InstDev& I, int y) {
    if (y < 0) return I.bc_lo == BC_PERIODIC ? y + I.ny : 0;
    if (y >= I.ny) return I.bc_hi == BC_PERIODIC ? y - I.ny : I.ny - 1;
    return y;
}

enum { MODE_STEP = 0, MODE_MOMENTS = 1 };

// ------------------------------------------------------------------ one node
// f: stored f deviations scaled back (f_i - w_i phi_ref), g: g_i, phi and its 8
// neighbours, q: phi u of the previous step (updated in place).  Writes the collided
// populations (same deviation form) into fo, go, or the moments into mom.
template <typename C, int MODE>
__device__ __forceinline__ void node_update(const InstDev& I, const C (&f)[9], const C (&g)[9],
                                            C phi, C pE, C pN, C pW, C pS, C pNE, C pNW,
                                            C pSW, C pSE, C& qx, C& qy, C (&fo)[9],
                                            C (&go)[9], double (&mom)[5]) {
    // isotropic gradient and Laplacian (Eqs. 27-28): weights over c_s^2
    const C dpx = C(3) * (C(1.0 / 9.0) * (pE - pW) + C(1.0 / 36.0) * ((pNE - pNW) + (pSE - pSW)));
    const C dpy = C(3) * (C(1.0 / 9.0) * (pN - pS) + C(1.0 / 36.0) * ((pNE + pNW) - (pSW + pSE)));
    const C lap = C(6) * (C(1.0 / 9.0) * ((pE + pW) + (pN + pS) - C(4) * phi) +
                          C(1.0 / 36.0) * ((pNE + pSW) + (pNW + pSE) - C(4) * phi));

    // closure (S3): rho (Eq. 13) in FP64, mu_phi (Eqs. 6-7), lambda (Eq. 3), n (Eq. 2)
    const double rho = (double)phi * I.drho + I.rho_g;
    const C mu_phi = C(4.0 * I.beta) * phi * (phi - C(1)) * (phi - C(0.5)) - C(I.kappa) * lap;
    const C lam = C(4) * phi * (C(1) - phi) * C(I.inv_w);
    const C mag = sqrt(dpx * dpx + dpy * dpy);
    C nx_ = C(0), ny_ = C(0);
    if (mag > C(1e-12)) {
        const C im = C(1) / mag;
        nx_ = dpx * im;
        ny_ = dpy * im;
    }
    C nu;
    if (I.visc_law == VISC_LINEAR) {
        nu = phi * C(I.nu_l - I.nu_g) + C(I.nu_g);
    } else if (I.visc_law == VISC_INVERSE) {
        nu = C(1) / (phi * C(I.inv_nu_l - I.inv_nu_g) + C(I.inv_nu_g));
    } else {
        nu = (phi >= C(0.5) ? C(I.mu_l) : C(I.mu_g)) / C(rho);
    }
    const C inv_tau_g = C(1) / (C(3) * nu + C(0.5));   // Eq. 23
    const C Fx = mu_phi * dpx + C(I.Gx);               // Eqs. 5, 19
    const C Fy = mu_phi * dpy + C(I.Gy);

    // moments in FP64 (Eq. 22): u first, then p
    double G[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) G[i] = (double)g[i];
    double jx = G[1];
    jx -= G[3];
    jx += G[5];
    jx -= G[6];
    jx -= G[7];
    jx += G[8];
    double jy = G[2];
    jy -= G[4];
    jy += G[5];
    jy += G[6];
    jy -= G[7];
    jy -= G[8];
    const double irho = 1.0 / rho;
    const double ux = (jx + 0.5 * (double)Fx) * irho;
    const double uy = (jy + 0.5 * (double)Fy) * irho;
    double sg = G[1];
#pragma unroll
    for (int i = 2; i < 9; ++i) sg += G[i];
    const double uu = ux * ux + uy * uy;
    const double pr = 0.6 * (sg + 0.5 * I.drho * (ux * (double)dpx + uy * (double)dpy) -
                             (2.0 / 3.0) * rho * uu);

    if (MODE == MODE_MOMENTS) {
        mom[0] = (double)phi;
        mom[1] = rho;
        mom[2] = pr;
        mom[3] = ux;
        mom[4] = uy;
        return;
    }

    const C cux = C(ux), cuy = C(uy), cp = C(pr), crho = C(rho), cuu = C(uu);

    // d_t(phi u) as a backward difference over one step; keep phi u for the next step
    const C pux = phi * cux, puy = phi * cuy;
    const C Dx = pux - qx, Dy = puy - qy;
    qx = pux;
    qy = puy;

    // f collision (Eqs. 8, 9, 11) in deviation form: d_i = f_i - w_i phi_ref
    const C itf = C(I.inv_tau_f), cf = C(I.cf);
    const C phid = phi - C(I.phi_ref);
    const C ax = C(3) * Dx + lam * nx_;
    const C ay = C(3) * Dy + lam * ny_;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const C w = wgt<C>(i);
        const C cu = C(CX[i]) * cux + C(CY[i]) * cuy;
        const C feq = w * phid + C(3) * w * phi * cu;
        const C src = cf * w * (C(CX[i]) * ax + C(CY[i]) * ay);
        fo[i] = f[i] - (f[i] - feq) * itf + src;
    }

    // g collision (Eqs. 15-17, 20)
    const C cg = C(1) - C(0.5) * inv_tau_g;
    const C drho = C(I.drho);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const C w = wgt<C>(i);
        const C cu = C(CX[i]) * cux + C(CY[i]) * cuy;
        const C s = w * (C(3) * cu + C(4.5) * cu * cu - C(1.5) * cuu);
        const C geq = (i == 0 ? C(-5.0 / 3.0) * cp : C(3) * w * cp) + crho * s;
        const C cF = C(CX[i]) * Fx + C(CY[i]) * Fy;
        const C cgp = C(CX[i]) * dpx + C(CY[i]) * dpy;
        const C frc = cg * w * (C(3) * cF + C(3) * drho * cu * cgp);
        go[i] = g[i] - (g[i] - geq) * inv_tau_g + frc;
    }
}

// ------------------------------------------------------------------ fused step kernel
// One block of 256 threads (64 x 4) owns a tile of 64 x 4K nodes.  Each thread pulls the
// f, g and q of its K nodes, writes their phi into an LDS tile, the block recomputes phi
// on the one-node halo ring from pulled f (neighbouring tiles' data, mostly L2 hits), and
// after one barrier every node has its 3 x 3 phi neighbourhood in LDS.
//
// Block b runs tile (b % 8) * per_xcd + b / 8: the hardware deals blocks round-robin to
// the 8 XCDs, so each XCD walks one contiguous run of tiles and finds the halo rows of
// its previous tiles in its own L2.
//
// RING_FROM_PLANE (split step): the halo ring is read from a phi plane written by
// k_phi_plane instead of being recomputed.
template <typename S, int K, bool PULL, int MODE, bool RING_FROM_PLANE>
__global__ __launch_bounds__(BLOCK) void k_step(const InstDev* __restrict__ insts,
                                                const TileDesc* __restrict__ tiles, int ntiles,
                                                int per_xcd, const S* __restrict__ fsrc,
                                                const S* __restrict__ gsrc, S* __restrict__ fdst,
                                                S* __restrict__ gdst,
                                                typename Store<S>::C* __restrict__ q,
                                                const typename Store<S>::C* __restrict__ phiplane,
                                                double* __restrict__ mom_out) {
    using C = typename Store<S>::C;
    constexpr int TY = 4 * K;
    constexpr int LW = TILE_X + 2;
    __shared__ C sphi[(TY + 2) * LW];

    const int b = blockIdx.x;
    const int t = (b % NXCD) * per_xcd + b / NXCD;
    if (t >= ntiles) return;
    const TileDesc T = tiles[t];
    const InstDev& I = insts[T.inst];
    const int nx = I.nx, ny = I.ny;
    const int w = min(TILE_X, nx - T.x0);
    const int h = min(TY, ny - T.y0);
    const int tid = threadIdx.x;
    const int lx = tid & (TILE_X - 1);
    const int ly = tid >> 6;
    const int x = T.x0 + lx;

    const S* fb = fsrc + I.off_dist;
    const S* gb = gsrc + I.off_dist;
    C* qb = q + I.off_q;
    const int plane = (int)I.plane;
    const C isf = C(I.inv_scale_f), isg = C(I.inv_scale_g);

    C f[K][9], g[K][9], qx[K], qy[K];
    bool valid[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int yl = ly + 4 * k;
        valid[k] = lx < w && yl < h;
        if (valid[k]) {
            const int y = T.y0 + yl;
            int o[9];
            pull_offsets<PULL>(I, x, y, o);
#pragma unroll
            for (int i = 0; i < 9; ++i) f[k][i] = Store<S>::get(fb, o[i]);
#pragma unroll
            for (int i = 0; i < 9; ++i) g[k][i] = Store<S>::get(gb, o[i]);
            const int self = y * I.pitch + x;
            qx[k] = qb[self];
            qy[k] = qb[plane + self];
        }
    }
    // phi of the tile's own nodes (Eq. 12)
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (valid[k]) {
            C s = f[k][0];
#pragma unroll
            for (int i = 1; i < 9; ++i) s += f[k][i];
            sphi[(ly + 4 * k + 1) * LW + lx + 1] = C(I.phi_ref) + s * isf;
        }
    }
    // halo ring: top row, bottom row (w + 2 each), left and right columns (h each)
    const int ring = 2 * (w + 2) + 2 * h;
    if (tid < ring) {
        int rx, ry;
        if (tid < w + 2) {
            rx = tid - 1;
            ry = -1;
        } else if (tid < 2 * (w + 2)) {
            rx = tid - (w + 2) - 1;
            ry = h;
        } else if (tid < 2 * (w + 2) + h) {
            rx = -1;
            ry = tid - 2 * (w + 2);
        } else {
            rx = w;
            ry = tid - 2 * (w + 2) - h;
        }
        int gx = T.x0 + rx;
        gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
        const int gy = ghost_row(I, T.y0 + ry);
        C v;
        if (RING_FROM_PLANE) {
            v = phiplane[I.off_phi + gy * I.pitch + gx];
        } else {
            v = pulled_phi<S, PULL>(I, fb, gx, gy);
        }
        sphi[(ry + 1) * LW + rx + 1] = v;
    }
    __syncthreads();

    S* fo_b = fdst + I.off_dist;
    S* go_b = gdst + I.off_dist;
    const C sf = C(I.scale_f), sgs = C(I.scale_g);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!valid[k]) continue;
        const int yl = ly + 4 * k;
        const int y = T.y0 + yl;
        const C* r0 = sphi + yl * LW + lx;        // row below (y - 1)
        const C* r1 = r0 + LW;                    // own row
        const C* r2 = r1 + LW;                    // row above (y + 1)
        C fd[9], gd[9], fo[9], go[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            fd[i] = f[k][i] * isf;
            gd[i] = g[k][i] * isg;
        }
        double mom[5];
        node_update<C, MODE>(I, fd, gd, r1[1], r1[2], r2[1], r1[0], r0[1], r2[2], r2[0], r0[0],
                             r0[2], qx[k], qy[k], fo, go, mom);
        const int self = y * I.pitch + x;
        if (MODE == MODE_MOMENTS) {
            const int64_t n = (int64_t)nx * ny;
            const int64_t c = (int64_t)y * nx + x;
#pragma unroll
            for (int m = 0; m < 5; ++m) mom_out[m * n + c] = mom[m];
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) Store<S>::put(fo_b, i * plane + self, fo[i] * sf);
#pragma unroll
            for (int i = 0; i < 9; ++i) Store<S>::put(go_b, i * plane + self, go[i] * sgs);
            qb[self] = qx[k];
            qb[plane + self] = qy[k];
        }
    }
}

// ------------------------------------------------------------------ split step: phi plane
// First half of the two-launch step: phi (Eq. 12) of every node from the pulled f.
template <typename S, int K>
__global__ __launch_bounds__(BLOCK) void k_phi_plane(const InstDev* __restrict__ insts,
                                                     const TileDesc* __restrict__ tiles,
                                                     int ntiles, int per_xcd,
                                                     const S* __restrict__ fsrc,
                                                     typename Store<S>::C* __restrict__ phiplane) {
    const int b = blockIdx.x;
    const int t = (b % NXCD) * per_xcd + b / NXCD;
    if (t >= ntiles) return;
    const TileDesc T = tiles[t];
    const InstDev& I = insts[T.inst];
    const int w = min(TILE_X, I.nx - T.x0);
    const int h = min(4 * K, I.ny - T.y0);
    const int lx = threadIdx.x & (TILE_X - 1);
    const int ly = threadIdx.x >> 6;
    const S* fb = fsrc + I.off_dist;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int yl = ly + 4 * k;
        if (lx < w && yl < h) {
            const int x = T.x0 + lx, y = T.y0 + yl;
            phiplane[I.off_phi + y * I.pitch + x] = pulled_phi<S, true>(I, fb, x, y);
        }
    }
}

// ------------------------------------------------------------------ initial state
// f = f^eq(phi0, u0) (Eq. 9), g = g^eq(p = 0, u0) with rho(phi0) (Eq. 16), q = phi0 u0, in
// the storage codec, already in streamed form.
template <typename S>
__global__ __launch_bounds__(BLOCK) void k_init(const InstDev* __restrict__ insts, int inst,
                                                const double* __restrict__ phi0,
                                                const double* __restrict__ ux0,
                                                const double* __restrict__ uy0,
                                                S* __restrict__ f, S* __restrict__ g,
                                                typename Store<S>::C* __restrict__ q) {
    using C = typename Store<S>::C;
    const InstDev& I = insts[inst];
    const int x = blockIdx.x * TILE_X + (threadIdx.x & (TILE_X - 1));
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= I.nx || y >= I.ny) return;
    const int c = y * I.nx + x;
    const double ph = phi0[c], ux = ux0[c], uy = uy0[c];
    const double rho = ph * I.drho + I.rho_g;
    const double uu = ux * ux + uy * uy;
    const int self = y * I.pitch + x;
    const int plane = (int)I.plane;
    S* fb = f + I.off_dist;
    S* gb = g + I.off_dist;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double w = wgt<double>(i);
        const double cu = CX[i] * ux + CY[i] * uy;
        const double feq = w * ph * (1.0 + 3.0 * cu);
        const double s = w * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        const double geq = rho * s;   // p = 0
        Store<S>::put(fb, i * plane + self, (C)((feq - w * I.phi_ref) * I.scale_f));
        Store<S>::put(gb, i * plane + self, (C)(geq * I.scale_g));
    }
    C* qb = q + I.off_q;
    qb[self] = (C)(ph * ux);
    qb[plane + self] = (C)(ph * uy);
}

// ------------------------------------------------------------------ reductions
// Per-block partials over the FP64 moment planes of one instance, then one block folds
// the partials in a fixed order: the result does not depend on timing.
constexpr int NRED = 13;
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

// fixed-shape tree over the block's 256 slots in LDS
__device__ __forceinline__ void block_fold(double (&acc)[NRED], double* sh) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NRED; ++k) sh[k * BLOCK + tid] = acc[k];
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (tid < s) {
            double other[NRED];
#pragma unroll
            for (int k = 0; k < NRED; ++k) other[k] = sh[k * BLOCK + tid + s];
            red_join(acc, other);
#pragma unroll
            for (int k = 0; k < NRED; ++k) sh[k * BLOCK + tid] = acc[k];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(BLOCK) void k_reduce_partial(const double* __restrict__ mom, int nx,
                                                          int ny, int periodic_y, double xc,
                                                          double yc, double r_in, double r_out,
                                                          double* __restrict__ partials) {
    __shared__ double sh[NRED * BLOCK];
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
    __shared__ double sh[NRED * BLOCK];
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

// ------------------------------------------------------------------ launchers
namespace {
inline int grid_for(int ntiles, int& per_xcd) {
    per_xcd = (ntiles + NXCD - 1) / NXCD;
    return per_xcd * NXCD;
}

template <typename S, int K>
hipError_t step_k(const StepArgs& a) {
    using C = typename Store<S>::C;
    int per;
    const int grid = grid_for(a.ntiles, per);
    const S* fs = (const S*)a.fsrc;
    const S* gs = (const S*)a.gsrc;
    S* fd = (S*)a.fdst;
    S* gd = (S*)a.gdst;
    C* q = (C*)a.q;
    C* ph = (C*)a.phiplane;
    if (!a.pull) {
        k_step<S, K, false, MODE_STEP, false><<<grid, BLOCK, 0, a.stream>>>(
            a.insts, a.tiles, a.ntiles, per, fs, gs, fd, gd, q, ph, nullptr);
    } else if (a.split) {
        k_phi_plane<S, K><<<grid, BLOCK, 0, a.stream>>>(a.insts, a.tiles, a.ntiles, per, fs, ph);
        k_step<S, K, true, MODE_STEP, true><<<grid, BLOCK, 0, a.stream>>>(
            a.insts, a.tiles, a.ntiles, per, fs, gs, fd, gd, q, ph, nullptr);
    } else {
        k_step<S, K, true, MODE_STEP, false><<<grid, BLOCK, 0, a.stream>>>(
            a.insts, a.tiles, a.ntiles, per, fs, gs, fd, gd, q, ph, nullptr);
    }
    return hipGetLastError();
}

template <typename S>
hipError_t step_s(const StepArgs& a) {
    switch (a.tile_rows) {
        case 4: return step_k<S, 1>(a);
        case 8: return step_k<S, 2>(a);
        case 16: return step_k<S, 4>(a);
        default: return hipErrorInvalidValue;
    }
}

template <typename S>
hipError_t moments_s(const StepArgs& a, double* out) {
    using C = typename Store<S>::C;
    int per;
    const int grid = grid_for(a.ntiles, per);
    if (a.pull)
        k_step<S, 1, true, MODE_MOMENTS, false><<<grid, BLOCK, 0, a.stream>>>(
            a.insts, a.tiles, a.ntiles, per, (const S*)a.fsrc, (const S*)a.gsrc, nullptr, nullptr,
            (C*)a.q, nullptr, out);
    else
        k_step<S, 1, false, MODE_MOMENTS, false><<<grid, BLOCK, 0, a.stream>>>(
            a.insts, a.tiles, a.ntiles, per, (const S*)a.fsrc, (const S*)a.gsrc, nullptr, nullptr,
            (C*)a.q, nullptr, out);
    return hipGetLastError();
}

template <typename S>
hipError_t init_s(const InstDev* insts, int inst, int nx, int ny, const double* phi0,
                  const double* ux0, const double* uy0, void* f, void* g, void* q,
                  hipStream_t st) {
    using C = typename Store<S>::C;
    dim3 grid((nx + TILE_X - 1) / TILE_X, (ny + 3) / 4);
    k_init<S><<<grid, BLOCK, 0, st>>>(insts, inst, phi0, ux0, uy0, (S*)f, (S*)g, (C*)q);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_step(int storage, const StepArgs& a) {
    switch (storage) {
        case STORE_F64: return step_s<double>(a);
        case STORE_F32: return step_s<float>(a);
        case STORE_F16: return step_s<_Float16>(a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_moments(int storage, const StepArgs& a, double* out) {
    switch (storage) {
        case STORE_F64: return moments_s<double>(a, out);
        case STORE_F32: return moments_s<float>(a, out);
        case STORE_F16: return moments_s<_Float16>(a, out);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(int storage, const InstDev* insts, int inst, int nx, int ny,
                       const double* phi0, const double* ux0, const double* uy0, void* f, void* g,
                       void* q, hipStream_t st) {
    switch (storage) {
        case STORE_F64: return init_s<double>(insts, inst, nx, ny, phi0, ux0, uy0, f, g, q, st);
        case STORE_F32: return init_s<float>(insts, inst, nx, ny, phi0, ux0, uy0, f, g, q, st);
        case STORE_F16: return init_s<_Float16>(insts, inst, nx, ny, phi0, ux0, uy0, f, g, q, st);
        default: return hipErrorInvalidValue;
    }
}

int reduce_blocks(int64_t n) {
    int64_t b = (n + BLOCK - 1) / BLOCK;
    return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
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
