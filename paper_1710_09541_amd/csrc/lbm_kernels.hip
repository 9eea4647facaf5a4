// HIP kernels (gfx950) of the phase-field lattice Boltzmann step of Liang et al.,
// arXiv:1710.09541: the conservative Allen-Cahn lattice f (Sec. 2.2) and the
// Navier-Stokes lattice g with the forcing distribution G_i (Sec. 2.3).
//
// State between steps (after the first): post-collision distributions, one array per
// lattice, x fastest: in FP64 and FP32 rows interleaved, [y][population i][pitch]; with
// 16-bit storage planes, [i][y][pitch] (rows_interleaved below).  A step pulls f_i(x - c_i), g_i(x - c_i) (streaming with
// the boundary rules), recomputes phi on the tile and a one-node halo into LDS, evaluates
// the isotropic stencils (Eqs. 27-28), the local closure (Eqs. 2-3, 5-7, 13, 19, 23-26),
// the moments u then p (Eq. 22), the backward difference of phi u (Eq. 11), collides
// both lattices (Eqs. 8-9, 11, 15-17, 20) and writes the result at the node itself into the
// other buffer.  The very first step reads the initial (already streamed) distributions
// in place instead of pulling.
//
// Storage.  FP64: the populations themselves, and phi u of the previous step.  FP32 /
// FP16 ("equilibrium deviation"): every node also writes its phi_w and u_w (phi and u
// rounded to FP32) and, in the 16-bit format, p_w, as one float3 or float4.  An f slot
// holds (f_i - w_i phi_w) 2^exp_f and a g slot (g_i - g^eq_i(rho(phi_w), p_w, u_w)) 2^exp_g
// (p_w = 0 in the FP32 format), both taken at the node that wrote the slot.  A reader
// decodes a pulled population with the (phi_w, p_w, u_w) of its source node,
// staged with a two-node halo in LDS; the g equilibrium is evaluated by one function,
// identically on both sides.  The moments, and the momentum the g relaxation must keep,
// are formed in FP64 (FP32 format) or from the FP32 deviations themselves (16-bit format).
// The stored numbers are thus the small
// non-equilibrium parts, a bulk at rest is stored exactly, and the short formats round
// small values only: slowly varying states keep their small increments (a weak body
// force, a drifting interface) instead of losing them to the rounding of full-size
// populations.  phi u of the previous step is phi_w u_w of the node itself.
//
// Boundary rules in pull form (y only; x is periodic):
//   periodic   the source row wraps
//   wall       half-way bounce-back: a population that would come from across the wall is
//              the node's own outgoing opposite population, f_i(x) = f*_opp(i)(x)
//   open       pressure outlet: one node beyond the edge row the pressure is the ambient
//              p = 0 and every other field has zero normal gradient, so an incoming
//              population of the edge row is what the edge node s = (x - c_ix, edge row)
//              sent out, f_i = f*_i(s), and g_i = g*_i(s) + (0 - p(s)) w_i / c_s^2 (the
//              pressure part of the flow equilibrium, Eq. 16, moved to the ambient one)
// The stencil's ghost rows at walls and open sides mirror the edge row.
//
// Variants, all compile-time: storage format S; rows per thread K (tiles of 64 x 4K nodes);
// PULL (false only for the first step); MODE (step, step with non-temporal population
// stores, or moments only); RING_FROM_PLANE (split step); INTERIOR (tiles away from every
// edge); QF, the velocities of the phase-field lattice (9 or 5).  The normal in F_i comes
// from the isotropic stencil (Eq. 2 with Eq. 27) or, per instance, from the local
// non-equilibrium scheme of Eq. 29, n = -C/|C|.
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

// Weights of the phase-field lattice with QF velocities: D2Q9 as above, or D2Q5 (the rest
// and the four axis velocities c_0..c_4, weights 1/3 and 1/6, the same c_s^2 = 1/3), which
// Sec. 2.2 admits for the Allen-Cahn lattice.  The flow lattice is always D2Q9.
template <typename C, int QF>
__device__ __forceinline__ C wf(int i) {
    if constexpr (QF == 5) return i == 0 ? C(1.0 / 3.0) : C(1.0 / 6.0);
    return wgt<C>(i);
}

// c_i . (a, b) written out per direction: with i known at compile time this folds to one
// add or none (IEEE arithmetic may not drop a product with a zero component by itself)
template <typename C>
__device__ __forceinline__ C dotc(int i, C a, C b) {
    switch (i) {
        case 0: return C(0);
        case 1: return a;
        case 2: return b;
        case 3: return -a;
        case 4: return -b;
        case 5: return a + b;
        case 6: return b - a;
        case 7: return -(a + b);
        default: return a - b;
    }
}

// fast reciprocal (about 1 ulp) for the FP32 arithmetic of the reduced formats
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ------------------------------------------------------------------ storage codecs
template <typename S>
struct Store;
// Element access through a 32-bit byte offset from a wave-uniform base, so the compiler can
// address with a scalar base register plus one 32-bit vector offset.
template <typename T>
__device__ __forceinline__ T ld(const T* p, int o) {
    return *(const T*)((const char*)p + (uint32_t)o * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st(T* p, int o, T v) {
    *(T*)((char*)p + (uint32_t)o * (uint32_t)sizeof(T)) = v;
}

template <>
struct Store<double> {
    using C = double;
    static __device__ __forceinline__ double get(const double* p, int o) { return ld(p, o); }
    static __device__ __forceinline__ void put(double* p, int o, double v) { st(p, o, v); }
};
template <>
struct Store<float> {
    using C = float;
    static __device__ __forceinline__ float get(const float* p, int o) { return ld(p, o); }
    static __device__ __forceinline__ void put(float* p, int o, float v) { st(p, o, v); }
};
template <>
struct Store<_Float16> {
    using C = float;
    static __device__ __forceinline__ float get(const _Float16* p, int o) {
        return (float)ld(p, o);
    }
    static __device__ __forceinline__ void put(_Float16* p, int o, float v) {
        st(p, o, (_Float16)v);
    }
};

// Buffer access to one instance's populations: a resource over its 9 planes, a per-lane byte
// offset (the node) and a wave-uniform byte offset in a scalar register (plane i and the
// pull shift), so the accesses of a node share one vector offset and cost no vector
// arithmetic.  Out-of-range offsets read zero and drop writes (hardware range check).  The
// descriptor's last word is the raw-buffer configuration of the gfx9 family.  The reduced
// formats use it (measured: FP16 +2 to +4 %, FP32 unchanged); the FP64 format keeps 64-bit
// global addressing, which measured 2 % faster at 1024^2.
using Rsrc = __amdgpu_buffer_rsrc_t;
template <typename S>
constexpr bool kBufAddr = sizeof(S) < 8;
__device__ __forceinline__ Rsrc rsrc_of(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
template <typename S>
struct Buf;
template <>
struct Buf<double> {
    static __device__ __forceinline__ double get(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    static __device__ __forceinline__ void put(Rsrc r, uint32_t vo, uint32_t so, double v) {
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned int, v), r, vo, so, 0);
    }
};
template <>
struct Buf<float> {
    static __device__ __forceinline__ float get(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    static __device__ __forceinline__ void put(Rsrc r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, vo, so, 0);
    }
};
template <>
struct Buf<_Float16> {
    static __device__ __forceinline__ float get(Rsrc r, uint32_t vo, uint32_t so) {
        return (float)__builtin_bit_cast(_Float16,
                                         __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0));
    }
    static __device__ __forceinline__ void put(Rsrc r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r,
                                              vo, so, 0);
    }
};

// f is kept as a rest deviation in every format shorter than FP64
template <typename S>
constexpr bool rest_deviation() {
    return sizeof(S) < sizeof(double);
}

// Per-node state of the reduced formats.  The 16-bit format keeps (phi_w, p_w, ux_w, uy_w),
// one float4 per node, and its g reference equilibrium holds p_w: a g slot rounded to 11
// bits relative must not carry the full pressure part 3 w_i p.  The FP32 format keeps
// (phi_w, ux_w, uy_w), one float3 per node, and references g to the equilibrium at p = 0:
// 24 bits hold that part with room to spare.  Its open sides need the pressure of the edge
// rows of the previous step, two rows of floats after the nodes' state.
template <typename S>
constexpr bool ref_has_p() {
    return sizeof(S) < sizeof(float);
}
template <typename S>
constexpr int state_floats() {
    return ref_has_p<S>() ? 4 : 3;
}

// Layout of the distribution arrays (one per lattice and buffer).  Planes: [i][y][pitch],
// population stride `plane`, row stride `pitch`.  Interleaved rows: [y][i][pitch],
// population stride `pitch`, row stride 9 pitch, so a tile's 9 rows of a lattice lie
// together in memory and a step runs fewer concurrent streams.  Measured: FP32 +0.7 to
// +1.5 %, FP64 +8.3 % at 4096^2 (-1 % on a batch), 16-bit storage -0.9 to -3.1 %; each
// format takes the faster one.
template <typename S>
constexpr bool rows_interleaved() {
    return sizeof(S) >= 4;
}
// population stride and row stride of the distribution arrays
template <typename S>
__device__ __forceinline__ int pop_stride(const InstDev& I) {
    return rows_interleaved<S>() ? I.pitch : (int)I.plane;
}
template <typename S>
__device__ __forceinline__ int row_stride(const InstDev& I) {
    return rows_interleaved<S>() ? 9 * I.pitch : I.pitch;
}

// ------------------------------------------------------------------ streaming offsets
// Element offsets (relative to the instance's plane 0) of the 9 populations arriving at
// node (x, y), and the source node (y * pitch + x) of each slot.  PULL = false reads the
// node's own slots (the initial state is already in streamed form).
// INTERIOR: the node and its neighbours are away from every edge (no wrap, no boundary).
template <bool PULL, bool INTERIOR = false>
__device__ __forceinline__ void pull_offsets_planes(const InstDev& I, int x, int y, int o[9],
                                                    int src[9]) {
    const int pitch = I.pitch;
    const int plane = (int)I.plane;
    const int self = y * pitch + x;
    if (!PULL) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            o[i] = i * plane + self;
            src[i] = self;
        }
        return;
    }
    if (INTERIOR) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            src[i] = self - dotc<int>(i, 1, pitch);
            o[i] = i * plane + src[i];
        }
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
    src[0] = self;
    src[1] = rc + xm;
    src[3] = rc + xp;
    src[2] = bl ? self : rm + x;
    src[5] = bl ? self : rm + xm;
    src[6] = bl ? self : rm + xp;
    src[4] = bh ? self : rp + x;
    src[7] = bh ? self : rp + xp;
    src[8] = bh ? self : rp + xm;
    o[0] = self;
    o[1] = plane + src[1];
    o[3] = 3 * plane + src[3];
    o[2] = bl ? 4 * plane + self : 2 * plane + src[2];
    o[5] = bl ? 7 * plane + self : 5 * plane + src[5];
    o[6] = bl ? 8 * plane + self : 6 * plane + src[6];
    o[4] = bh ? 2 * plane + self : 4 * plane + src[4];
    o[7] = bh ? 5 * plane + self : 7 * plane + src[7];
    o[8] = bh ? 6 * plane + self : 8 * plane + src[8];
}

// the same with interleaved rows: population stride pitch, row stride 9 pitch
template <bool PULL, bool INTERIOR = false>
__device__ __forceinline__ void pull_offsets_rows(const InstDev& I, int x, int y, int o[9],
                                                  int src[9]) {
    const int pitch = I.pitch;
    const int dp = 9 * pitch;
    const int self = y * pitch + x;
    const int selfd = y * dp + x;
    if (!PULL) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            o[i] = i * pitch + selfd;
            src[i] = self;
        }
        return;
    }
    if (INTERIOR) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            src[i] = self - dotc<int>(i, 1, pitch);
            o[i] = i * pitch + selfd - dotc<int>(i, 1, dp);
        }
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
    src[0] = self;
    src[1] = rc + xm;
    src[3] = rc + xp;
    src[2] = bl ? self : rm + x;
    src[5] = bl ? self : rm + xm;
    src[6] = bl ? self : rm + xp;
    src[4] = bh ? self : rp + x;
    src[7] = bh ? self : rp + xp;
    src[8] = bh ? self : rp + xm;
    const int dc = y * dp, dm = ym * dp, dq = yp * dp;
    o[0] = selfd;
    o[1] = pitch + dc + xm;
    o[3] = 3 * pitch + dc + xp;
    o[2] = bl ? 4 * pitch + selfd : 2 * pitch + dm + x;
    o[5] = bl ? 7 * pitch + selfd : 5 * pitch + dm + xm;
    o[6] = bl ? 8 * pitch + selfd : 6 * pitch + dm + xp;
    o[4] = bh ? 2 * pitch + selfd : 4 * pitch + dq + x;
    o[7] = bh ? 5 * pitch + selfd : 7 * pitch + dq + xp;
    o[8] = bh ? 6 * pitch + selfd : 8 * pitch + dq + xm;
}

template <typename S, bool PULL, bool INTERIOR = false>
__device__ __forceinline__ void pull_offsets(const InstDev& I, int x, int y, int o[9],
                                             int src[9]) {
    if constexpr (rows_interleaved<S>())
        pull_offsets_rows<PULL, INTERIOR>(I, x, y, o, src);
    else
        pull_offsets_planes<PULL, INTERIOR>(I, x, y, o, src);
}

// Scalar (wave-uniform) part of the element offset of slot i of a node, for distribution
// arrays with population stride ps and row stride dp: i ps - c_ix - c_iy dp when pulling
// (PULL) and i ps when reading in place.  With interleaved rows (ROWS) that can be negative,
// so the per-lane part (pull_vo) is taken one distribution row below the node when pulling
// (rows >= 1 there) and the scalar part is i ps + dp - c_i.(1, dp); with planes
// i ps - c_i.(1, dp) is never negative (i >= 1 wherever c_i is not zero, and ps > 2 dp).
template <bool PULL, bool ROWS>
__device__ __forceinline__ uint32_t pull_so(int i, int ps, int dp) {
    return (uint32_t)(i * ps + (PULL ? (ROWS ? dp : 0) - dotc<int>(i, 1, dp) : 0));
}
template <bool PULL, bool ROWS>
__device__ __forceinline__ uint32_t pull_vo(int x, int y, int dp) {
    return (uint32_t)(y * dp + x - (PULL && ROWS ? dp : 0));
}

// The same sources as LDS indices of an RW-wide region (the tile's width + 4) with a
// two-node halo: (lx, ly) is the node's unwrapped position relative to the tile origin and
// gy its row.  dir[i] is the direction of the slot that was read (the opposite one after a
// bounce-back).
template <bool PULL, bool INTERIOR, int RW>
__device__ __forceinline__ void pull_local(const InstDev& I, int gy, int lx, int ly, int r[9],
                                           int dir[9]) {
    const int c = (ly + 2) * RW + lx + 2;
#pragma unroll
    for (int i = 0; i < 9; ++i) dir[i] = i;
    if (!PULL) {
#pragma unroll
        for (int i = 0; i < 9; ++i) r[i] = c;
        return;
    }
    if (INTERIOR) {
#pragma unroll
        for (int i = 0; i < 9; ++i) r[i] = c - dotc<int>(i, 1, RW);
        return;
    }
    const bool at_lo = gy == 0, at_hi = gy == I.ny - 1;
    const bool bl = at_lo && I.bc_lo == BC_WALL, bh = at_hi && I.bc_hi == BC_WALL;
    const int dm = (at_lo && I.bc_lo == BC_OPEN) ? 0 : RW;  // row step to upward sources
    const int dp = (at_hi && I.bc_hi == BC_OPEN) ? 0 : RW;  // row step to downward sources
    r[0] = c;
    r[1] = c - 1;
    r[3] = c + 1;
    r[2] = bl ? c : c - dm;
    r[5] = bl ? c : c - dm - 1;
    r[6] = bl ? c : c - dm + 1;
    r[4] = bh ? c : c + dp;
    r[7] = bh ? c : c + dp + 1;
    r[8] = bh ? c : c + dp - 1;
    if (bl) {
        dir[2] = 4;
        dir[5] = 7;
        dir[6] = 8;
    }
    if (bh) {
        dir[4] = 2;
        dir[7] = 5;
        dir[8] = 6;
    }
}

// phi from the QF arriving stored values v (unscaled) and, for the rest-deviation formats,
// the phi of their source nodes ref[] and of the node itself (base):
//   phi = base + sum_i w_i (ref_i - base) + 2^-exp_f sum_i v_i           (Eq. 12)
// For the rest-deviation formats *res receives the rounding error of the final addition
// (exact, by Knuth's two-sum): phi + res is the sum before rounding to the phi format.
// SCALED (16-bit storage): the scaled sum is formed with one fused multiply-add per value,
// which reads the 16-bit value directly; 2^-exp_f is a power of two, so every product is
// exact and the partial sums round exactly as those of the unscaled values.
template <typename C, bool REF, int QF, bool SCALED = false>
__device__ __forceinline__ C phi_of(const C (&v)[9], const C (&ref)[9], C base, C isf,
                                    C* res = nullptr) {
    C s;
    if constexpr (SCALED) {
        s = __builtin_fmaf(v[0], isf, 0.0f);
#pragma unroll
        for (int i = 1; i < QF; ++i) s = __builtin_fmaf(v[i], isf, s);
    } else {
        s = v[0];
#pragma unroll
        for (int i = 1; i < QF; ++i) s += v[i];
        s = s * isf;
    }
    if (!REF) return s;
    C a = wf<C, QF>(0) * (ref[0] - base);
#pragma unroll
    for (int i = 1; i < QF; ++i) a += wf<C, QF>(i) * (ref[i] - base);
    const C d = a + s;
    const C phi = base + d;
    if (res) {
        const C bv = phi - base;
        *res = (base - (phi - bv)) + (d - bv);
    }
    return phi;
}

// row of the stencil's ghost node: wrap if periodic, else mirror the edge row
__device__ __forceinline__ int ghost_row(const InstDev& I, int y) {
    if (y < 0) return I.bc_lo == BC_PERIODIC ? y + I.ny : 0;
    if (y >= I.ny) return I.bc_hi == BC_PERIODIC ? y - I.ny : I.ny - 1;
    return y;
}

// MODE_STEP_NT: a step whose population stores are non-temporal (they do not allocate in
// the caches on their way to memory), which pays when the working set is larger than the
// last-level cache and costs when it fits; the autotuner chooses.
enum { MODE_STEP = 0, MODE_MOMENTS = 1, MODE_STEP_NT = 2 };

// store of a collided population into population offset po (i times the population stride)
// at the node's own distribution offset `self` (y times the row stride, plus x): through the
// buffer resource r over the destination array (reduced formats), non-temporal in
// MODE_STEP_NT
template <int MODE, typename S, typename C>
__device__ __forceinline__ void put_pop(Rsrc r, S* p, int po, int self, C v) {
    if constexpr (MODE == MODE_STEP_NT)
        __builtin_nontemporal_store(
            (S)v, (S*)((char*)p + (uint32_t)(po + self) * (uint32_t)sizeof(S)));
    else if constexpr (kBufAddr<S>)
        Buf<S>::put(r, (uint32_t)self * (uint32_t)sizeof(S), (uint32_t)po * (uint32_t)sizeof(S), v);
    else
        Store<S>::put(p, po + self, v);
}

// ------------------------------------------------------------------ FP64 node
// The FP64 format keeps the operations and their order of the plain CPU reference
// (sequential stencil sums, divisions by tau, rho and W, no fused multiply-add), so the two
// round alike and agree to the last bits over long runs.
__device__ __forceinline__ double s_exact(int i, double ux, double uy) {
#pragma clang fp contract(off)
    const double cu = CX[i] * ux + CY[i] * uy;
    const double uu = ux * ux + uy * uy;
    return wgt<double>(i) * (cu * 3.0 + cu * cu * 4.5 - uu * 1.5);   // Eq. 17
}

template <int MODE, int QF>
__device__ __forceinline__ void node_update_f64(const InstDev& I, const double (&f)[9],
                                                const double (&g)[9], const double (&nb)[9],
                                                double& qx, double& qy, double (&fo)[9],
                                                double (&go)[9], double (&mom)[5],
                                                double& p_out) {
#pragma clang fp contract(off)
    // nb[0] = phi, nb[1..8] = phi(x + c_i); stencils of Eqs. 27-28 as sequential sums
    const double phi = nb[0];
    double sx = 0.0, sy = 0.0, sl = 0.0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        sx += wgt<double>(i) * CX[i] * nb[i];
        sy += wgt<double>(i) * CY[i] * nb[i];
        sl += 2.0 * wgt<double>(i) * (nb[i] - phi);
    }
    const double dpx = sx * 3.0, dpy = sy * 3.0, lap = sl * 3.0;
    const double rho = phi * I.drho + I.rho_g;                                   // Eq. 13
    const double mu_phi = 4.0 * I.beta * phi * (phi - 1.0) * (phi - 0.5) - I.kappa * lap;
    const double lam = 4.0 * phi * (1.0 - phi) / I.W;                            // Eq. 3
    const double mag = sqrt(dpx * dpx + dpy * dpy);
    double nx_ = 0.0, ny_ = 0.0;
    if (mag > 1e-12) {
        nx_ = dpx / mag;
        ny_ = dpy / mag;
    }
    double nu;
    if (I.visc_law == VISC_LINEAR)
        nu = phi * (I.nu_l - I.nu_g) + I.nu_g;
    else if (I.visc_law == VISC_INVERSE)
        nu = 1.0 / (phi * (I.inv_nu_l - I.inv_nu_g) + I.inv_nu_g);
    else
        nu = (phi >= 0.5 ? I.mu_l : I.mu_g) / rho;
    const double tau_g = nu * 3.0 + 0.5;                                         // Eq. 23
    const double Fx = mu_phi * dpx + I.Gx, Fy = mu_phi * dpy + I.Gy;
    double mx = 0.0, my = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        mx += CX[i] * g[i];
        my += CY[i] * g[i];
    }
    const double ux = (mx + 0.5 * Fx) / rho, uy = (my + 0.5 * Fy) / rho;       // Eq. 22a
    double sg = 0.0;
#pragma unroll
    for (int i = 1; i < 9; ++i) sg += g[i];
    const double ugp = ux * dpx + uy * dpy;
    const double pr = 0.6 * (sg + 0.5 * I.drho * ugp + rho * s_exact(0, ux, uy));  // Eq. 22b
    p_out = pr;
    if (MODE == MODE_MOMENTS) {
        mom[0] = phi;
        mom[1] = rho;
        mom[2] = pr;
        mom[3] = ux;
        mom[4] = uy;
        return;
    }
    const double pux = phi * ux, puy = phi * uy;
    const double dtx = pux - qx, dty = puy - qy;
    qx = pux;
    qy = puy;
    double fe[9];
#pragma unroll
    for (int i = 0; i < QF; ++i) {
        const double cu = CX[i] * ux + CY[i] * uy;
        fe[i] = wf<double, QF>(i) * phi * (1.0 + cu * 3.0);                      // Eq. 9
    }
    if (I.grad_scheme == GRAD_LOCAL_NEQ) {
        // Eq. 29: n = -C/|C|, C = sum_i c_i (f_i - f_i^eq) + d_t(phi u)/2, the sums taken
        // over i in increasing order
        double cx = f[1] - fe[1];
        cx -= f[3] - fe[3];
        double cy = f[2] - fe[2];
        cy -= f[4] - fe[4];
        if (QF == 9) {
            cx += f[5] - fe[5];
            cx -= f[6] - fe[6];
            cx -= f[7] - fe[7];
            cx += f[8] - fe[8];
            cy += f[5] - fe[5];
            cy += f[6] - fe[6];
            cy -= f[7] - fe[7];
            cy -= f[8] - fe[8];
        }
        cx += 0.5 * dtx;
        cy += 0.5 * dty;
        const double cm = sqrt(cx * cx + cy * cy);
        nx_ = 0.0;
        ny_ = 0.0;
        if (cm > 1e-12) {
            nx_ = -cx / cm;
            ny_ = -cy / cm;
        }
    }
    const double vx = dtx * 3.0 + lam * nx_, vy = dty * 3.0 + lam * ny_;
    const double cf = 1.0 - 1.0 / (2.0 * I.tau_f);
    const double cg = 1.0 - 1.0 / (2.0 * tau_g);
#pragma unroll
    for (int i = 0; i < QF; ++i) {
        const double fs = cf * wf<double, QF>(i) * (CX[i] * vx + CY[i] * vy);   // Eq. 11
        fo[i] = f[i] - (f[i] - fe[i]) / I.tau_f + fs;                            // Eq. 8
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double w = wgt<double>(i);
        const double cu = CX[i] * ux + CY[i] * uy;
        const double ge = (i == 0 ? pr * 3.0 * (w - 1.0) : pr * 3.0 * w) + rho * s_exact(i, ux, uy);
        const double cF = CX[i] * Fx + CY[i] * Fy;
        const double cgp = CX[i] * dpx + CY[i] * dpy;
        const double gf = cg * w * (cF * 3.0 + I.drho * cu * cgp * 3.0);         // Eq. 20
        go[i] = g[i] - (g[i] - ge) / tau_g + gf;                                 // Eq. 15
    }
}

// ------------------------------------------------------------------ reduced-precision node
// FP32 reference equilibrium of the flow lattice (Eqs. 13, 16-17).  The per-node terms
// A = rho(phi_w), B = 3 p_w (p_w / c_s^2), ux_w, uy_w and H = 1.5 |u_w|^2 are formed once,
// then g^eq_i = w_i (B + A s_i) for i != 0, with s_i = c.u (3 + 4.5 c.u) - H, and
// g^eq_0 = B (w_0 - 1) - A w_0 H.  The same functions, with explicit fused multiply-adds
// and no other contraction, encode a g slot and decode it, so both agree bit for bit.
struct RefTerms {
    float A, B, ux, uy, H;
};
__device__ __forceinline__ RefTerms ref_terms(const InstDev& I, float phi, float p, float ux,
                                              float uy) {
#pragma clang fp contract(off)
    RefTerms r;
    r.A = __builtin_fmaf(phi, I.f_drho, I.f_rho_g);
    r.B = p * 3.0f;
    r.ux = ux;
    r.uy = uy;
    r.H = __builtin_fmaf(ux, ux, uy * uy) * 1.5f;
    return r;
}
__device__ __forceinline__ float geq_ref(int i, float A, float B, float ux, float uy, float H) {
#pragma clang fp contract(off)
    const float w = wgt<float>(i);
    if (i == 0) return __builtin_fmaf(B, w - 1.0f, -(A * (w * H)));
    const float cu = dotc<float>(i, ux, uy);
    const float s = __builtin_fmaf(cu, __builtin_fmaf(4.5f, cu, 3.0f), -H);
    return w * __builtin_fmaf(A, s, B);
}

// f: e_i = f_i - w_i phi of the arriving populations; eg, gs: the arriving g_i as stored
// deviation and reference equilibrium of its source node (g_i = eg_i + gs_i, summed for
// the moments in FP64, or in FP32 with M32); phi and its 8 neighbours; res: rounding error
// of phi (the f populations sum to phi + res); qx, qy: phi_w u_w of this node at the
// previous step.
// Writes the collided e_i into fo, the g deviations g*_i - g^eq_i(published moments) into
// go and the published p_w, u_w into pw, or the moments into mom.  FIRST: the state is the
// initial one, f = f^eq(phi0, u0) and g = g^eq(p = 0, u0) at every node.  REFP: the g
// reference holds the published p_w (16-bit format); otherwise p = 0 (FP32 format).  M32:
// the moments in FP32 (16-bit format), otherwise in FP64.
template <int MODE, bool FIRST, int QF, bool REFP, bool M32>
__device__ __forceinline__ void node_update_ref(const InstDev& I, const float (&f)[9],
                                                const float (&eg)[9], const float (&gs)[9],
                                                float phi, float pE, float pN, float pW,
                                                float pS, float pNE, float pNW, float pSW,
                                                float pSE, float res, float qx, float qy,
                                                float (&fo)[9], float (&go)[9], float (&pw)[3],
                                                double (&mom)[5]) {
    using C = float;
    // isotropic gradient and Laplacian (Eqs. 27-28): weights over c_s^2
    const C dpx = C(3) * (C(1.0 / 9.0) * (pE - pW) + C(1.0 / 36.0) * ((pNE - pNW) + (pSE - pSW)));
    const C dpy = C(3) * (C(1.0 / 9.0) * (pN - pS) + C(1.0 / 36.0) * ((pNE + pNW) - (pSW + pSE)));
    const C lap = C(6) * (C(1.0 / 9.0) * ((pE + pW) + (pN + pS) - C(4) * phi) +
                          C(1.0 / 36.0) * ((pNE + pSW) + (pNW + pSE) - C(4) * phi));

    // closure (S3): rho (Eq. 13), mu_phi (Eqs. 6-7), lambda (Eq. 3), n (Eq. 2)
    double rho64 = 0.0;
    C rho;
    if constexpr (M32) {
        rho = __builtin_fmaf(phi, I.f_drho, I.f_rho_g);
    } else {
        rho64 = (double)phi * I.drho + I.rho_g;
        rho = C(rho64);
    }
    const C mu_phi = I.f_beta4 * phi * (phi - C(1)) * (phi - C(0.5)) - I.f_kappa * lap;
    const C lam = C(4) * phi * (C(1) - phi) * I.f_inv_w;
    const C mag2 = dpx * dpx + dpy * dpy;
    C nx_ = C(0), ny_ = C(0);
    if (mag2 > C(1e-24)) {   // |grad phi| > 1e-12
        const C im = __builtin_amdgcn_rsqf(mag2);
        nx_ = dpx * im;
        ny_ = dpy * im;
    }
    C nu;
    if (I.visc_law == VISC_LINEAR) {
        nu = phi * I.f_dnu + I.f_nu_g;
    } else if (I.visc_law == VISC_INVERSE) {
        nu = rcp(phi * I.f_dinv_nu + I.f_inv_nu_g);
    } else {
        nu = (phi >= C(0.5) ? I.f_mu_l : I.f_mu_g) * rcp(rho);
    }
    const C inv_tau_g = rcp(C(3) * nu + C(0.5));       // Eq. 23
    const C Fx = mu_phi * dpx + I.f_Gx;                // Eqs. 5, 19
    const C Fy = mu_phi * dpy + I.f_Gy;

    // moments (Eq. 22), u first, then p.
    // M32 (16-bit format): in FP32.  Each population is its stored deviation plus the source's
    // reference equilibrium, rounded relative to that reference, so u and p carry errors of
    // the order of their own FP32 rounding, far below the format's own.  Momentum
    // conservation does not rest on them: the collision's momentum correction below is
    // formed from the same FP32 deviations it relaxes.
    // Otherwise (FP32 format): in FP64 from the exact sums of the FP32 parts.
    C cux, cuy, cp, irho;
    double mx = 0.0, my = 0.0;
    if constexpr (M32) {
        C G[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) G[i] = eg[i] + gs[i];
        C jx = G[1];
        jx -= G[3];
        jx += G[5];
        jx -= G[6];
        jx -= G[7];
        jx += G[8];
        C jy = G[2];
        jy -= G[4];
        jy += G[5];
        jy += G[6];
        jy -= G[7];
        jy -= G[8];
        irho = rcp(rho);
        const C ux = (jx + C(0.5) * Fx) * irho;   // (rho u) / rho
        const C uy = (jy + C(0.5) * Fy) * irho;
        C sg = G[1];
#pragma unroll
        for (int i = 2; i < 9; ++i) sg += G[i];
        const C uu = ux * ux + uy * uy;
        const C pr = C(0.6) * (sg + C(0.5) * I.f_drho * (ux * dpx + uy * dpy) -
                               C(2.0 / 3.0) * rho * uu);
        if (MODE == MODE_MOMENTS) {
            mom[0] = (double)phi;
            mom[1] = (double)rho;
            mom[2] = (double)pr;
            mom[3] = (double)ux;
            mom[4] = (double)uy;
            return;
        }
        cux = ux;
        cuy = uy;
        cp = pr;
    } else {
        double G[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) G[i] = (double)eg[i] + (double)gs[i];
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
        mx = jx + 0.5 * (double)Fx;   // rho u
        my = jy + 0.5 * (double)Fy;
        const double irho64 = 1.0 / rho64;
        const double ux = mx * irho64;
        const double uy = my * irho64;
        double sg = G[1];
#pragma unroll
        for (int i = 2; i < 9; ++i) sg += G[i];
        const double uu = ux * ux + uy * uy;
        const double pr = 0.6 * (sg + 0.5 * I.drho * (ux * (double)dpx + uy * (double)dpy) -
                                 (2.0 / 3.0) * rho64 * uu);
        if (MODE == MODE_MOMENTS) {
            mom[0] = (double)phi;
            mom[1] = rho64;
            mom[2] = pr;
            mom[3] = ux;
            mom[4] = uy;
            return;
        }
        cux = C(ux);
        cuy = C(uy);
        cp = C(pr);
        irho = C(irho64);
    }

    // the FP32 moments this node publishes (and encodes its g against)
    pw[0] = cp;
    pw[1] = cux;
    pw[2] = cuy;

    // d_t(phi u) as a backward difference over one step
    const C Dx = phi * cux - qx, Dy = phi * cuy - qy;

    if (I.grad_scheme == GRAD_LOCAL_NEQ) {
        // Eq. 29: n = -C/|C| with C = sum_i c_i (f_i - f_i^eq) + D/2.  On the rest
        // deviations sum_i c_i (f_i - f_i^eq) = sum_i c_i e_i - phi u, so
        // C = sum_i c_i e_i - (phi u + Q)/2 with Q = phi u of the previous step.
        // On the initial state f = f^eq(phi0, u0), Q = phi0 u0 and sum_i c_i g_i = rho u0,
        // so u - u0 = F/(2 rho) (Eq. 22a) and C = phi0 (u0 - u)/2 = -phi F/(4 rho) exactly.
        // That C is of the order of the force, below the rounding of the stored first
        // moment, so the first step takes the closed form.
        C cx, cy;
        if (FIRST) {
            const C k = C(-0.25) * phi * irho;
            cx = k * Fx;
            cy = k * Fy;
        } else {
            C ex = f[1] - f[3], ey = f[2] - f[4];
            if (QF == 9) {
                ex = (ex + (f[5] - f[7])) + (f[8] - f[6]);
                ey = (ey + (f[5] - f[7])) + (f[6] - f[8]);
            }
            cx = ex - C(0.5) * (phi * cux + qx);
            cy = ey - C(0.5) * (phi * cuy + qy);
        }
        const C cm2 = cx * cx + cy * cy;
        nx_ = C(0);
        ny_ = C(0);
        if (cm2 > C(1e-24)) {   // |C| > 1e-12
            const C im = __builtin_amdgcn_rsqf(cm2);
            nx_ = -cx * im;
            ny_ = -cy * im;
        }
    }

    // f collision (Eqs. 8, 9, 11) on e_i = f_i - w_i phi.  The populations sum to phi + res
    // before and after the collision (sum f^eq = phi, sum F_i = 0); the rest population is
    // taken from that invariant, so neither the rounding of phi nor the inexact FP32 weights
    // can bias the total phi.
    // With f^eq_i - w_i phi = 3 w_i phi c_i.u (Eq. 9) and the source F_i = (1 - 1/(2 tau_phi))
    // w_i c_i.a, a = 3 D + lambda n (Eq. 11), the update e_i - (e_i - (f^eq_i - w_i phi)) /
    // tau_phi + F_i is e_i (1 - 1/tau_phi) + w_i c_i.v with one vector
    // v = 3 phi u / tau_phi + (1 - 1/(2 tau_phi)) a per node.
    const C itf = I.f_inv_tau_f, cf = I.f_cf;
    const C ax = C(3) * Dx + lam * nx_;
    const C ay = C(3) * Dy + lam * ny_;
    const C phi3t = C(3) * phi * itf;
    const C vx = phi3t * cux + cf * ax;
    const C vy = phi3t * cuy + cf * ay;
    const C keepf = C(1) - itf;
#pragma unroll
    for (int i = 1; i < QF; ++i) fo[i] = f[i] * keepf + wf<C, QF>(i) * dotc<C>(i, vx, vy);
    C t = fo[1];
#pragma unroll
    for (int i = 2; i < QF; ++i) t += fo[i];
    fo[0] = res - t;

    // g collision (Eqs. 15-17, 20) on deviations from the published equilibrium gw:
    // g*_i - gw_i = (1 - 1/tau_g)(g_i - gw_i) + G_i + (1/tau_g)(g^eq_i - gw_i).  The last
    // term holds the FP32 rounding of the published moments and, where the reference is
    // taken at p = 0 (REFP false), the pressure part of the equilibrium, 3 p (w_i - [i = 0])
    // (Eq. 16), which is added as such.  Of the rounding, the part that carries momentum is
    // kept exactly: a 3 w_i c_i.dj correction with dj = rho u - sum_i c_i gw_i.  With the
    // moments in FP64, dj is formed in FP64 from them; with the moments in FP32 (M32), as
    // sum_i c_i d_i + F/2 from the very deviations d_i = g_i - gw_i the collision relaxes,
    // small numbers rounded relative to themselves.  Either way the collision conserves
    // momentum to FP32 rounding of small deviations, and a weak body force is not lost to
    // rounding.
    const RefTerms R = ref_terms(I, phi, REFP ? cp : 0.0f, cux, cuy);
    float gw[9], d[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        gw[i] = geq_ref(i, R.A, R.B, cux, cuy, R.H);
        d[i] = eg[i] + (gs[i] - gw[i]);
    }
    C cjx, cjy;
    if constexpr (M32) {
        C djx = d[1];
        djx -= d[3];
        djx += d[5];
        djx -= d[6];
        djx -= d[7];
        djx += d[8];
        C djy = d[2];
        djy -= d[4];
        djy += d[5];
        djy += d[6];
        djy -= d[7];
        djy -= d[8];
        cjx = C(3) * inv_tau_g * (djx + C(0.5) * Fx);
        cjy = C(3) * inv_tau_g * (djy + C(0.5) * Fy);
    } else {
        double wx = (double)gw[1];
        wx -= (double)gw[3];
        wx += (double)gw[5];
        wx -= (double)gw[6];
        wx -= (double)gw[7];
        wx += (double)gw[8];
        double wy = (double)gw[2];
        wy -= (double)gw[4];
        wy += (double)gw[5];
        wy += (double)gw[6];
        wy -= (double)gw[7];
        wy -= (double)gw[8];
        cjx = C(3) * inv_tau_g * C(mx - wx);
        cjy = C(3) * inv_tau_g * C(my - wy);
    }
    // G_i (Eq. 20) = w_i [c_i.(3 cg F) + 3 cg (rho_l - rho_g) (c_i.u)(c_i.grad phi)] with
    // cg = 1 - 1/(2 tau_g); its c_i-linear part and the momentum correction share one vector
    // e = 3 cg F + cj, and the pressure part (REFP false) is w_i pt for i != 0.
    const C cg3 = C(3) - C(1.5) * inv_tau_g;
    const C keep = C(1) - inv_tau_g;
    const C bq = cg3 * I.f_drho;
    const C ex = cg3 * Fx + cjx, ey = cg3 * Fy + cjy;
    const C pt = REFP ? C(0) : inv_tau_g * (C(3) * cp);
    go[0] = keep * d[0];
    if (!REFP) go[0] += (wgt<C>(0) - C(1)) * pt;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        C t = dotc<C>(i, ex, ey) + bq * dotc<C>(i, cux, cuy) * dotc<C>(i, dpx, dpy);
        if (!REFP) t += pt;
        go[i] = keep * d[i] + wgt<C>(i) * t;
    }
}

// ------------------------------------------------------------------ fused step kernel
// One block of 256 threads (64 x 4) owns a tile of 64 x 4K nodes.  Each thread pulls the
// f and g of its K nodes and puts their phi into an LDS tile; the block recomputes phi on
// the one-node halo ring from pulled f (neighbouring tiles' data, mostly L2 hits), and
// after a barrier every node has its 3 x 3 phi neighbourhood in LDS.  In the reduced
// formats the block first stages the previous step's per-node state (phi_w, u_w and, 16-bit
// format, p_w) over the tile plus two nodes into LDS, to decode the pulled populations.
//
// The hardware deals blocks round-robin to the 8 XCDs, so block b runs on XCD b % 8 as that
// XCD's (b / 8)-th block.  The tile list is handed to the XCDs in chunks of `chunk`
// consecutive tiles, chunk after chunk in turn: XCD x takes chunks x, x + 8, x + 16, ...  An
// XCD thus walks runs of neighbouring tiles and finds the halo rows of its previous tiles in
// its own L2.  One chunk per XCD (chunk = ntiles / 8 rounded up) gives each XCD one
// contiguous band, the best order for a single large grid; shorter chunks even out the
// work of the dies when the tiles' costs vary along the list (a batch of instances of
// different shapes).  With a persistent grid (stride < chunk blocks per XCD, as many as stay
// resident; one band per XCD) block b then moves on to every stride-th tile of its band, with
// a barrier between tiles so the next tile's LDS writes wait for this one's reads.
//
// RING_FROM_PLANE (split step): the halo ring is read from a phi plane written by
// k_phi_plane instead of being recomputed.
//
// q: FP64 format, phi u of the previous step (one double2 per node, updated in place).
// msrc / mdst: the per-node state of the previous step (read) and of this step (written):
// 16-bit format, (phi_w, p_w, ux_w, uy_w) as one float4 per node; FP32 format,
// (phi_w, ux_w, uy_w) as one float3 per node, then the pressure of the first and the last
// row (two rows of floats); FP64 format, only those two rows, of doubles.  An open side
// needs the edge rows' pressure.
template <typename S, int K, bool PULL, int MODE, bool RING_FROM_PLANE, bool INTERIOR, int QF,
          int TXW>
__device__ __forceinline__ void step_tile(
    const InstDev& I, const TileDesc& T, const S* __restrict__ fsrc,
    const S* __restrict__ gsrc, S* __restrict__ fdst, S* __restrict__ gdst,
    double* __restrict__ q, const typename Store<S>::C* __restrict__ phiplane,
    const float* __restrict__ msrc, float* __restrict__ mdst, double* __restrict__ mom_out,
    typename Store<S>::C* sphi, float4* sq, float2* sw) {
    using C = typename Store<S>::C;
    constexpr bool REF = rest_deviation<S>();
    constexpr bool REFP = ref_has_p<S>();
    constexpr bool SCALED = sizeof(S) < sizeof(float);   // only the 16-bit format is scaled
    // a stored 16-bit value times 2^-exp as one fused multiply-add that reads it directly
    // (the product is exact; with no scale the value is used as it is)
    const auto unscale = [](C v, C is) -> C {
        if constexpr (SCALED) return __builtin_fmaf(v, is, 0.0f);
        else return v;
    };
    constexpr int RPG = BLOCK / TXW;   // rows of the block's threads: 4, 8 or 16
    constexpr int TY = RPG * K;
    constexpr int RW = TXW + 4;        // staged region: the tile and two nodes around it
    constexpr int LW = TXW + 2;        // phi tile: the tile and one node around it
    constexpr int NR = REF ? (TY + 4) * RW : 1;
    const int nx = I.nx, ny = I.ny, pitch = I.pitch;
    const int w = INTERIOR ? TXW : min(TXW, nx - T.x0);
    const int h = INTERIOR ? TY : min(TY, ny - T.y0);
    const int tid = threadIdx.x;
    const int lx = tid & (TXW - 1);
    const int ly = tid / TXW;
    const int x = T.x0 + lx;

    const S* fb = fsrc + I.off_dist;
    const S* gb = gsrc + I.off_dist;
    const int plane = (int)I.plane;
    constexpr bool ROWS = rows_interleaved<S>();
    const int ps = ROWS ? pitch : plane, dp = ROWS ? 9 * pitch : pitch;   // distribution strides
    const C isf = SCALED ? C(I.f_inv_scale_f) : C(1), isg = SCALED ? C(I.f_inv_scale_g) : C(1);

    // The loads of the tile are issued at raised wave priority (reduced formats), so a
    // block's memory requests go out ahead of other waves' arithmetic.  Every load of the
    // tile (the staged previous state, the node's populations, the ring's) is issued before
    // the first wait, so a block spends one memory round trip, not one per staging pass.
    if (REF) __builtin_amdgcn_s_setprio(3);
    // previous per-node state over the tile and a two-node halo (wrapped; clamped rows
    // beyond a wall or an open side are never sources), NIT entries per thread
    constexpr int NIT = (NR + BLOCK - 1) / BLOCK;
    float4 m4[REF && REFP ? NIT : 1];
    float3 m3[REF && !REFP ? NIT : 1];
    if (REF) {
        const float* mb = msrc + I.off_mp;
        const bool pery = I.bc_lo == BC_PERIODIC;
        // one wrap suffices when the grid is at least as wide / tall as the staged block
        const bool wide = nx >= RW, tall = ny >= TY + 4;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int idx = tid + it * BLOCK;
            if (idx >= NR) break;
            const int sy = idx / RW - 2, sx = idx - (idx / RW) * RW - 2;
            int gx = T.x0 + sx;
            if (INTERIOR) {
            } else if (wide) {
                gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
            } else {
                gx %= nx;
                gx = gx < 0 ? gx + nx : gx;
            }
            int gy = T.y0 + sy;
            if (INTERIOR) {
            } else if (!pery) {
                gy = min(max(gy, 0), ny - 1);
            } else if (tall) {
                gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
            } else {
                gy %= ny;
                gy = gy < 0 ? gy + ny : gy;
            }
            if constexpr (REFP) m4[it] = ld((const float4*)mb, gy * pitch + gx);
            else m3[it] = ld((const float3*)mb, gy * pitch + gx);
        }
    }

    // slot i of a node arrives from node - c_i: away from the edges (and on the first step,
    // which reads the node's own slots) that shift is the same for every node, and the loads
    // of the reduced formats go through buffer resources with the shift in a scalar offset
    constexpr bool UNIFORM = (INTERIOR || !PULL) && kBufAddr<S>;
    const uint32_t pop_bytes = 9u * (uint32_t)plane * (uint32_t)sizeof(S);
    const Rsrc rf = rsrc_of(fb, pop_bytes), rg = rsrc_of(gb, pop_bytes);
    C f[K][9], g[K][9];
    bool valid[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int yl = ly + RPG * k;
        valid[k] = lx < w && yl < h;
        if (valid[k]) {
            const int y = T.y0 + yl;
            if (UNIFORM) {
                const uint32_t vo = pull_vo<PULL, ROWS>(x, y, dp) * (uint32_t)sizeof(S);
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const uint32_t so = pull_so<PULL, ROWS>(i, ps, dp) * (uint32_t)sizeof(S);
                    if (i < QF) f[k][i] = Buf<S>::get(rf, vo, so);
                    g[k][i] = Buf<S>::get(rg, vo, so);
                }
            } else {
                int o[9], src[9];
                pull_offsets<S, PULL, INTERIOR>(I, x, y, o, src);
#pragma unroll
                for (int i = 0; i < QF; ++i) f[k][i] = Store<S>::get(fb, o[i]);
#pragma unroll
                for (int i = 0; i < 9; ++i) g[k][i] = Store<S>::get(gb, o[i]);
            }
        }
    }
    // halo ring: top row, bottom row (w + 2 each), left and right columns (h each); the
    // ring's populations are requested together with the node's own
    const int ring = 2 * (w + 2) + 2 * h;
    const bool on_ring = tid < ring;
    int rx = 0, ry = 0, rgx = 0, rgy = 0, ryraw = 0;
    C rfv[9];
    if (on_ring) {
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
        rgx = T.x0 + rx;
        if (!INTERIOR) rgx = rgx < 0 ? rgx + nx : (rgx >= nx ? rgx - nx : rgx);
        ryraw = T.y0 + ry;
        rgy = INTERIOR ? ryraw : ghost_row(I, ryraw);
        if (!RING_FROM_PLANE) {
            if (UNIFORM) {
                const uint32_t vo = pull_vo<PULL, ROWS>(rgx, rgy, dp) * (uint32_t)sizeof(S);
#pragma unroll
                for (int i = 0; i < QF; ++i)
                    rfv[i] = Buf<S>::get(rf, vo,
                                         pull_so<PULL, ROWS>(i, ps, dp) * (uint32_t)sizeof(S));
            } else {
                int o[9], src[9];
                pull_offsets<S, PULL, INTERIOR>(I, rgx, rgy, o, src);
#pragma unroll
                for (int i = 0; i < QF; ++i) rfv[i] = Store<S>::get(fb, o[i]);
            }
        }
    }
    // the staged state's decode terms, into LDS
    if (REF) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int idx = tid + it * BLOCK;
            if (idx >= NR) break;
            float ph, pp, ux, uy;
            if constexpr (REFP) {
                ph = m4[it].x;
                pp = m4[it].y;
                ux = m4[it].z;
                uy = m4[it].w;
            } else {
                ph = m3[it].x;
                pp = 0.0f;
                ux = m3[it].y;
                uy = m3[it].z;
            }
            const RefTerms R = ref_terms(I, ph, pp, ux, uy);
            sq[idx] = make_float4(R.A, R.B, R.ux, R.uy);
            sw[idx] = make_float2(ph, R.H);
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
    }

    // phi of the tile's own nodes (and, reduced formats, its rounding residual)
    C res[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        res[k] = C(0);
        if (valid[k]) {
            const int yl = ly + RPG * k;
            C ref[9], base = C(0);
            if (REF) {
                int r[9], dir[9];
                pull_local<PULL, INTERIOR, RW>(I, T.y0 + yl, lx, yl, r, dir);
#pragma unroll
                for (int i = 0; i < QF; ++i) ref[i] = sw[r[i]].x;
                base = sw[(yl + 2) * RW + lx + 2].x;
            }
            sphi[(yl + 1) * LW + lx + 1] = phi_of<C, REF, QF, SCALED>(f[k], ref, base, isf, &res[k]);
        }
    }
    if (on_ring) {
        const int gx = rgx, gy = rgy, yraw = ryraw;
        C v;
        if (RING_FROM_PLANE) {
            v = phiplane[I.off_phi + gy * pitch + gx];
        } else {
            C ref[9], base = C(0);
            if (REF) {
                const bool mirrored = (yraw < 0 && I.bc_lo != BC_PERIODIC) ||
                                      (yraw >= ny && I.bc_hi != BC_PERIODIC);
                const int lyl = mirrored ? gy - T.y0 : ry;
                int r[9], dir[9];
                pull_local<PULL, INTERIOR, RW>(I, gy, rx, lyl, r, dir);
#pragma unroll
                for (int i = 0; i < QF; ++i) ref[i] = sw[r[i]].x;
                base = sw[(lyl + 2) * RW + rx + 2].x;
            }
            v = phi_of<C, REF, QF, SCALED>(rfv, ref, base, isf);
        }
        sphi[(ry + 1) * LW + rx + 1] = v;
    }
    __syncthreads();

    S* fo_b = fdst + I.off_dist;
    S* go_b = gdst + I.off_dist;
    const Rsrc rfo = rsrc_of(fo_b, pop_bytes), rgo = rsrc_of(go_b, pop_bytes);
    const C sf = SCALED ? C(I.f_scale_f) : C(1), sgs = SCALED ? C(I.f_scale_g) : C(1);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!valid[k]) continue;
        const int yl = ly + RPG * k;
        const int y = T.y0 + yl;
        const C* r0 = sphi + yl * LW + lx;        // row below (y - 1)
        const C* r1 = r0 + LW;                    // own row
        const C* r2 = r1 + LW;                    // row above (y + 1)
        const C phi = r1[1];
        const int self = y * pitch + x;     // per-node state
        const int selfd = y * dp + x;       // distributions
        double mom[5];
        // an edge row on an open side (pressure outlet): the populations entering through it
        const bool open_lo = PULL && !INTERIOR && y == 0 && I.bc_lo == BC_OPEN;
        const bool open_hi = PULL && !INTERIOR && y == ny - 1 && I.bc_hi == BC_OPEN;
        if constexpr (REF) {
            int r[9], dir[9];
            pull_local<PULL, INTERIOR, RW>(I, y, lx, yl, r, dir);
            float fd[9], eg[9], gs[9], fo[9], go[9], pw[3];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const float4 q4 = sq[r[i]];
                const float2 q2 = sw[r[i]];
                if (i < QF) fd[i] = __builtin_fmaf(wf<float, QF>(i), q2.x - phi, unscale(f[k][i], isf));
                eg[i] = unscale(g[k][i], isg);
                // decoded against the source node's equilibrium, at the ambient pressure 0 for
                // a population entering through an open side: g*_i(s) + (0 - p(s)) w_i / c_s^2.
                // The 16-bit format's reference holds p_w(s); the FP32 format's holds 0 and
                // takes p(s) from the edge-pressure row.
                const bool amb = (open_lo && CY[i] > 0) || (open_hi && CY[i] < 0);
                float B = q4.y;
                if (amb) {
                    if constexpr (REFP) {
                        B = 0.0f;
                    } else {
                        const float* pe = msrc + I.off_mp + 3 * (int64_t)plane + (open_hi ? pitch : 0);
                        int xs = x - CX[i];
                        xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
                        B = -3.0f * pe[xs];
                    }
                }
                gs[i] = geq_ref(dir[i], q4.x, B, q4.z, q4.w, q2.y);
            }
            const int me = (yl + 2) * RW + lx + 2;
            const float qx = sw[me].x * sq[me].z, qy = sw[me].x * sq[me].w;
            node_update_ref<MODE, !PULL, QF, REFP, SCALED>(I, fd, eg, gs, phi, r1[2], r2[1], r1[0], r0[1], r2[2], r2[0],
                                  r0[0], r0[2], res[k], qx, qy, fo, go, pw, mom);
            if (MODE != MODE_MOMENTS) {
#pragma unroll
                for (int i = 0; i < QF; ++i) put_pop<MODE>(rfo, fo_b, i * ps, selfd, fo[i] * sf);
#pragma unroll
                for (int i = 0; i < 9; ++i) put_pop<MODE>(rgo, go_b, i * ps, selfd, go[i] * sgs);
                if constexpr (REFP) {
                    st((float4*)(mdst + I.off_mp), self, make_float4(phi, pw[0], pw[1], pw[2]));
                } else {
                    st((float3*)(mdst + I.off_mp), self, make_float3(phi, pw[1], pw[2]));
                    // the pressure of an edge row on an open side, for the populations that
                    // enter through it at the next step
                    if (!INTERIOR && ((y == 0 && I.bc_lo == BC_OPEN) ||
                                      (y == ny - 1 && I.bc_hi == BC_OPEN)))
                        st(mdst + I.off_mp + 3 * (int64_t)plane, (y == 0 ? 0 : pitch) + x, pw[0]);
                }
            }
        } else {
            // phi u of the previous step, one double2 per node
            double2* qb = (double2*)(q + I.off_q);
            const double2 q2 = ld((const double2*)qb, self);
            double qx = q2.x, qy = q2.y;
            const double nb[9] = {phi, r1[2], r2[1], r1[0], r0[1], r2[2], r2[0], r0[0], r0[2]};
            // open side: the populations entering through it carry the pressure part of the
            // equilibrium at the ambient 0 instead of the source node's p(s), s = (x - c_ix,
            // edge row), kept from its collision in the edge-pressure rows
            if (open_lo || open_hi) {
#pragma clang fp contract(off)
                const double* pe = (const double*)(msrc + I.off_mp) + (open_hi ? pitch : 0);
                const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
                if (open_hi) {   // (0,-1) from x, (-1,-1) from x + 1, (1,-1) from x - 1
                    g[k][4] = g[k][4] + ((0.0 - pe[x]) * 3.0) * wgt<double>(4);
                    g[k][7] = g[k][7] + ((0.0 - pe[xp]) * 3.0) * wgt<double>(7);
                    g[k][8] = g[k][8] + ((0.0 - pe[xm]) * 3.0) * wgt<double>(8);
                } else {         // (0,1) from x, (1,1) from x - 1, (-1,1) from x + 1
                    g[k][2] = g[k][2] + ((0.0 - pe[x]) * 3.0) * wgt<double>(2);
                    g[k][5] = g[k][5] + ((0.0 - pe[xm]) * 3.0) * wgt<double>(5);
                    g[k][6] = g[k][6] + ((0.0 - pe[xp]) * 3.0) * wgt<double>(6);
                }
            }
            double fo[9], go[9], pr;
            node_update_f64<MODE, QF>(I, f[k], g[k], nb, qx, qy, fo, go, mom, pr);
            if (MODE != MODE_MOMENTS) {
#pragma unroll
                for (int i = 0; i < QF; ++i) put_pop<MODE>(rfo, fo_b, i * ps, selfd, fo[i]);
#pragma unroll
                for (int i = 0; i < 9; ++i) put_pop<MODE>(rgo, go_b, i * ps, selfd, go[i]);
                st(qb, self, make_double2(qx, qy));
                // the pressure of an edge row on an open side, for the populations that enter
                // through it at the next step
                if (!INTERIOR && ((y == 0 && I.bc_lo == BC_OPEN) ||
                                  (y == ny - 1 && I.bc_hi == BC_OPEN)))
                    st((double*)(mdst + I.off_mp), (y == 0 ? 0 : pitch) + x, pr);
            }
        }
        if (MODE == MODE_MOMENTS) {
            const int64_t n = (int64_t)nx * ny;
            const int64_t c = (int64_t)y * nx + x;
#pragma unroll
            for (int m = 0; m < 5; ++m) mom_out[m * n + c] = mom[m];
        }
    }
}


// A tile whose staged region (two nodes around it) lies inside the grid runs a copy of the
// body without wrap and boundary logic; edge tiles take the general path.  Tiles are
// TILE_X = 64 nodes wide (4K rows), except at the right end of an instance whose width is
// not a multiple of 64, where narrower tiles cover the rest: 32 wide (8K rows) or 16 wide
// (16K rows), width class 1 or 2 in TileDesc::pad.  The block's 256 threads then hold
// 2 or 4 rows per wavefront instead of lanes with no node.  Every tile shape fits the LDS
// arrays sized for the 64-wide one.
template <typename S, int K, bool PULL, int MODE, bool RING_FROM_PLANE, int QF,
          bool PERSIST = false>
__global__ __launch_bounds__(BLOCK) void k_step(
    const InstDev* __restrict__ insts, const TileDesc* __restrict__ tiles, int ntiles,
    int chunk, int stride, const S* __restrict__ fsrc, const S* __restrict__ gsrc, S* __restrict__ fdst,
    S* __restrict__ gdst, double* __restrict__ q,
    const typename Store<S>::C* __restrict__ phiplane, const float* __restrict__ msrc,
    float* __restrict__ mdst, double* __restrict__ mom_out) {
    using C = typename Store<S>::C;
    constexpr int TY = 4 * K;
    constexpr int NR = rest_deviation<S>() ? (TY + 4) * (TILE_X + 4) : 1;
    static_assert((8 * K + 4) * (TILE_X / 2 + 4) <= (TY + 4) * (TILE_X + 4) &&
                  (16 * K + 4) * (TILE_X / 4 + 4) <= (TY + 4) * (TILE_X + 4) &&
                  (8 * K + 2) * (TILE_X / 2 + 2) <= (TY + 2) * (TILE_X + 2) &&
                  (16 * K + 2) * (TILE_X / 4 + 2) <= (TY + 2) * (TILE_X + 2),
                  "narrow tiles fit the LDS arrays of the 64-wide tile");
    __shared__ C sphi[(TY + 2) * (TILE_X + 2)];
    // previous step's per-node terms with a two-node halo: (A, B, ux, uy) and (phi_w, H)
    __shared__ float4 sq[NR];
    __shared__ float2 sw[NR];

    const auto run = [&](int t) {
        const TileDesc T = tiles[t];
        const InstDev& I = insts[T.inst];
        const bool interior = PULL && T.pad == 0 && T.x0 >= 2 && T.x0 + TILE_X + 2 <= I.nx &&
                              T.y0 >= 2 && T.y0 + TY + 2 <= I.ny;
        if (interior)
            step_tile<S, K, PULL, MODE, RING_FROM_PLANE, true, QF, TILE_X>(
                I, T, fsrc, gsrc, fdst, gdst, q, phiplane, msrc, mdst, mom_out, sphi, sq, sw);
        else if (T.pad == 0)
            step_tile<S, K, PULL, MODE, RING_FROM_PLANE, false, QF, TILE_X>(
                I, T, fsrc, gsrc, fdst, gdst, q, phiplane, msrc, mdst, mom_out, sphi, sq, sw);
        else if (T.pad == 1)
            step_tile<S, K, PULL, MODE, RING_FROM_PLANE, false, QF, TILE_X / 2>(
                I, T, fsrc, gsrc, fdst, gdst, q, phiplane, msrc, mdst, mom_out, sphi, sq, sw);
        else
            step_tile<S, K, PULL, MODE, RING_FROM_PLANE, false, QF, TILE_X / 4>(
                I, T, fsrc, gsrc, fdst, gdst, q, phiplane, msrc, mdst, mom_out, sphi, sq, sw);
    };
    const int b = blockIdx.x;
    if constexpr (!PERSIST) {
        // one tile per block (a loop here, even of one pass, costs the compiler 15 to 35
        // more registers)
        const int xcd = b % NXCD, j = b / NXCD, jc = j / chunk;
        const int t = (jc * NXCD + xcd) * chunk + (j - jc * chunk);
        if (t < ntiles) run(t);
    } else {
        const int xcd = b % NXCD;
        for (int j = b / NXCD; j < chunk; j += stride) {
            const int t = xcd * chunk + j;
            if (t >= ntiles) return;
            run(t);
            if (j + stride < chunk) __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ split step: phi plane
// First half of the two-launch step: phi (Eq. 12) of every node from the pulled f, with the
// same arithmetic as the fused kernel (source-node phi read from memory, not LDS).
template <typename S, int K, int QF>
__global__ __launch_bounds__(BLOCK) void k_phi_plane(
    const InstDev* __restrict__ insts, const TileDesc* __restrict__ tiles, int ntiles,
    int per_xcd, const S* __restrict__ fsrc, const float* __restrict__ msrc,
    typename Store<S>::C* __restrict__ phiplane) {
    using C = typename Store<S>::C;
    constexpr bool REF = rest_deviation<S>();
    const int b = blockIdx.x;
    const int t = (b % NXCD) * per_xcd + b / NXCD;
    if (t >= ntiles) return;
    const TileDesc T = tiles[t];
    const InstDev& I = insts[T.inst];
    // tile width 64 >> T.pad, with 256 / width rows of threads (see k_step)
    const int txw = TILE_X >> T.pad, rpg = BLOCK / txw;
    const int w = min(txw, I.nx - T.x0);
    const int h = min(rpg * K, I.ny - T.y0);
    const int lx = threadIdx.x & (txw - 1);
    const int ly = threadIdx.x >> (6 - T.pad);
    const S* fb = fsrc + I.off_dist;
    // phi_w, the first component of each node's state (3 or 4 floats)
    constexpr int NSF = state_floats<S>();
    const float* rb = REF ? msrc + I.off_mp : nullptr;
    const C isf = C(I.f_inv_scale_f);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int yl = ly + rpg * k;
        if (lx < w && yl < h) {
            const int x = T.x0 + lx, y = T.y0 + yl;
            int o[9], src[9];
            pull_offsets<S, true>(I, x, y, o, src);
            C v[9], ref[9], base = C(0);
#pragma unroll
            for (int i = 0; i < QF; ++i) v[i] = Store<S>::get(fb, o[i]);
            if (REF) {
#pragma unroll
                for (int i = 0; i < QF; ++i) ref[i] = rb[(int64_t)src[i] * NSF];
                base = rb[(int64_t)(y * I.pitch + x) * NSF];
            }
            phiplane[I.off_phi + y * I.pitch + x] =
                phi_of<C, REF, QF, (sizeof(S) < sizeof(float))>(v, ref, base, isf);
        }
    }
}

// ------------------------------------------------------------------ initial state
__device__ __forceinline__ double init_feq(double w, double ph, double cu) {
#pragma clang fp contract(off)
    return w * ph * (1.0 + cu * 3.0);
}
__device__ __forceinline__ double init_rho(double ph, double drho, double rho_g) {
#pragma clang fp contract(off)
    return ph * drho + rho_g;
}

// f = f^eq(phi0, u0) (Eq. 9), g = g^eq(p = 0, u0) with rho(phi0) (Eq. 16), phi u = phi0 u0,
// in the storage format, already in streamed form (FP64: q planes; reduced formats: the
// per-node phi_w, u_w (and p_w = 0 in the 16-bit format) and deviations from them).
template <typename S, int QF>
__global__ __launch_bounds__(BLOCK) void k_init(const InstDev* __restrict__ insts, int inst,
                                                const double* __restrict__ phi0,
                                                const double* __restrict__ ux0,
                                                const double* __restrict__ uy0,
                                                S* __restrict__ f, S* __restrict__ g,
                                                double* __restrict__ q, float* __restrict__ mp) {
    using C = typename Store<S>::C;
    constexpr bool REF = rest_deviation<S>();
    const InstDev& I = insts[inst];
    const int x = blockIdx.x * TILE_X + (threadIdx.x & (TILE_X - 1));
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= I.nx || y >= I.ny) return;
    const int c = y * I.nx + x;
    const double ph = phi0[c], ux = ux0[c], uy = uy0[c];
    const double rho = init_rho(ph, I.drho, I.rho_g);
    const int self = y * I.pitch + x;                  // per-node state
    const int selfd = y * row_stride<S>(I) + x;        // distributions
    const int ps = pop_stride<S>(I);
    S* fb = f + I.off_dist;
    S* gb = g + I.off_dist;
    const float phw = (float)ph, uxw = (float)ux, uyw = (float)uy;
    const RefTerms R = ref_terms(I, phw, 0.0f, uxw, uyw);
#pragma unroll
    for (int i = 0; i < QF; ++i) {
        const double w = wf<double, QF>(i);
        const double cu = CX[i] * ux + CY[i] * uy;
        const double fe = init_feq(w, ph, cu);
        if (REF) {
            const double ed = fe - w * (double)phw;
            Store<S>::put(fb, i * ps + selfd, (float)ed * I.f_scale_f);
        } else {
            Store<S>::put(fb, i * ps + selfd, (C)fe);
        }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double ge = rho * s_exact(i, ux, uy);   // p = 0
        if (REF) {
            const double eg = ge - (double)geq_ref(i, R.A, R.B, uxw, uyw, R.H);
            Store<S>::put(gb, i * ps + selfd, (float)eg * I.f_scale_g);
        } else {
            Store<S>::put(gb, i * ps + selfd, (C)ge);
        }
    }
    if constexpr (ref_has_p<S>()) {
        ((float4*)(mp + I.off_mp))[self] = make_float4(phw, 0.0f, uxw, uyw);
    } else if constexpr (REF) {
        // the edge-pressure rows after the nodes' state start at p = 0 (cleared at set-up)
        ((float3*)(mp + I.off_mp))[self] = make_float3(phw, uxw, uyw);
    } else {
        ((double2*)(q + I.off_q))[self] = make_double2(ph * ux, ph * uy);
    }
}

// ------------------------------------------------------------------ launchers
namespace {
inline int grid_for(int ntiles, int& per_xcd) {
    per_xcd = (ntiles + NXCD - 1) / NXCD;
    return per_xcd * NXCD;
}

// one block per tile, the tiles dealt to the XCDs in chunks of `chunk` (0 or at least
// ntiles / 8: one band per XCD); returns the grid and sets the chunk the kernel takes
inline int grid_dealt(int ntiles, int chunk, int& ch) {
    int per;
    const int g = grid_for(ntiles, per);
    if (chunk <= 0 || chunk >= per) {
        ch = per;
        return g;
    }
    ch = chunk;
    return (ntiles + NXCD * chunk - 1) / (NXCD * chunk) * (NXCD * chunk);
}

template <typename S, int K, int QF>
hipError_t step_k(const StepArgs& a) {
    using C = typename Store<S>::C;
    int per;
    const int tile_grid = grid_for(a.ntiles, per);  // one block per tile, a band per XCD
    int ch;
    const int dealt_grid = grid_dealt(a.ntiles, a.chunk, ch);  // one block per tile, dealt
    // persistent grid (fused pull step only): a.persist blocks per XCD, each looping over
    // that XCD's tiles
    int stride = per;
    if (a.persist > 0 && a.persist < per) stride = a.persist;
    const int grid = NXCD * stride;
    const S* fs = (const S*)a.fsrc;
    const S* gs = (const S*)a.gsrc;
    S* fd = (S*)a.fdst;
    S* gd = (S*)a.gdst;
    double* q = (double*)a.q;
    C* ph = (C*)a.phiplane;
    const float* rs = (const float*)a.rsrc;
    float* rd = (float*)a.rdst;
    if (!a.pull) {
        k_step<S, K, false, MODE_STEP, false, QF><<<tile_grid, BLOCK, 0, a.stream>>>(
            a.insts, a.tiles, a.ntiles, per, per, fs, gs, fd, gd, q, ph, rs, rd, nullptr);
    } else if (a.split) {
        k_phi_plane<S, K, QF><<<tile_grid, BLOCK, 0, a.stream>>>(a.insts, a.tiles, a.ntiles, per,
                                                                 fs, rs, ph);
        if (a.nt_store)
            k_step<S, K, true, MODE_STEP_NT, true, QF><<<dealt_grid, BLOCK, 0, a.stream>>>(
                a.insts, a.tiles, a.ntiles, ch, ch, fs, gs, fd, gd, q, ph, rs, rd, nullptr);
        else
            k_step<S, K, true, MODE_STEP, true, QF><<<dealt_grid, BLOCK, 0, a.stream>>>(
                a.insts, a.tiles, a.ntiles, ch, ch, fs, gs, fd, gd, q, ph, rs, rd, nullptr);
    } else if (stride < per) {
        // fused step on a persistent grid
        if (a.nt_store)
            k_step<S, K, true, MODE_STEP_NT, false, QF, true><<<grid, BLOCK, 0, a.stream>>>(
                a.insts, a.tiles, a.ntiles, per, stride, fs, gs, fd, gd, q, ph, rs, rd, nullptr);
        else
            k_step<S, K, true, MODE_STEP, false, QF, true><<<grid, BLOCK, 0, a.stream>>>(
                a.insts, a.tiles, a.ntiles, per, stride, fs, gs, fd, gd, q, ph, rs, rd, nullptr);
    } else if (a.nt_store) {
        k_step<S, K, true, MODE_STEP_NT, false, QF><<<dealt_grid, BLOCK, 0, a.stream>>>(
            a.insts, a.tiles, a.ntiles, ch, ch, fs, gs, fd, gd, q, ph, rs, rd, nullptr);
    } else {
        k_step<S, K, true, MODE_STEP, false, QF><<<dealt_grid, BLOCK, 0, a.stream>>>(
            a.insts, a.tiles, a.ntiles, ch, ch, fs, gs, fd, gd, q, ph, rs, rd, nullptr);
    }
    return hipGetLastError();
}

template <typename S, int QF>
hipError_t step_s(const StepArgs& a) {
    switch (a.tile_rows) {
        case 4: return step_k<S, 1, QF>(a);
        case 8: return step_k<S, 2, QF>(a);
        case 16: return step_k<S, 4, QF>(a);
        default: return hipErrorInvalidValue;
    }
}

template <typename S, int QF>
hipError_t moments_s(const StepArgs& a, double* out) {
    int per;
    const int grid = grid_for(a.ntiles, per);
    const S* fs = (const S*)a.fsrc;
    const S* gs = (const S*)a.gsrc;
    const float* rs = (const float*)a.rsrc;
    if (a.pull)
        k_step<S, 1, true, MODE_MOMENTS, false, QF><<<grid, BLOCK, 0, a.stream>>>(
            a.insts, a.tiles, a.ntiles, per, per, fs, gs, nullptr, nullptr, (double*)a.q,
            nullptr, rs, nullptr, out);
    else
        k_step<S, 1, false, MODE_MOMENTS, false, QF><<<grid, BLOCK, 0, a.stream>>>(
            a.insts, a.tiles, a.ntiles, per, per, fs, gs, nullptr, nullptr, (double*)a.q,
            nullptr, rs, nullptr, out);
    return hipGetLastError();
}

template <typename S, int QF>
hipError_t init_s(const InstDev* insts, int inst, int nx, int ny, const double* phi0,
                  const double* ux0, const double* uy0, void* f, void* g, void* q, void* rplane,
                  hipStream_t st) {
    dim3 grid((nx + TILE_X - 1) / TILE_X, (ny + 3) / 4);
    k_init<S, QF><<<grid, BLOCK, 0, st>>>(insts, inst, phi0, ux0, uy0, (S*)f, (S*)g,
                                          (double*)q, (float*)rplane);
    return hipGetLastError();
}

template <typename S>
hipError_t step_q(const StepArgs& a) {
    return a.qf == 5 ? step_s<S, 5>(a) : step_s<S, 9>(a);
}
template <typename S>
hipError_t moments_q(const StepArgs& a, double* out) {
    return a.qf == 5 ? moments_s<S, 5>(a, out) : moments_s<S, 9>(a, out);
}
template <typename S>
hipError_t init_q(int qf, const InstDev* insts, int inst, int nx, int ny, const double* phi0,
                  const double* ux0, const double* uy0, void* f, void* g, void* q, void* rplane,
                  hipStream_t st) {
    return qf == 5 ? init_s<S, 5>(insts, inst, nx, ny, phi0, ux0, uy0, f, g, q, rplane, st)
                   : init_s<S, 9>(insts, inst, nx, ny, phi0, ux0, uy0, f, g, q, rplane, st);
}
// resident blocks per compute unit of the fused pull-step kernel on a persistent grid
template <typename S, int K, int QF>
int occ_k(bool nt) {
    int nb = 0;
    const hipError_t e =
        nt ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                 &nb, k_step<S, K, true, MODE_STEP_NT, false, QF, true>, BLOCK, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                 &nb, k_step<S, K, true, MODE_STEP, false, QF, true>, BLOCK, 0);
    return e == hipSuccess ? nb : 0;
}

template <typename S, int QF>
int occ_s(int rows, bool nt) {
    switch (rows) {
        case 4: return occ_k<S, 1, QF>(nt);
        case 8: return occ_k<S, 2, QF>(nt);
        case 16: return occ_k<S, 4, QF>(nt);
        default: return 0;
    }
}

template <typename S>
int occ_q(int qf, int rows, bool nt) {
    return qf == 5 ? occ_s<S, 5>(rows, nt) : occ_s<S, 9>(rows, nt);
}

}  // namespace

int step_blocks_per_cu(int storage, int qf, int rows, bool nt) {
    switch (storage) {
        case STORE_F64: return occ_q<double>(qf, rows, nt);
        case STORE_F32: return occ_q<float>(qf, rows, nt);
        case STORE_F16: return occ_q<_Float16>(qf, rows, nt);
        default: return 0;
    }
}

hipError_t launch_step(int storage, const StepArgs& a) {
    if (a.qf != 5 && a.qf != 9) return hipErrorInvalidValue;
    switch (storage) {
        case STORE_F64: return step_q<double>(a);
        case STORE_F32: return step_q<float>(a);
        case STORE_F16: return step_q<_Float16>(a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_moments(int storage, const StepArgs& a, double* out) {
    if (a.qf != 5 && a.qf != 9) return hipErrorInvalidValue;
    switch (storage) {
        case STORE_F64: return moments_q<double>(a, out);
        case STORE_F32: return moments_q<float>(a, out);
        case STORE_F16: return moments_q<_Float16>(a, out);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(int storage, int qf, const InstDev* insts, int inst, int nx, int ny,
                       const double* phi0, const double* ux0, const double* uy0, void* f, void* g,
                       void* q, void* rplane, hipStream_t st) {
    if (qf != 5 && qf != 9) return hipErrorInvalidValue;
    switch (storage) {
        case STORE_F64:
            return init_q<double>(qf, insts, inst, nx, ny, phi0, ux0, uy0, f, g, q, rplane, st);
        case STORE_F32:
            return init_q<float>(qf, insts, inst, nx, ny, phi0, ux0, uy0, f, g, q, rplane, st);
        case STORE_F16:
            return init_q<_Float16>(qf, insts, inst, nx, ny, phi0, ux0, uy0, f, g, q, rplane, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
