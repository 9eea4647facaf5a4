// Device-side data structures shared by the kernels and the host runtime of liblbm_hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_OPEN = 2 };
enum { VISC_LINEAR = 0, VISC_INVERSE = 1, VISC_STEP_MU = 2 };
enum { GRAD_ISOTROPIC = 0, GRAD_LOCAL_NEQ = 1 };
enum { STORE_F64 = 0, STORE_F32 = 1, STORE_F16 = 2 };

constexpr int TILE_X = 64;      // tile width = one wavefront of 64 lanes
constexpr int BLOCK = 256;      // 4 wavefronts; a tile row group is 4 rows
constexpr int NXCD = 8;         // MI355X: 8 accelerator complex dies, each with its own L2
constexpr int REDUCE_SLOTS = 13;        // FP64 partial sums per block of the reductions
constexpr int REDUCE_MAX_BLOCKS = 1024; // blocks of the partial pass at most

// Per-instance constants, read with uniform (scalar) loads.  Distances are in elements.
struct InstDev {
    int32_t nx, ny, pitch, bc_lo, bc_hi, visc_law, grad_scheme;
    int64_t off_dist;   // offset of this instance's distributions in the f and g arrays:
                        // 9 * plane elements, [y][i][x] (FP64, FP32) or [i][y][x] (16-bit)
    int64_t off_q;      // FP64 format: offset of its two (phi u) planes in the q array
    int64_t off_phi;    // offset of its phi plane (split kernel)
    int64_t off_mp;     // offset (in floats) of its per-node state: 16-bit format, a float4
                        // (phi_w, p_w, ux_w, uy_w) per node; FP32, a float3 (phi_w, ux_w,
                        // uy_w) per node, then two rows of floats holding the pressure of the
                        // first and the last row (open sides); FP64, only those two rows, of
                        // doubles
    int64_t plane;      // ny * pitch
    double rho_l, rho_g, drho;      // drho = rho_l - rho_g
    double nu_l, nu_g, inv_nu_l, inv_nu_g, mu_l, mu_g;
    double kappa, beta, W, inv_w;   // k = 1.5 sigma W, beta = 12 sigma / W, W, 1 / W
    double tau_f, inv_tau_f, cf;    // tau_phi, 1 / tau_phi and 1 - 1 / (2 tau_phi)
    double Gx, Gy;
    double scale_f, inv_scale_f, scale_g, inv_scale_g;  // storage scales 2^exp
    // FP32 copies for the reduced formats' arithmetic, each rounded on the host from the FP64
    // expression the kernels would otherwise round in every lane (the same bits): 4 beta,
    // kappa, 1 / W, nu_l - nu_g, nu_g, 1/nu_l - 1/nu_g, 1/nu_g, mu_l, mu_g, Gx, Gy, 1/tau_phi,
    // 1 - 1/(2 tau_phi), rho_l - rho_g, rho_g and the four storage scales
    float f_beta4, f_kappa, f_inv_w, f_dnu, f_nu_g, f_dinv_nu, f_inv_nu_g, f_mu_l, f_mu_g;
    float f_Gx, f_Gy, f_inv_tau_f, f_cf, f_drho, f_rho_g;
    float f_scale_f, f_inv_scale_f, f_scale_g, f_inv_scale_g;
};

// One tile of one instance: origin (x0, y0) and width class pad: 0 for TILE_X nodes wide
// and 4K rows (K = rows per thread), 1 for TILE_X / 2 wide and 8K rows, 2 for TILE_X / 4 wide
// and 16K rows (the last columns of an instance whose width is not a multiple of TILE_X).
struct TileDesc {
    int32_t inst, x0, y0, pad;
};

}  // namespace lbm

namespace lbm {

// Arguments of one step launch over a tile list.
struct StepArgs {
    const InstDev* insts;
    const TileDesc* tiles;
    int ntiles;
    int tile_rows;      // 4, 8 or 16
    int qf;             // velocities of the phase-field lattice: 9 (D2Q9) or 5 (D2Q5)
    bool pull;          // false only for the first step (initial state in streamed form)
    bool split;         // two launches: phi plane, then stencil + collide
    bool nt_store;      // non-temporal population stores
    int persist;        // > 0: persistent grid of that many blocks per XCD, each looping over
                        // tiles; 0: one block per tile
    int chunk;          // one block per tile: the tiles go to the XCDs in chunks of this
                        // many consecutive tiles, in turn; 0: one contiguous band per XCD
    const void* fsrc;
    const void* gsrc;
    void* fdst;
    void* gdst;
    void* q;
    void* phiplane;     // split step: phi of the current step
    const void* rsrc;   // reduced formats: per-node (phi_w, p_w, u_w) of the previous step
    void* rdst;         // and of this step
    hipStream_t stream;
};

hipError_t launch_step(int storage, const StepArgs& a);
// resident blocks per compute unit of the fused step kernel (0 if the runtime cannot say)
int step_blocks_per_cu(int storage, int qf, int rows, bool nt);
hipError_t launch_moments(int storage, const StepArgs& a, double* out);
hipError_t launch_init(int storage, int qf, const InstDev* insts, int inst, int nx, int ny,
                       const double* phi0, const double* ux0, const double* uy0, void* f, void* g,
                       void* q, void* rplane, hipStream_t st);
int reduce_blocks(int64_t n);
hipError_t launch_reduce(const double* mom, int nx, int ny, int periodic_y, const double* mask,
                         double* partials, double* out, hipStream_t st);

}  // namespace lbm
