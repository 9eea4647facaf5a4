/*
 * lbm.h -- C-ABI of the MI355X (gfx950) phase-field lattice Boltzmann library.
 *
 * The library advances the two coupled lattices of Liang et al., "Phase-field-based lattice
 * Boltzmann modeling of large-density-ratio two-phase flows" (arXiv:1710.09541):
 *   f_i  conservative Allen-Cahn equation for the order parameter phi  (Sec. 2.2, Eqs. 8-14;
 *        D2Q9, or D2Q5, which the section also admits)
 *   g_i  incompressible Navier-Stokes with the forcing distribution G_i (Sec. 2.3, Eqs. 15-28;
 *        D2Q9)
 * on one GPU, for one or many independent instances ("batch") at once.
 *
 * Problem statement (Sec. 2.1 and the set-ups of Sec. 3): a 2D nx x ny lattice with
 * dx = dt = 1, x always periodic, each y side periodic, a half-way bounce-back wall or an
 * open side; phase densities rho_l, rho_g, viscosities nu_l, nu_g with a
 * viscosity law (Eqs. 24-26), surface tension sigma, interface width W, mobility M, a
 * uniform body-force density G = (Gx, Gy); initial phi(x, y) and u(x, y).
 *
 * Conventions
 *   - Fields on the host are double, row-major [ny][nx] (x fastest).  Node (i, j) sits at the
 *     cell centre (i + 0.5, j + 0.5); a wall lies on the domain edge y = 0 or y = ny.
 *   - All calls return LBM_OK (0) or a negative LBM_ERR_* code; lbm_last_error() gives the
 *     message.  Parameters are validated before any device call, so a bad parameter set is
 *     reported as LBM_ERR_PARAM even on a machine without a GPU.
 *   - Kernel faults surface at the next synchronising call as LBM_ERR_DEVICE.
 *   - lbm_step is stream-ordered and returns before the work completes; lbm_moments,
 *     lbm_reduce and the state calls synchronise the library's stream.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx; /* opaque; owned by the library until lbm_destroy */

enum {
    LBM_OK = 0,
    LBM_ERR_PARAM = -1,     /* invalid parameter or argument */
    LBM_ERR_ALLOC = -2,     /* host or device allocation failed */
    LBM_ERR_DEVICE = -3,    /* HIP runtime error (no device, launch failure, fault) */
    LBM_ERR_NONFINITE = -4, /* a non-finite value was found by a periodic check */
    LBM_ERR_RANGE = -5      /* index or size out of range */
};

/* y boundary of one side (x is always periodic).  PERIODIC wraps.  WALL is half-way
 * bounce-back half a node beyond the edge row, for f and g alike (Sec. 3.2, the channel
 * walls; Sec. 3.4, the impact's floor).  OPEN is the open boundary of the impact's top
 * (Sec. 3.4), for which the paper gives no formula; it is read as a pressure outlet: one
 * node beyond the edge row the pressure is the ambient p = 0 (the reference pressure of
 * the initial state), and phi and u have zero normal gradient.  In the manner of the
 * non-equilibrium extrapolation of Guo, Zheng & Shi (2002), a population i entering the
 * edge row at x is what the edge node s = (x - c_ix, edge) sent out in direction i, with,
 * for g, the pressure part of its equilibrium (Eq. 16) moved from p(s) to 0:
 *   f_i = f*_i(s),   g_i = g*_i(s) + (0 - p(s)) w_i / c_s^2.
 * The stencil's ghost row at a wall or an open side mirrors the edge row. */
enum { LBM_BC_PERIODIC = 0, LBM_BC_WALL = 1, LBM_BC_OPEN = 2 };

/* viscosity law: Eq. 24 nu linear in phi; Eq. 25 1/nu linear in phi; Eq. 26 step in the
 * dynamic viscosity (mu_l for phi >= 0.5, else mu_g) with nu = mu / rho(phi) */
enum { LBM_VISC_LINEAR = 0, LBM_VISC_INVERSE = 1, LBM_VISC_STEP_MU = 2 };

/* interface normal n in the phase-field source F_i (Eq. 11).  ISOTROPIC: n = grad phi /
 * |grad phi| from the isotropic stencil of Eq. 27 (Eq. 2).  LOCAL_NEQ: the local
 * non-equilibrium scheme of Eq. 29, which reduces exactly to n = -C / |C| with
 * C = sum_i c_i (f_i - f_i^eq) + d_t(phi u) / 2.  Either way n = 0 where the magnitude
 * (|grad phi| or |C|) does not exceed 1e-12.  The chemical potential, the force and the
 * moments always use Eqs. 27-28. */
enum { LBM_GRAD_ISOTROPIC = 0, LBM_GRAD_LOCAL_NEQ = 1 };

/* velocity set of the phase-field lattice f (Sec. 2.2 admits either): D2Q9 (the paper's
 * choice, weights 4/9, 1/9, 1/36) or D2Q5 (the rest and the four axis velocities, weights
 * 1/3 and 1/6, the same c_s^2 = 1/3).  0 selects D2Q9.  The flow lattice g and the
 * stencils of Eqs. 27-28 are D2Q9 in either case.  Every instance of a context uses the
 * same set. */
enum { LBM_LATTICE_D2Q9 = 9, LBM_LATTICE_D2Q5 = 5 };

/* storage of the distributions.  F64: doubles, FP64 arithmetic.  F32 / F16: float / IEEE
 * half holding rest deviations (f_i - w_i phi_w) 2^exp_f, phi_w the order parameter of the
 * node that wrote the slot, and deviations of g_i from the flow equilibrium (Eq. 16) of that
 * node's published phi_w, u_w (and, F16 only, p_w), times 2^exp_g; those published values
 * are kept per node in FP32 (12 bytes per node in F32, 16 in F16).  Arithmetic in FP32;
 * F32 forms phi-to-rho and the velocity and pressure moments (Eqs. 13, 22) in FP64. */
enum { LBM_STORE_F64 = 0, LBM_STORE_F32 = 1, LBM_STORE_F16 = 2 };

/* population stores of the step: AUTO lets the autotuner choose; CACHED are ordinary
 * stores; STREAMING are non-temporal stores that do not allocate in the caches (they pay
 * when the working set exceeds the last-level cache, 256 MB on MI355X, and cost when it
 * fits).  Results are bitwise identical either way. */
enum { LBM_STORES_AUTO = 0, LBM_STORES_CACHED = 1, LBM_STORES_STREAMING = 2 };

/* Launch grid of the fused step kernel: one block per tile, or a persistent grid of as many
 * blocks as stay resident on the GPU (or, if the environment variable LBM_PERSIST_BLOCKS is
 * set at lbm_init, that many blocks per XCD), each looping over a contiguous run of tiles.
 * The split kernel and the first step always run one block per tile, as does a persistent
 * grid with at least as many blocks as tiles.  Results are bitwise identical either way.
 * AUTO runs one block per tile: the persistent grid measured 3-14 % slower on every workload
 * and format on MI355X (the loop costs registers, and the hardware dispatcher balances the
 * tiles better than a fixed assignment). */
enum { LBM_GRID_AUTO = 0, LBM_GRID_TILES = 1, LBM_GRID_PERSISTENT = 2 };

/* Order of the tiles within each instance: whole rows of tiles one after the other, or
 * vertical strips 8 or 16 tiles (512 or 1024 nodes) wide, row after row inside a strip.
 * Strips keep the halo rows a tile re-reads in the L2 cache when the grid is much larger
 * than the caches; whole rows win where it fits.  Results are bitwise identical. */
enum { LBM_STRIP_AUTO = 0, LBM_STRIP_ROWS = -1 };   /* or a strip width of 8 or 16 tiles */

/* Tiles at the right end of an instance whose width is not a multiple of 64.  Tiles are 64
 * nodes wide; with narrow tiles ON, the last nx mod 64 = r columns (r <= 48) are covered by
 * 32- and/or 16-wide tiles, 2 or 4 times as tall, so fewer of the block's threads hold no
 * node (the step's time follows the threads launched, not the nodes).  AUTO lets the
 * autotuner time both where they differ.  Results are bitwise identical either way. */
enum { LBM_NARROW_AUTO = 0, LBM_NARROW_OFF = -1, LBM_NARROW_ON = 1 };

/* How the step's tiles are dealt to the 8 XCDs of MI355X (each with its own L2), one block
 * per tile.  BANDS: each XCD takes one contiguous eighth of the tile list, so it finds the
 * halo rows of its previous tiles in its own L2: the best order for one large grid.  A chunk
 * of n tiles (1 to 4096): the XCDs take chunks of n consecutive tiles in turn, which evens
 * out their work when tile costs vary along the list (a batch of instances of different
 * shapes).  AUTO lets the autotuner time bands against chunks of 16 tiles.  A persistent
 * grid always runs bands.  Results are bitwise identical either way. */
enum { LBM_DEAL_AUTO = 0, LBM_DEAL_BANDS = -1 };

/* kernel choice for the step */
enum {
    LBM_KERNEL_AUTO = 0,  /* the autotuner picks */
    LBM_KERNEL_FUSED = 1, /* one launch per step: pull-stream, phi tile with recomputed halo
                             in LDS, stencil, closure, moments, collide, store */
    LBM_KERNEL_SPLIT = 2  /* two launches per step: phi plane, then stencil + collide */
};

#define LBM_EXP_AUTO (-1000) /* let the library choose a storage exponent */

/* Per-instance problem parameters. */
typedef struct {
    int32_t nx, ny;           /* lattice size, each >= 3; one instance's 9 populations of a
                                 lattice (9 x ny x nx rounded up to 64) must stay below 4 GiB
                                 in the chosen storage (FP64: about 7700 x 7700 nodes) */
    int32_t bc_ylo, bc_yhi;   /* LBM_BC_*; PERIODIC must be set on both sides or on neither */
    int32_t visc_law;         /* LBM_VISC_* */
    int32_t grad_scheme;      /* LBM_GRAD_* */
    double rho_l, rho_g;      /* phase densities, > 0 (Eq. 13) */
    double nu_l, nu_g;        /* phase kinematic viscosities, > 0 */
    double sigma;             /* surface tension, >= 0 (Eq. 7) */
    double W;                 /* interface width, > 0 (Eqs. 3, 7) */
    double M;                 /* mobility, > 0; tau_phi = M / c_s^2 + 0.5 (Eq. 14) */
    double Gx, Gy;            /* body-force density (Eq. 4b) */
    int32_t exp_f, exp_g;     /* F16 storage exponents (stored value = deviation * 2^exp), or
                                 LBM_EXP_AUTO to derive them from the initial fields;
                                 ignored for F32 and F64 */
    int32_t f_lattice;        /* LBM_LATTICE_D2Q9 (or 0) or LBM_LATTICE_D2Q5 */
    int32_t reserved1;
} lbm_params;

/* Context-wide options. */
typedef struct {
    int32_t storage;          /* LBM_STORE_*, the same for every instance */
    int32_t kernel;           /* LBM_KERNEL_* */
    int32_t tile_rows;        /* rows per fused-kernel tile (4, 8 or 16); 0 = autotune/default */
    int32_t use_graph;        /* 1: lbm_step replays captured HIP graphs of 64, 16 and 2 steps */
    int32_t check_every;      /* > 0: every that many steps lbm_step checks for non-finite
                                 values and returns LBM_ERR_NONFINITE (synchronises) */
    int32_t stores;           /* LBM_STORES_* (with kernel / tile_rows AUTO or 0 the choice is
                                 timed at lbm_init; if the environment variable
                                 LBM_AUTOTUNE_CACHE names a file, choices are read from and
                                 appended to it, keyed by GPU, storage, lattice, options and
                                 grid sizes) */
    int32_t grid;             /* LBM_GRID_* (AUTO: one block per tile) */
    int32_t strip;            /* LBM_STRIP_AUTO (timed at lbm_init), LBM_STRIP_ROWS, 8 or 16 */
    int32_t narrow_tiles;     /* LBM_NARROW_AUTO (timed at lbm_init), LBM_NARROW_OFF or _ON */
    int32_t deal;             /* LBM_DEAL_AUTO (timed at lbm_init), LBM_DEAL_BANDS or a chunk
                                 of 1 to 4096 tiles */
} lbm_options;

/* Integral diagnostics of one instance, FP64 accumulation in a fixed order, over the
 * fields lbm_moments returns (phi, rho, p, u of Eqs. 12, 13, 22).  Sums and extrema run
 * over all nx * ny nodes. */
typedef struct {
    double sum_phi;             /* sum of phi: conserved by the collision and streaming of f
                                   (sum_i f_i^eq = phi and sum_i F_i = 0, Eqs. 9, 11, 12; the
                                   mass-conservation remark closing Sec. 2) with periodic and
                                   wall sides; an open side changes it by what crosses it */
    double sum_rho;             /* sum of rho (Eq. 13) */
    double kinetic;             /* sum of rho |u|^2 / 2 */
    double max_u;               /* max |u|: the spurious velocity of the static drop,
                                   Sec. 3.1 */
    double min_rho;             /* min rho: rho(phi) falls below rho_g where phi < 0 */
    double min_phi, max_phi;    /* extrema of phi (Sec. 2.2: 0 gas, 1 liquid) */
    double p_in, p_out;         /* mean p inside r < r_in / outside r > r_out of (xc, yc),
                                   periodic distance; 0 if the set is empty.  p_in - p_out
                                   is the static drop's pressure jump (Sec. 3.1), against
                                   sigma / R by the Young-Laplace law */
    double interface_crossings; /* x- and y-neighbour pairs on different sides of phi = 0.5
                                   (the interface of Sec. 2.2); the spinodal's length scale
                                   (Sec. 3.3) is 2 nx ny / interface_crossings */
    double spread_radius;       /* the impact's spreading radius r (Sec. 3.4, where
                                   r / D = C (U t / D)^1/2): on row y_row, max |x* - xc| over
                                   the crossings x* of phi = 0.5 between x-neighbours,
                                   linearly interpolated; 0 if none.  The paper does not
                                   define r; the row read is H_w + W above the floor */
    int64_t nonfinite;          /* nodes with a non-finite phi, rho, p or u */
    int64_t step;               /* steps taken so far */
} lbm_diag;

/* Creates a context of n_inst instances.  p[k] are the parameters of instance k; phi0[k],
 * ux0[k], uy0[k] its initial fields (host, double, [ny][nx]), copied during the call.
 * The initial distributions are the equilibria f = f^eq(phi0, u0) (Eq. 9) and
 * g = g^eq(p = 0, u0) (Eq. 16) with rho = rho(phi0), and phi u of the previous step is
 * phi0 u0.  opt may be NULL (F32 storage, every choice autotuned, graphs on).  hip_stream
 * is a hipStream_t the work is ordered on (NULL: the library creates its own).
 * On success *out receives the context. */
int lbm_init(const lbm_params* p, int32_t n_inst, const lbm_options* opt,
             const double* const* phi0, const double* const* ux0, const double* const* uy0,
             void* hip_stream, lbm_ctx** out);

/* Advances every instance by nsteps >= 0 time steps (Eqs. 8 and 15, collide then stream).
 * Stream-ordered: returns before completion unless check_every > 0. */
int lbm_step(lbm_ctx* c, int64_t nsteps);

/* Macroscopic fields of instance inst on the current state: phi (Eq. 12), rho (Eq. 13),
 * p (Eq. 22b), u (Eq. 22a) -- exactly the values the next collision uses.  Host buffers of
 * nx*ny doubles each, [ny][nx]; any may be NULL.  Synchronises. */
int lbm_moments(lbm_ctx* c, int32_t inst, double* phi, double* rho, double* p, double* ux,
                double* uy);

/* Same, into a caller-owned device buffer of 5*nx*ny doubles laid out as the planes
 * phi, rho, p, ux, uy.  Stream-ordered, does not synchronise. */
int lbm_moments_device(lbm_ctx* c, int32_t inst, double* d_out5);

/* Integral diagnostics of instance inst (the quantities through which Sec. 3 reads its
 * four experiments: sum phi, the static drop's pressure jump and spurious velocity
 * (Sec. 3.1), the spinodal's interface length (Sec. 3.3), the impact's spreading radius
 * (Sec. 3.4); see lbm_diag) on the current state.  mask = {xc, yc, r_in, r_out, y_row}, five
 * host doubles (may be NULL: all zero, and y_row < 0 disables the spreading radius); out is
 * a caller-owned host struct.  Uses the moment and reduction buffers the context allocated
 * at lbm_init.  LBM_ERR_PARAM if c or out is NULL, LBM_ERR_RANGE for a bad inst,
 * LBM_ERR_DEVICE on a HIP error.  Synchronises. */
int lbm_reduce(lbm_ctx* c, int32_t inst, const double* mask, lbm_diag* out);

/* lbm_reduce for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same diagnostics, bit for bit,
 * from the same kernels, but the moment planes, partials and result go to a fixed device
 * scratch array the library holds on each GPU from its load until the process ends
 * (42 MB: five FP64 planes of at most 1,048,576 nodes, plus 13,312 partials).  The call
 * itself allocates nothing: no hipMalloc, hipFree or allocating library routine (the
 * scratch address is looked up once per GPU at lbm_init, and the pinned host result buffer
 * is the context's own from lbm_init).  LBM_ERR_RANGE for an instance of more than
 * 1,048,576 nodes (nothing is computed), otherwise as lbm_reduce.  Every context on one GPU
 * shares that GPU's scratch, which keeps the last call's contents: calls that overlap in
 * time on one GPU (other threads, other streams) race and must be serialised by the
 * caller.  Synchronises the context's stream. */
int lbm_reduce_noalloc(lbm_ctx* c, int32_t inst, const double* mask, lbm_diag* out);

/* Serialises the complete state: a versioned header, both lattices' distributions, the
 * per-node state that carries phi u of the previous step (FP64: phi u; F32 / F16: the
 * published phi_w, u_w and, F16, p_w) with the pressure of the edge rows of open sides, and
 * the step count.  With buf == NULL only *bytes is set to the size needed.  Synchronises. */
int lbm_get_state(lbm_ctx* c, void* buf, size_t* bytes);

/* Restores a state written by lbm_get_state of a context with the same storage format,
 * phase-field lattice, instance grid sizes, densities rho_l and rho_g, and FP16 storage
 * scales; any other state is refused with LBM_ERR_PARAM and the context left as it was.
 * The other parameters (viscosities, sigma, W, M, body force, boundaries) may differ: a
 * restart may change them.  Synchronises. */
int lbm_set_state(lbm_ctx* c, const void* buf, size_t bytes);

/* Number of steps taken; the kernel (LBM_KERNEL_FUSED / SPLIT), tile rows, population
 * stores (LBM_STORES_CACHED / STREAMING), launch grid (LBM_GRID_TILES / PERSISTENT), tile
 * order (LBM_STRIP_ROWS, 8 or 16), narrow tiles (LBM_NARROW_ON / OFF) and dealing of the
 * tiles to the XCDs (LBM_DEAL_BANDS, or the chunk in tiles) the context runs with.  A chunk
 * at least as long as an XCD's band is reported as LBM_DEAL_BANDS, which it then is.  Any
 * pointer may be NULL; LBM_ERR_PARAM if c is NULL. */
int lbm_info(const lbm_ctx* c, int64_t* step, int32_t* kernel, int32_t* tile_rows,
             int32_t* stores, int32_t* grid, int32_t* strip, int32_t* narrow_tiles,
             int32_t* deal);

/* Build provenance: the sha256 (64 hex digits) of the source files the library was built
 * from, fixed at compile time; the Python binding compares it with the sources beside the
 * library and refuses a stale build.  Static string, never NULL; needs no device. */
const char* lbm_build_id(void);

/* Message of the last error of c, or of the calling thread if c is NULL. */
const char* lbm_last_error(const lbm_ctx* c);

/* Frees every device and host resource of c; NULL is ignored. */
void lbm_destroy(lbm_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
