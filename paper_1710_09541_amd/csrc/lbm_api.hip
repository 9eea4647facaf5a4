// Host runtime and C-ABI of liblbm_hip (see include/lbm.h): parameter validation, derived
// constants, SoA buffer layout, tile work-lists, HIP-graph replay of step pairs, the
// autotuner, moments, reductions and state save/restore.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_device.h"

using namespace lbm;

// sha256 of the sources the library was built from (set by the build script)
#ifndef LBM_SOURCE_SHA256
#define LBM_SOURCE_SHA256 "unknown"
#endif

namespace {

thread_local std::string g_thread_err;

constexpr uint64_t STATE_MAGIC = 0x4c424d5046534154ull;  // "LBMPFSAT"
constexpr int STATE_VERSION = 7;
// steps per captured graph, shortest first: each graph launch costs a few microseconds
// between the last kernel of one graph and the first of the next, which long graphs spread
// over more steps (measured: 64 steps per graph 0.6 % faster than 16 at 1024^2 FP32 and 4 %
// on a 64^2 grid; 256 no faster than 64)
constexpr int NGRAPH = 3;
// tile orders: whole rows (0), or vertical strips of 8 or 16 tiles (512 or 1024 nodes), rows
// inside a strip.  Strips keep the halo rows a tile re-reads within the last few dozen tiles,
// so they are still in the die's L2 when the working set is far larger than the caches
// (measured at 4096^2: +10 % FP32, +5 % FP16, +4 % FP64); whole rows win where it fits.
constexpr int NSTRIP = 3;
constexpr int STRIP_TILES[NSTRIP] = {0, 8, 16};
constexpr int GRAPH_STEPS[NGRAPH] = {2, 16, 64};
constexpr int PLANE_PAD = 192;  // elements added to each plane: breaks power-of-two plane strides
// tiles per chunk when the tiles are dealt to the XCDs in chunks: the longest accepted, and
// the one the autotuner times against one band per XCD (measured on a batch of 256 ragged
// instances, FP32: chunks of 4, 8, 16 and 64 tiles +8.5, +9.6, +10.2 and +7.6 % over bands;
// on single grids of 1024^2 and 4096^2 bands win by 4 to 12 %)
constexpr int MAX_CHUNK = 4096;
constexpr int AUTO_CHUNK = 16;

// Device scratch of lbm_reduce_noalloc, for callers that cannot allocate: the five FP64
// moment planes of one instance of at most NOALLOC_MAX_NODES nodes, then the reduction's
// per-block partials and its result.  Every GPU the library runs on holds one copy, from the
// library's load until the process ends; all contexts on that GPU share it.  Host code uses
// the address hipGetSymbolAddress returned for the device (noalloc_scratch_of), never the
// array's name, which on the host is only a stand-in.
constexpr int64_t NOALLOC_MAX_NODES = 1 << 20;
constexpr int64_t NOALLOC_PARTIALS = (int64_t)REDUCE_MAX_BLOCKS * REDUCE_SLOTS;
constexpr int64_t NOALLOC_DOUBLES = 5 * NOALLOC_MAX_NODES + NOALLOC_PARTIALS + 16;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

struct Instance {
    lbm_params p;
    InstDev d;
    int64_t n_nodes;
    int tile_begin_k1, tile_count_k1;  // this instance's tiles in the 4-row list
};

struct TileList {
    int rows = 0;
    int count = 0;
    TileDesc* dev = nullptr;
};

struct StateHeader {
    uint64_t magic;
    int32_t version, storage, n_inst, streamed;
    int64_t step;
    int32_t cur, reserved;
    uint64_t bytes_dist, bytes_q, bytes_mp;
    uint64_t total;
    uint64_t layout;   // fingerprint of how the bytes are laid out (state_layout)
};

}  // namespace

struct lbm_ctx {
    std::vector<Instance> inst;
    lbm_options opt;
    int storage = STORE_F32;
    size_t esize = 4;          // bytes per stored distribution value
    size_t qsize = 4;          // bytes per split-kernel phi value (compute type)
    int64_t dist_elems = 0;    // elements of one distribution set (all instances, 9 populations)
    int64_t q_elems = 0;       // FP64 phi u: a double2 per node and instance
    int64_t phi_elems = 0;     // split-kernel phi: 1 plane per instance
    int64_t mp_elems = 0;      // per-node state, in floats: 16-bit format, a float4 per node;
                               // FP32, a float3 per node and two rows of floats per instance;
                               // FP64, two rows of doubles per instance
    void* f[2] = {nullptr, nullptr};
    void* g[2] = {nullptr, nullptr};
    void* q = nullptr;
    void* q_tune = nullptr;
    void* phiplane = nullptr;
    void* rplane[2] = {nullptr, nullptr};  // that state, written with buffer i
    InstDev* d_insts = nullptr;
    // by tile height (4, 8, 16 rows), tile order and whether the last columns of an instance
    // whose width is not a multiple of 64 take narrower tiles
    TileList lists[3][NSTRIP][2];
    int strip = 0;             // tile order in use (index into STRIP_TILES)
    int narrow = 0;            // 1: narrow tiles at the right end of ragged instances
    int chunk = 0;             // tiles per chunk dealt to an XCD in turn; 0: one band per XCD
    double* mom = nullptr;     // 5 * max nodes, moments scratch
    double* partials = nullptr;
    double* red_out = nullptr;
    double* h_red = nullptr;   // pinned
    int64_t max_nodes = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    // captured step sequences starting from buffer 0 / 1: graph[g][from] holds
    // GRAPH_STEPS[g] consecutive steps (an even number, so the buffer parity returns)
    hipGraphExec_t graph[NGRAPH][2] = {};
    int cur = 0;               // buffer holding the current state
    bool streamed = true;      // the current state is still the initial, streamed one
    int64_t step = 0;
    int kernel = LBM_KERNEL_FUSED;
    int tile_rows = 8;
    int qf = 9;                // velocities of the phase-field lattice
    bool nt_store = false;     // non-temporal population stores
    bool persistent = false;   // persistent grid of resident blocks
    int num_cu = 0;            // compute units of the device
    int device = 0;            // the device current at lbm_init
    double* noalloc = nullptr; // that device's scratch of lbm_reduce_noalloc
    int persist_override = 0;  // LBM_PERSIST_BLOCKS: blocks per XCD of a persistent grid
    // resident blocks per CU, by tile rows and store policy (-1: not asked yet)
    mutable int per_cu[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};
    std::string err;
};

namespace {

int fail(lbm_ctx* c, int code, const std::string& msg) {
    g_thread_err = msg;
    if (c) c->err = msg;
    return code;
}

int hip_fail(lbm_ctx* c, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, LBM_ERR_DEVICE, m);
}

#define HIPCHK(c, call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(c, e_, #call); \
    } while (0)

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// copies and fills that accept empty buffers (a format does not allocate the other
// format's state planes)
hipError_t copy_n(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
    return bytes ? hipMemcpy(dst, src, bytes, kind) : hipSuccess;
}
hipError_t copy_n_async(void* dst, const void* src, size_t bytes, hipStream_t st) {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) : hipSuccess;
}
hipError_t zero_n_async(void* dst, size_t bytes, hipStream_t st) {
    return bytes ? hipMemsetAsync(dst, 0, bytes, st) : hipSuccess;
}

int list_index(int rows) { return rows == 4 ? 0 : (rows == 8 ? 1 : (rows == 16 ? 2 : -1)); }

std::string check_params(const lbm_params& p, int k) {
    char b[256];
    auto bad = [&](const char* what) {
        snprintf(b, sizeof b, "instance %d: %s", k, what);
        return std::string(b);
    };
    if (p.nx < 3 || p.ny < 3) return bad("nx and ny must be >= 3");
    if (p.bc_ylo < 0 || p.bc_ylo > 2 || p.bc_yhi < 0 || p.bc_yhi > 2)
        return bad("unknown boundary type");
    if ((p.bc_ylo == LBM_BC_PERIODIC) != (p.bc_yhi == LBM_BC_PERIODIC))
        return bad("periodic must be set on both y sides or on neither");
    if (p.visc_law < 0 || p.visc_law > 2) return bad("unknown viscosity law");
    if (p.grad_scheme < 0 || p.grad_scheme > 1) return bad("unknown gradient scheme");
    if (p.f_lattice != 0 && p.f_lattice != LBM_LATTICE_D2Q9 && p.f_lattice != LBM_LATTICE_D2Q5)
        return bad("unknown phase-field lattice (use 9 or 5)");
    if (!(p.rho_l > 0) || !(p.rho_g > 0)) return bad("densities must be > 0");
    if (!(p.nu_l > 0) || !(p.nu_g > 0)) return bad("viscosities must be > 0");
    if (!(p.W > 0)) return bad("W must be > 0");
    if (!(p.M > 0)) return bad("M must be > 0");
    if (!(p.sigma >= 0)) return bad("sigma must be >= 0");
    if (!isfinite(p.Gx) || !isfinite(p.Gy)) return bad("non-finite body force");
    const int64_t pitch = round_up(p.nx, TILE_X);
    if (9 * ((int64_t)p.ny * pitch + PLANE_PAD) >= (int64_t)1 << 31)
        return bad("grid too large for one instance");
    return std::string();
}

int pick_exponent(int given, double bound, int storage) {
    if (storage != STORE_F16) return 0;   // only the 16-bit format is scaled
    if (given != LBM_EXP_AUTO) return given;
    // keep 32x head-room below the largest half (65504)
    int e = (int)floor(log2(65504.0 / (32.0 * bound)));
    return std::max(-8, std::min(24, e));
}

void fill_inst(Instance& I, int storage, const double* phi0, const double* ux0, const double* uy0) {
    const lbm_params& p = I.p;
    InstDev& d = I.d;
    memset(&d, 0, sizeof d);
    d.nx = p.nx;
    d.ny = p.ny;
    d.pitch = (int)round_up(p.nx, TILE_X);
    d.bc_lo = p.bc_ylo;
    d.bc_hi = p.bc_yhi;
    d.visc_law = p.visc_law;
    d.grad_scheme = p.grad_scheme;
    d.plane = (int64_t)p.ny * d.pitch + PLANE_PAD;
    d.rho_l = p.rho_l;
    d.rho_g = p.rho_g;
    d.drho = p.rho_l - p.rho_g;
    d.nu_l = p.nu_l;
    d.nu_g = p.nu_g;
    d.inv_nu_l = 1.0 / p.nu_l;
    d.inv_nu_g = 1.0 / p.nu_g;
    d.mu_l = p.rho_l * p.nu_l;
    d.mu_g = p.rho_g * p.nu_g;
    d.kappa = 1.5 * p.sigma * p.W;      // Eq. 7
    d.beta = 12.0 * p.sigma / p.W;
    d.W = p.W;
    d.inv_w = 1.0 / p.W;
    const double tau_f = p.M * 3.0 + 0.5;  // Eq. 14
    d.tau_f = tau_f;
    d.inv_tau_f = 1.0 / tau_f;
    d.cf = 1.0 - 1.0 / (2.0 * tau_f);
    d.Gx = p.Gx;
    d.Gy = p.Gy;
    // bound of the initial g (equilibria at p = 0), floor for fluids at rest
    double gb = 1e-3 * std::max(p.rho_l, p.rho_g);
    const int64_t n = (int64_t)p.nx * p.ny;
    for (int64_t k = 0; k < n; ++k) {
        const double rho = phi0[k] * d.drho + p.rho_g;
        const double u = fabs(ux0[k]) + fabs(uy0[k]);
        gb = std::max(gb, rho * (3.0 * u + 4.5 * u * u) * (4.0 / 9.0));
    }
    // stored f are rest deviations, of the size of w_i phi 3 c_i.u: 0.15 covers |u| < 0.3
    const int ef = pick_exponent(p.exp_f, 0.15, storage);
    const int eg = pick_exponent(p.exp_g, gb, storage);
    d.scale_f = ldexp(1.0, ef);
    d.inv_scale_f = ldexp(1.0, -ef);
    d.scale_g = ldexp(1.0, eg);
    d.inv_scale_g = ldexp(1.0, -eg);
    I.p.exp_f = ef;
    I.p.exp_g = eg;
    I.n_nodes = n;
    // FP32 copies of the constants (lbm_device.h): the same roundings the kernels would make
    d.f_beta4 = (float)(4.0 * d.beta);
    d.f_kappa = (float)d.kappa;
    d.f_inv_w = (float)d.inv_w;
    d.f_dnu = (float)(d.nu_l - d.nu_g);
    d.f_nu_g = (float)d.nu_g;
    d.f_dinv_nu = (float)(d.inv_nu_l - d.inv_nu_g);
    d.f_inv_nu_g = (float)d.inv_nu_g;
    d.f_mu_l = (float)d.mu_l;
    d.f_mu_g = (float)d.mu_g;
    d.f_Gx = (float)d.Gx;
    d.f_Gy = (float)d.Gy;
    d.f_inv_tau_f = (float)d.inv_tau_f;
    d.f_cf = (float)d.cf;
    d.f_drho = (float)d.drho;
    d.f_rho_g = (float)d.rho_g;
    d.f_scale_f = (float)d.scale_f;
    d.f_inv_scale_f = (float)d.inv_scale_f;
    d.f_scale_g = (float)d.scale_g;
    d.f_inv_scale_g = (float)d.inv_scale_g;
}

// Narrow tiles for the last r = nx mod 64 columns of an instance (narrow = true): 16 wide
// for r <= 16, 32 wide for r <= 32, 32 + 16 wide for r <= 48; a 64-wide column otherwise.
// A narrow tile keeps the block's 256 threads busy with 2 or 4 rows per wavefront where a
// 64-wide one would leave 64 - r lanes of every row without a node.  Every column of tiles
// is appended to cols as (x0, width class).
void narrow_columns(int nx, bool narrow, std::vector<std::pair<int, int>>& cols) {
    const int full = nx / TILE_X * TILE_X, r = nx - full;
    for (int x0 = 0; x0 < full; x0 += TILE_X) cols.push_back({x0, 0});
    if (r == 0) return;
    if (!narrow || r > 48) {
        cols.push_back({full, 0});
    } else if (r <= 16) {
        cols.push_back({full, 2});
    } else {
        cols.push_back({full, 1});
        if (r > 32) cols.push_back({full + 32, 2});
    }
}

// the tiles of every instance in turn; within an instance, row after row (strip_tiles = 0)
// or strip after strip of strip_tiles tiles, row after row inside each strip.  A tile of
// width class w is rows << w rows tall; it is listed in the row of tiles where it starts.
std::vector<TileDesc> build_tiles(const std::vector<Instance>& v, int rows, int strip_tiles,
                                  bool narrow) {
    std::vector<TileDesc> t;
    for (size_t k = 0; k < v.size(); ++k) {
        const int nx = v[k].p.nx;
        std::vector<std::pair<int, int>> cols;
        narrow_columns(nx, narrow, cols);
        const int sw = (strip_tiles > 0 && strip_tiles * TILE_X < nx) ? strip_tiles * TILE_X : nx;
        for (int xs = 0; xs < nx; xs += sw)
            for (int y0 = 0; y0 < v[k].p.ny; y0 += rows)
                for (const auto& col : cols)
                    if (col.first >= xs && col.first < std::min(nx, xs + sw) &&
                        y0 % (rows << col.second) == 0)
                        t.push_back({(int32_t)k, col.first, y0, col.second});
    }
    return t;
}

// whether narrow tiles give another tiling than 64-wide ones for some instance
bool narrow_differs(const lbm_ctx* c) {
    for (const Instance& I : c->inst) {
        const int r = I.p.nx % TILE_X;
        if (r > 0 && r <= 48) return true;
    }
    return false;
}

// whether strips of strip_tiles tiles give another order than whole rows for some instance
bool strip_differs(const lbm_ctx* c, int strip_tiles) {
    for (const Instance& I : c->inst)
        if (strip_tiles > 0 && strip_tiles * TILE_X < I.p.nx) return true;
    return false;
}

// FNV-1a over what fixes the meaning of a state's bytes beyond their count: every
// instance's grid size, FP16 storage scales and the two densities (the reduced formats store
// deviations from equilibria whose g part holds rho(phi)), and the phase-field lattice.
// Two contexts whose instances differ only in their transposes have equal byte counts,
// for instance.
uint64_t state_layout(const lbm_ctx* c) {
    uint64_t h = 0xcbf29ce484222325ull;
    const auto mix = [&h](const void* p, size_t n) {
        for (size_t i = 0; i < n; ++i) {
            h ^= ((const unsigned char*)p)[i];
            h *= 0x100000001b3ull;
        }
    };
    mix(&c->qf, sizeof c->qf);
    for (const Instance& I : c->inst) {
        mix(&I.d.nx, sizeof I.d.nx);
        mix(&I.d.ny, sizeof I.d.ny);
        mix(&I.d.scale_f, sizeof I.d.scale_f);
        mix(&I.d.scale_g, sizeof I.d.scale_g);
        mix(&I.d.rho_l, sizeof I.d.rho_l);
        mix(&I.d.rho_g, sizeof I.d.rho_g);
    }
    return h;
}

void free_all(lbm_ctx* c) {
    for (int i = 0; i < 2; ++i) {
        for (int g = 0; g < NGRAPH; ++g) {
            if (c->graph[g][i]) (void)hipGraphExecDestroy(c->graph[g][i]);
            c->graph[g][i] = nullptr;
        }
        if (c->f[i]) (void)hipFree(c->f[i]);
        if (c->g[i]) (void)hipFree(c->g[i]);
        c->f[i] = c->g[i] = nullptr;
    }
    void* ptrs[] = {c->q,       c->q_tune,    c->phiplane, c->rplane[0], c->rplane[1],
                    c->d_insts, c->mom,       c->partials, c->red_out};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& by_rows : c->lists)
        for (auto& by_order : by_rows)
            for (auto& l : by_order)
                if (l.dev) (void)hipFree(l.dev);
    if (c->h_red) (void)hipHostFree(c->h_red);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

// blocks per XCD of a persistent grid: as many as stay resident on the whole GPU (0 if
// the runtime cannot say, and then no persistent grid is used), or the number the
// environment variable LBM_PERSIST_BLOCKS gives
int persist_blocks(const lbm_ctx* c, int rows, bool nt) {
    if (c->persist_override > 0) return c->persist_override;
    const int li = list_index(rows);
    if (li < 0) return 0;
    int& cached = c->per_cu[li][nt ? 1 : 0];
    if (cached < 0) cached = step_blocks_per_cu(c->storage, c->qf, rows, nt);
    const int per_cu = cached;
    if (per_cu <= 0 || c->num_cu <= 0) return 0;
    return std::max(1, per_cu * c->num_cu / NXCD);
}

// whether steps run on a persistent grid: the fused kernel with fewer resident blocks than
// tiles (otherwise every block has one tile anyway)
bool runs_persistent(const lbm_ctx* c) {
    if (!c->persistent || c->kernel != LBM_KERNEL_FUSED) return false;
    const int pb = persist_blocks(c, c->tile_rows, c->nt_store);
    const int per = (c->lists[list_index(c->tile_rows)][c->strip][c->narrow].count + NXCD - 1) /
                    NXCD;
    return pb > 0 && pb < per;
}

StepArgs step_args(lbm_ctx* c, int src, bool pull, int rows, bool split, void* q, int strip,
                   int narrow) {
    StepArgs a;
    const TileList& L = c->lists[list_index(rows)][strip][narrow];
    a.insts = c->d_insts;
    a.tiles = L.dev;
    a.ntiles = L.count;
    a.tile_rows = rows;
    a.qf = c->qf;
    a.nt_store = false;
    a.persist = 0;
    a.chunk = 0;
    a.pull = pull;
    a.split = split;
    a.fsrc = c->f[src];
    a.gsrc = c->g[src];
    a.fdst = c->f[1 - src];
    a.gdst = c->g[1 - src];
    a.q = q;
    a.phiplane = c->phiplane;
    a.rsrc = c->rplane[src];
    a.rdst = c->rplane[1 - src];
    a.stream = c->stream;
    return a;
}

int launch_one(lbm_ctx* c, hipStream_t st) {
    StepArgs a;
    if (c->streamed)
        a = step_args(c, c->cur, false, 4, false, c->q, c->strip, c->narrow);
    else
    {
        a = step_args(c, c->cur, true, c->tile_rows, c->kernel == LBM_KERNEL_SPLIT, c->q,
                      c->strip, c->narrow);
        a.nt_store = c->nt_store;
        a.persist = runs_persistent(c) ? persist_blocks(c, c->tile_rows, c->nt_store) : 0;
        a.chunk = c->chunk;
    }
    a.stream = st;
    hipError_t e = launch_step(c->storage, a);
    if (e != hipSuccess) return hip_fail(c, e, "step launch");
    c->cur = 1 - c->cur;
    c->streamed = false;
    return LBM_OK;
}

void drop_graphs(lbm_ctx* c) {
    for (int g = 0; g < NGRAPH; ++g)
        for (int i = 0; i < 2; ++i) {
            if (c->graph[g][i]) (void)hipGraphExecDestroy(c->graph[g][i]);
            c->graph[g][i] = nullptr;
        }
}

// captures GRAPH_STEPS[g] consecutive steps starting from buffer `from`
int capture_steps(lbm_ctx* c, int g, int from) {
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const int save_cur = c->cur;
    const bool save_streamed = c->streamed;
    c->cur = from;
    c->streamed = false;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = LBM_OK;
    for (int k = 0; k < GRAPH_STEPS[g] && rc == LBM_OK; ++k) rc = launch_one(c, c->cap_stream);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &gr);
    c->cur = save_cur;
    c->streamed = save_streamed;
    if (rc != LBM_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&c->graph[g][from], gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
    return LBM_OK;
}

int moments_to(lbm_ctx* c, int inst, double* out) {
    const Instance& I = c->inst[inst];
    // whole-row order: an instance's tiles are one contiguous run of the 4-row list
    StepArgs a = step_args(c, c->cur, !c->streamed, 4, false, c->q, 0, 0);
    a.tiles = c->lists[0][0][0].dev + I.tile_begin_k1;
    a.ntiles = I.tile_count_k1;
    hipError_t e = launch_moments(c->storage, a, out);
    if (e != hipSuccess) return hip_fail(c, e, "moments launch");
    return LBM_OK;
}

int reduce_inst(lbm_ctx* c, int inst, const double* mask, double* res /*12*/) {
    int rc = moments_to(c, inst, c->mom);
    if (rc) return rc;
    const Instance& I = c->inst[inst];
    double m[5] = {0, 0, 0, 0, -1};
    if (mask) memcpy(m, mask, sizeof m);
    hipError_t e = launch_reduce(c->mom, I.p.nx, I.p.ny, I.p.bc_ylo == LBM_BC_PERIODIC, m,
                                 c->partials, c->red_out, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reduce launch");
    HIPCHK(c, hipMemcpyAsync(c->h_red, c->red_out, 12 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    memcpy(res, c->h_red, 12 * sizeof(double));
    return LBM_OK;
}

// The device address of `scratch` on device dev (current), taken once per device with
// hipGetSymbolAddress; nullptr (and the message in c) on failure.
double* noalloc_scratch_of(lbm_ctx* c, int dev) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        fail(c, LBM_ERR_DEVICE, "device index beyond the no-allocation scratch table");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            hip_fail(c, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
            return nullptr;
        }
        g_noalloc_ptr[dev] = (double*)ptr;
    }
    return g_noalloc_ptr[dev];
}

int check_finite(lbm_ctx* c) {
    for (size_t k = 0; k < c->inst.size(); ++k) {
        double r[12];
        int rc = reduce_inst(c, (int)k, nullptr, r);
        if (rc) return rc;
        if (r[11] > 0) {
            char b[160];
            snprintf(b, sizeof b, "instance %zu: %.0f nodes with non-finite values at step %lld", k,
                     r[11], (long long)c->step);
            return fail(c, LBM_ERR_NONFINITE, b);
        }
    }
    return LBM_OK;
}

// ------------------------------------------------------------------ autotuner cache
// If the environment variable LBM_AUTOTUNE_CACHE names a file, tuned choices are kept there,
// one text line per configuration:
//   lbm-tune-v5 <key> <kernel> <tile_rows> <streaming stores 0/1> <persistent grid 0/1>
//               <tile order 0/1/2: whole rows, strips of 8, strips of 16 tiles>
//               <narrow tiles at the right end of ragged instances 0/1>
//               <tiles per chunk dealt to the XCDs, 0: one band per XCD>
// The key covers everything the timing depends on: the GPU architecture, storage, phase-
// field lattice, the requested kernel / tile rows / store policy / grid / order, the number of
// instances and every instance's grid size.  A missing, unreadable or malformed file only means the
// tuner runs; a write failure is ignored.
std::string tune_key(const lbm_ctx* c) {
    std::ostringstream k;
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == ' ') ch = '_';
    k << arch << ":s" << c->storage << ":q" << c->qf << ":k" << c->opt.kernel << ":r"
      << c->opt.tile_rows << ":w" << c->opt.stores << ":g" << c->opt.grid << ":o" << c->opt.strip
      << ":t" << c->opt.narrow_tiles << ":d" << c->opt.deal << ":n" << c->inst.size();
    for (const Instance& I : c->inst) k << ":" << I.p.nx << "x" << I.p.ny;
    return k.str();
}

bool tune_cache_lookup(lbm_ctx* c, const std::string& key) {
    const char* path = getenv("LBM_AUTOTUNE_CACHE");
    if (!path || !*path) return false;
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string tag, k;
        int kernel = 0, rows = 0, nt = 0, pg = 0, si = 0, nw = 0, ch = 0;
        if (!(ls >> tag >> k >> kernel >> rows >> nt >> pg >> si >> nw >> ch) ||
            tag != "lbm-tune-v5" || k != key)
            continue;
        if ((kernel != LBM_KERNEL_FUSED && kernel != LBM_KERNEL_SPLIT) || list_index(rows) < 0 ||
            (nt != 0 && nt != 1) || (pg != 0 && pg != 1) || si < 0 || si >= NSTRIP ||
            (nw != 0 && nw != 1) || ch < 0 || ch > MAX_CHUNK)
            continue;
        c->strip = si;
        c->narrow = nw;
        c->chunk = ch;
        c->kernel = kernel;   // the last valid line for the key wins
        c->tile_rows = rows;
        c->nt_store = nt == 1;
        c->persistent = pg == 1;
        found = true;
    }
    return found;
}

void tune_cache_store(const lbm_ctx* c, const std::string& key) {
    const char* path = getenv("LBM_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream out(path, std::ios::app);
    if (out) out << "lbm-tune-v5 " << key << " " << c->kernel << " " << c->tile_rows << " "
                 << (c->nt_store ? 1 : 0) << " " << (c->persistent ? 1 : 0) << " " << c->strip
                 << " " << c->narrow << " " << c->chunk << "\n";
}

// ------------------------------------------------------------------ autotuner
// Times each candidate (kernel, tile rows) on the context's own data, launched the way the
// time loop launches them: alternating between two buffers, here the spare buffer and a
// temporary copy of the current state, with a scratch copy of phi u, so the state itself
// is left untouched.  (The alternation matters: the buffer a step reads was written by the
// step before, partly still in the last-level cache.)  If the temporary cannot be
// allocated, the launches repeat from the current buffer into the spare one.  The fastest
// median of interleaved rounds wins, by a margin of 1 % over the candidates listed before
// it: smaller tiles first, and the store policy expected to win first (streaming stores when
// a step's working set exceeds the 256 MB last-level cache of MI355X, cached ones below).
int autotune(lbm_ctx* c) {
    struct Cand {
        int kernel, rows;
        bool nt, persistent;
        int strip, narrow, chunk;
    };
    std::vector<Cand> cands;
    const bool want_fused = c->opt.kernel != LBM_KERNEL_SPLIT;
    const bool want_split = c->opt.kernel != LBM_KERNEL_FUSED;
    const bool want_cached = c->opt.stores != LBM_STORES_STREAMING;
    const bool want_nt = c->opt.stores != LBM_STORES_CACHED;
    // the persistent grid only when asked for: it measured 3-14 % slower than one block per
    // tile on every workload and format, so timing it at every init is not worth its cost
    const bool want_tiles = c->opt.grid != LBM_GRID_PERSISTENT;
    const bool want_persistent = c->opt.grid == LBM_GRID_PERSISTENT;
    // bytes one step reads and writes: both buffers of both lattices and the per-node state
    const double step_bytes = 4.0 * (double)c->dist_elems * c->esize +
                              (double)c->q_elems * sizeof(double) * 2.0 +
                              (double)c->mp_elems * sizeof(float) * 2.0;
    const bool streaming_first = step_bytes > 256.0 * 1024.0 * 1024.0;
    // tile orders: the requested one, or whole rows first and then the strip widths that
    // change the order of some instance
    std::vector<int> strips;
    if (c->opt.strip != LBM_STRIP_AUTO) {
        strips.push_back(c->strip);
    } else {
        strips.push_back(0);
        for (int si = 1; si < NSTRIP; ++si)
            if (strip_differs(c, STRIP_TILES[si])) strips.push_back(si);
    }
    // narrow tiles at the right end of ragged instances: the requested choice, or both
    // (narrow first: fewer idle lanes) where they change the tiling
    std::vector<int> narrows;
    if (c->opt.narrow_tiles != LBM_NARROW_AUTO)
        narrows.push_back(c->narrow);
    else if (narrow_differs(c))
        narrows = {1, 0};
    else
        narrows.push_back(0);
    // dealing of the tiles to the XCDs: the requested one, or one band per XCD and then
    // chunks of AUTO_CHUNK tiles where a band is longer than that
    std::vector<int> chunks;
    if (c->opt.deal != LBM_DEAL_AUTO)
        chunks.push_back(c->chunk);
    else
        chunks = {0, AUTO_CHUNK};
    const int rows_opts[3] = {4, 8, 16};
    for (int r : rows_opts) {
        if (c->opt.tile_rows && c->opt.tile_rows != r) continue;
        if (c->storage == STORE_F64 && r == 16) continue;  // 16 rows of doubles spill
        for (int k = 0; k < 2; ++k) {
            const int nt = streaming_first ? 1 - k : k;
            if ((nt && !want_nt) || (!nt && !want_cached)) continue;
            for (int pg = 0; pg < 2; ++pg) {
                if ((pg && !want_persistent) || (!pg && !want_tiles)) continue;
                for (int si : strips)
                    for (int nw : narrows)
                        for (int ch : chunks) {
                            // a persistent grid runs one band per XCD; a chunk at least as
                            // long as the band is the band
                            const int per =
                                (c->lists[list_index(r)][si][nw].count + NXCD - 1) / NXCD;
                            if (ch != chunks[0] && (pg || ch >= per)) continue;
                            if (want_fused)
                                cands.push_back({LBM_KERNEL_FUSED, r, nt == 1, pg == 1, si, nw,
                                                 pg ? 0 : ch});
                            // the split kernel runs one block per tile
                            if (want_split && !pg)
                                cands.push_back({LBM_KERNEL_SPLIT, r, nt == 1, false, si, nw, ch});
                        }
            }
        }
    }
    if (cands.size() == 1) {
        c->kernel = cands[0].kernel;
        c->tile_rows = cands[0].rows;
        c->nt_store = cands[0].nt;
        c->persistent = cands[0].persistent;
        c->strip = cands[0].strip;
        c->narrow = cands[0].narrow;
        c->chunk = cands[0].chunk;
        return LBM_OK;
    }
    HIPCHK(c, copy_n_async(c->q_tune, c->q, c->q_elems * sizeof(double), c->stream));
    // temporary copy of the current buffers
    void *tf = nullptr, *tg = nullptr, *tr = nullptr;
    const size_t dbytes = (size_t)c->dist_elems * c->esize;
    const size_t rbytes = (size_t)c->mp_elems * sizeof(float);
    bool alt = hipMalloc(&tf, dbytes) == hipSuccess && hipMalloc(&tg, dbytes) == hipSuccess &&
               (rbytes == 0 || hipMalloc(&tr, rbytes) == hipSuccess);
    (void)hipGetLastError();
    auto free_temps = [&]() {
        if (tf) (void)hipFree(tf);
        if (tg) (void)hipFree(tg);
        if (tr) (void)hipFree(tr);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    {
        hipError_t e = hipSuccess;
        if (alt) {
            e = hipMemcpyAsync(tf, c->f[c->cur], dbytes, hipMemcpyDeviceToDevice, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(tg, c->g[c->cur], dbytes, hipMemcpyDeviceToDevice, c->stream);
            if (e == hipSuccess) e = copy_n_async(tr, c->rplane[c->cur], rbytes, c->stream);
        }
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            free_temps();
            return hip_fail(c, e, "autotune set-up");
        }
    }
    int64_t nodes = 0;
    for (auto& I : c->inst) nodes += I.n_nodes;
    // an even number of launches: whole temporary -> spare -> temporary pairs
    const int reps = 2 * std::max(2, (int)std::min<int64_t>(25, 100000000 / std::max<int64_t>(nodes, 1)));
    // Every candidate runs once untimed (clocks and caches reach their running state), then
    // NREP timed rounds visit the candidates in turn, so a slow drift of the clocks does not
    // favour the candidates timed first; the median of each candidate's rounds decides.
    constexpr int NREP = 5;
    const int nc = (int)cands.size();
    std::vector<float> t((size_t)nc * NREP, 0.0f);
    int rc = LBM_OK;
    auto args_of = [&](const Cand& cd, StepArgs& a, StepArgs& b) {
        a = step_args(c, c->cur, true, cd.rows, cd.kernel == LBM_KERNEL_SPLIT, c->q_tune,
                      cd.strip, cd.narrow);
        a.nt_store = cd.nt;
        a.persist = cd.persistent ? persist_blocks(c, cd.rows, cd.nt) : 0;
        a.chunk = cd.chunk;
        b = a;
        if (alt) {
            // temporary -> spare, then spare -> temporary
            a.fsrc = tf;
            a.gsrc = tg;
            a.rsrc = tr;
            b.fsrc = a.fdst;
            b.gsrc = a.gdst;
            b.rsrc = a.rdst;
            b.fdst = tf;
            b.gdst = tg;
            b.rdst = tr;
        }
    };
    for (int round = -1; round < NREP && rc == LBM_OK; ++round) {
        for (int ci = 0; ci < nc && rc == LBM_OK; ++ci) {
            StepArgs a, b;
            args_of(cands[ci], a, b);
            hipError_t e = hipEventRecord(e0, c->stream);
            if (e != hipSuccess) {
                rc = hip_fail(c, e, "autotune event");
                break;
            }
            for (int k = 0; k < reps; ++k) {
                e = launch_step(c->storage, (k & 1) ? b : a);
                if (e != hipSuccess) {
                    rc = hip_fail(c, e, "autotune launch");
                    break;
                }
            }
            if (rc != LBM_OK) break;
            e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            // a time that could not be read must not make its candidate look fastest
            if (e == hipSuccess && round >= 0)
                e = hipEventElapsedTime(&t[(size_t)ci * NREP + round], e0, e1);
            if (e != hipSuccess) {
                rc = hip_fail(c, e, "autotune timing");
                break;
            }
        }
    }
    if (rc == LBM_OK) {
        // candidates come smallest tile first, the expected store policy first; a later one
        // must win by more than 1 % (several times the spread of a candidate's timed rounds),
        // so noise does not flip the choice between near-equal configurations
        float best = 1e30f;
        for (int ci = 0; ci < nc; ++ci) {
            float* tc = t.data() + (size_t)ci * NREP;
            std::sort(tc, tc + NREP);
            if (tc[NREP / 2] < 0.99f * best) {
                best = tc[NREP / 2];
                c->kernel = cands[ci].kernel;
                c->tile_rows = cands[ci].rows;
                c->nt_store = cands[ci].nt;
                c->persistent = cands[ci].persistent;
                c->strip = cands[ci].strip;
                c->narrow = cands[ci].narrow;
                c->chunk = cands[ci].chunk;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    free_temps();
    return rc;
}

}  // namespace

// ====================================================================== C-ABI

extern "C" {

int lbm_init(const lbm_params* p, int32_t n_inst, const lbm_options* opt,
             const double* const* phi0, const double* const* ux0, const double* const* uy0,
             void* hip_stream, lbm_ctx** out) {
    if (!out) return fail(nullptr, LBM_ERR_PARAM, "out is NULL");
    *out = nullptr;
    if (!p || n_inst < 1) return fail(nullptr, LBM_ERR_PARAM, "need at least one instance");
    if (!phi0 || !ux0 || !uy0) return fail(nullptr, LBM_ERR_PARAM, "initial fields are NULL");
    lbm_options o;
    memset(&o, 0, sizeof o);
    o.storage = LBM_STORE_F32;
    o.kernel = LBM_KERNEL_AUTO;
    o.use_graph = 1;
    if (opt) o = *opt;
    if (o.storage < 0 || o.storage > 2) return fail(nullptr, LBM_ERR_PARAM, "unknown storage");
    if (o.kernel < 0 || o.kernel > 2) return fail(nullptr, LBM_ERR_PARAM, "unknown kernel");
    if (o.tile_rows != 0 && list_index(o.tile_rows) < 0)
        return fail(nullptr, LBM_ERR_PARAM, "tile_rows must be 0, 4, 8 or 16");
    if (o.check_every < 0) return fail(nullptr, LBM_ERR_PARAM, "check_every must be >= 0");
    if (o.stores < 0 || o.stores > 2) return fail(nullptr, LBM_ERR_PARAM, "unknown store policy");
    if (o.grid < 0 || o.grid > 2) return fail(nullptr, LBM_ERR_PARAM, "unknown launch grid");
    if (o.strip != LBM_STRIP_AUTO && o.strip != LBM_STRIP_ROWS && o.strip != 8 && o.strip != 16)
        return fail(nullptr, LBM_ERR_PARAM, "strip must be 0 (auto), -1 (whole rows), 8 or 16");
    if (o.narrow_tiles != LBM_NARROW_AUTO && o.narrow_tiles != LBM_NARROW_OFF &&
        o.narrow_tiles != LBM_NARROW_ON)
        return fail(nullptr, LBM_ERR_PARAM, "narrow_tiles must be 0 (auto), -1 (off) or 1 (on)");
    if (o.deal != LBM_DEAL_AUTO && o.deal != LBM_DEAL_BANDS && (o.deal < 1 || o.deal > MAX_CHUNK))
        return fail(nullptr, LBM_ERR_PARAM, "deal must be 0 (auto), -1 (bands) or 1 to 4096 tiles");
    const auto lattice_of = [](const lbm_params& q) {
        return q.f_lattice == 0 ? (int)LBM_LATTICE_D2Q9 : (int)q.f_lattice;
    };
    for (int k = 0; k < n_inst; ++k) {
        std::string m = check_params(p[k], k);
        if (!m.empty()) return fail(nullptr, LBM_ERR_PARAM, m);
        if (!phi0[k] || !ux0[k] || !uy0[k])
            return fail(nullptr, LBM_ERR_PARAM, "initial field of an instance is NULL");
        if (lattice_of(p[k]) != lattice_of(p[0]))
            return fail(nullptr, LBM_ERR_PARAM, "all instances must use the same phase-field lattice");
    }

    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_ERR_ALLOC, "host allocation failed");
    c->opt = o;
    c->storage = o.storage;
    c->esize = o.storage == STORE_F64 ? 8 : (o.storage == STORE_F32 ? 4 : 2);
    c->qsize = o.storage == STORE_F64 ? 8 : 4;
    c->qf = lattice_of(p[0]);
    c->inst.resize(n_inst);
    int64_t off_dist = 0, off_q = 0, off_phi = 0, off_mp = 0;
    for (int k = 0; k < n_inst; ++k) {
        Instance& I = c->inst[k];
        I.p = p[k];
        fill_inst(I, c->storage, phi0[k], ux0[k], uy0[k]);
        // the kernels address one instance's 9 planes through a buffer resource with a 32-bit
        // byte range
        if (9 * I.d.plane * (int64_t)c->esize >= ((int64_t)1 << 32)) {
            char b[160];
            snprintf(b, sizeof b, "instance %d: grid too large for one instance in this storage "
                     "format (9 planes must stay below 4 GiB)", k);
            const std::string m(b);
            delete c;
            return fail(nullptr, LBM_ERR_PARAM, m);
        }
        I.d.off_dist = off_dist;
        I.d.off_q = off_q;
        I.d.off_phi = off_phi;
        I.d.off_mp = off_mp;
        off_dist += round_up(9 * I.d.plane, 64);
        // phi u of the previous step: two double planes (FP64 format) or, in the reduced
        // formats, the per-node FP32 state that also carries it: (phi_w, p_w, ux_w, uy_w) in
        // the 16-bit format, (phi_w, ux_w, uy_w) and the pressure of the first and the last
        // row (open sides) in the FP32 format.  The FP64 format keeps the pressure of those
        // rows in that place: two rows of pitch doubles.  All double-buffered.
        if (c->storage == STORE_F64) {
            off_q += round_up(2 * I.d.plane, 64);
            off_mp += round_up(2 * 2 * (int64_t)I.d.pitch, 64);
        } else if (c->storage == STORE_F32) {
            off_mp += round_up(3 * I.d.plane + 2 * (int64_t)I.d.pitch, 64);
        } else {
            off_mp += round_up(4 * I.d.plane, 64);
        }
        off_phi += round_up(I.d.plane, 64);
        c->max_nodes = std::max(c->max_nodes, I.n_nodes);
    }
    c->dist_elems = off_dist;
    c->q_elems = off_q;
    c->phi_elems = off_phi;
    c->mp_elems = off_mp;

    auto bail = [&](int rc) {
        free_all(c);
        delete c;
        return rc;
    };
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) {
        fail(c, LBM_ERR_DEVICE, "no HIP device available");
        return bail(LBM_ERR_DEVICE);
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(hip_fail(c, e, "hipStreamCreate"));
        c->own_stream = true;
    }
    const size_t dist_bytes = c->dist_elems * c->esize;
    struct {
        void** ptr;
        size_t bytes;
    } allocs[] = {
        {&c->f[0], dist_bytes},
        {&c->f[1], dist_bytes},
        {&c->g[0], dist_bytes},
        {&c->g[1], dist_bytes},
        {&c->q, c->q_elems * sizeof(double)},
        {&c->q_tune, c->q_elems * sizeof(double)},
        {&c->phiplane, c->phi_elems * c->qsize},
        {&c->rplane[0], c->mp_elems * sizeof(float)},
        {&c->rplane[1], c->mp_elems * sizeof(float)},
        {(void**)&c->d_insts, n_inst * sizeof(InstDev)},
        {(void**)&c->mom, 5 * c->max_nodes * sizeof(double)},
        {(void**)&c->partials, REDUCE_MAX_BLOCKS * REDUCE_SLOTS * sizeof(double)},
        {(void**)&c->red_out, 16 * sizeof(double)},
    };
    for (auto& a : allocs) {
        *a.ptr = nullptr;
        if (a.bytes == 0) continue;   // a buffer this format does not use
        e = hipMalloc(a.ptr, a.bytes);
        if (e != hipSuccess) {
            fail(c, LBM_ERR_ALLOC, std::string("device allocation failed: ") + hipGetErrorString(e));
            return bail(LBM_ERR_ALLOC);
        }
    }
    e = hipHostMalloc((void**)&c->h_red, 16 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipHostMalloc"));
    // padding between and inside planes is never read, but keep it defined
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipMemsetAsync(c->f[i], 0, dist_bytes, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->g[i], 0, dist_bytes, c->stream);
    }
    if (e == hipSuccess) e = zero_n_async(c->phiplane, c->phi_elems * c->qsize, c->stream);
    if (e == hipSuccess) e = zero_n_async(c->q, c->q_elems * sizeof(double), c->stream);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        e = zero_n_async(c->rplane[i], c->mp_elems * sizeof(float), c->stream);
    if (e != hipSuccess) return bail(hip_fail(c, e, "clearing the state buffers"));

    std::vector<InstDev> hd(n_inst);
    for (int k = 0; k < n_inst; ++k) hd[k] = c->inst[k].d;
    e = hipMemcpyAsync(c->d_insts, hd.data(), n_inst * sizeof(InstDev), hipMemcpyHostToDevice,
                       c->stream);
    if (e != hipSuccess) return bail(hip_fail(c, e, "copy instances"));
    const int rows_of[3] = {4, 8, 16};
    for (int li = 0; li < 3; ++li)
    for (int si = 0; si < NSTRIP; ++si)
    for (int nw = 0; nw < 2; ++nw) {
        std::vector<TileDesc> t = build_tiles(c->inst, rows_of[li], STRIP_TILES[si], nw == 1);
        TileList& L = c->lists[li][si][nw];
        L.rows = rows_of[li];
        L.count = (int)t.size();
        e = hipMalloc((void**)&L.dev, t.size() * sizeof(TileDesc));
        if (e != hipSuccess) return bail(hip_fail(c, e, "tile list"));
        e = hipMemcpy(L.dev, t.data(), t.size() * sizeof(TileDesc), hipMemcpyHostToDevice);
        if (e != hipSuccess) return bail(hip_fail(c, e, "tile list copy"));
        if (li == 0 && si == 0 && nw == 0) {
            int pos = 0;
            for (int k = 0; k < n_inst; ++k) {
                c->inst[k].tile_begin_k1 = pos;
                while (pos < (int)t.size() && t[pos].inst == k) ++pos;
                c->inst[k].tile_count_k1 = pos - c->inst[k].tile_begin_k1;
            }
        }
    }
    // initial fields -> device staging -> equilibrium distributions
    double* stage = nullptr;
    e = hipMalloc((void**)&stage, 3 * c->max_nodes * sizeof(double));
    if (e != hipSuccess) return bail(hip_fail(c, e, "staging allocation"));
    for (int k = 0; k < n_inst; ++k) {
        const int64_t n = c->inst[k].n_nodes;
        e = hipMemcpy(stage, phi0[k], n * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(stage + n, ux0[k], n * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(stage + 2 * n, uy0[k], n * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_init(c->storage, c->qf, c->d_insts, k, c->inst[k].p.nx, c->inst[k].p.ny, stage,
                            stage + n, stage + 2 * n, c->f[0], c->g[0], c->q, c->rplane[0],
                            c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            (void)hipFree(stage);
            return bail(hip_fail(c, e, "initial state"));
        }
    }
    (void)hipFree(stage);
    c->cur = 0;
    c->streamed = true;
    c->step = 0;
    c->kernel = o.kernel == LBM_KERNEL_AUTO ? LBM_KERNEL_FUSED : o.kernel;
    c->tile_rows = o.tile_rows ? o.tile_rows : (c->storage == STORE_F64 ? 4 : 8);
    c->nt_store = o.stores == LBM_STORES_STREAMING;
    c->persistent = o.grid == LBM_GRID_PERSISTENT;
    c->strip = o.strip == 8 ? 1 : (o.strip == 16 ? 2 : 0);
    c->narrow = o.narrow_tiles == LBM_NARROW_ON ? 1 : 0;
    c->chunk = o.deal > 0 ? o.deal : 0;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess)
            c->num_cu = 0;
        c->device = dev;
        // the no-allocation scratch of this device, looked up once per device at set-up
        c->noalloc = noalloc_scratch_of(c, dev);
        if (!c->noalloc) return bail(LBM_ERR_DEVICE);
        const char* pb = getenv("LBM_PERSIST_BLOCKS");
        if (pb && *pb) c->persist_override = std::max(0, atoi(pb));
    }
    if (o.kernel == LBM_KERNEL_AUTO || o.tile_rows == 0 || o.stores == LBM_STORES_AUTO ||
        o.grid == LBM_GRID_AUTO || o.strip == LBM_STRIP_AUTO ||
        o.narrow_tiles == LBM_NARROW_AUTO || o.deal == LBM_DEAL_AUTO) {
        const std::string key = tune_key(c);
        if (!tune_cache_lookup(c, key)) {
            int rc = autotune(c);
            if (rc) return bail(rc);
            tune_cache_store(c, key);
        }
    }
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return bail(hip_fail(c, e, "init synchronise"));
    *out = c;
    return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t nsteps) {
    if (!c) return fail(nullptr, LBM_ERR_PARAM, "context is NULL");
    if (nsteps < 0) return fail(c, LBM_ERR_PARAM, "nsteps must be >= 0");
    int64_t left = nsteps;
    while (left > 0) {
        int64_t chunk = left;
        if (c->opt.check_every > 0) {
            const int64_t to_check = c->opt.check_every - (c->step % c->opt.check_every);
            chunk = std::min(chunk, to_check);
        }
        int64_t done = 0;
        while (done < chunk) {
            if (!c->streamed && c->opt.use_graph && chunk - done >= GRAPH_STEPS[0]) {
                int g = NGRAPH - 1;
                while (chunk - done < GRAPH_STEPS[g]) --g;
                if (!c->graph[g][c->cur]) {
                    int rc = capture_steps(c, g, c->cur);
                    if (rc) return rc;
                }
                hipError_t e = hipGraphLaunch(c->graph[g][c->cur], c->stream);
                if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
                done += GRAPH_STEPS[g];
                c->step += GRAPH_STEPS[g];
            } else {
                int rc = launch_one(c, c->stream);
                if (rc) return rc;
                done += 1;
                c->step += 1;
            }
        }
        left -= chunk;
        if (c->opt.check_every > 0 && c->step % c->opt.check_every == 0) {
            int rc = check_finite(c);
            if (rc) return rc;
        }
    }
    return LBM_OK;
}

int lbm_moments(lbm_ctx* c, int32_t inst, double* phi, double* rho, double* p, double* ux,
                double* uy) {
    if (!c) return fail(nullptr, LBM_ERR_PARAM, "context is NULL");
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, LBM_ERR_RANGE, "no such instance");
    int rc = moments_to(c, inst, c->mom);
    if (rc) return rc;
    const int64_t n = c->inst[inst].n_nodes;
    double* outs[5] = {phi, rho, p, ux, uy};
    for (int m = 0; m < 5; ++m)
        if (outs[m])
            HIPCHK(c, hipMemcpyAsync(outs[m], c->mom + m * n, n * sizeof(double),
                                     hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_moments_device(lbm_ctx* c, int32_t inst, double* d_out5) {
    if (!c) return fail(nullptr, LBM_ERR_PARAM, "context is NULL");
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, LBM_ERR_RANGE, "no such instance");
    if (!d_out5) return fail(c, LBM_ERR_PARAM, "output is NULL");
    return moments_to(c, inst, d_out5);
}

int lbm_reduce(lbm_ctx* c, int32_t inst, const double* mask, lbm_diag* out) {
    if (!c) return fail(nullptr, LBM_ERR_PARAM, "context is NULL");
    if (!out) return fail(c, LBM_ERR_PARAM, "output is NULL");
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, LBM_ERR_RANGE, "no such instance");
    double r[12];
    int rc = reduce_inst(c, inst, mask, r);
    if (rc) return rc;
    out->sum_phi = r[0];
    out->sum_rho = r[1];
    out->kinetic = r[2];
    out->max_u = r[3];
    out->min_rho = r[4];
    out->min_phi = r[5];
    out->max_phi = r[6];
    out->p_in = r[7];
    out->p_out = r[8];
    out->interface_crossings = r[9];
    out->spread_radius = r[10];
    out->nonfinite = (int64_t)r[11];
    out->step = c->step;
    return LBM_OK;
}

int lbm_reduce_noalloc(lbm_ctx* c, int32_t inst, const double* mask, lbm_diag* out) {
    if (!c) return fail(nullptr, LBM_ERR_PARAM, "context is NULL");
    if (!out) return fail(c, LBM_ERR_PARAM, "output is NULL");
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, LBM_ERR_RANGE, "no such instance");
    const Instance& I = c->inst[inst];
    if (I.n_nodes > NOALLOC_MAX_NODES) {
        char b[200];
        snprintf(b, sizeof b, "lbm_reduce_noalloc: instance %d has %lld nodes, more than the "
                 "%lld its fixed device scratch holds; use lbm_reduce", (int)inst,
                 (long long)I.n_nodes, (long long)NOALLOC_MAX_NODES);
        return fail(c, LBM_ERR_RANGE, b);
    }
    if (!c->noalloc) return fail(c, LBM_ERR_DEVICE, "no-allocation scratch unavailable");
    // the moment planes, the partials and the result, all in the device's fixed scratch;
    // every slot read is written first by this call's kernels, so nothing needs clearing
    double* mom = c->noalloc;
    double* partials = mom + 5 * NOALLOC_MAX_NODES;
    double* res = partials + NOALLOC_PARTIALS;
    int rc = moments_to(c, inst, mom);
    if (rc) return rc;
    double m[5] = {0, 0, 0, 0, -1};
    if (mask) memcpy(m, mask, sizeof m);
    hipError_t e = launch_reduce(mom, I.p.nx, I.p.ny, I.p.bc_ylo == LBM_BC_PERIODIC, m, partials,
                                 res, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reduce launch");
    HIPCHK(c, hipMemcpyAsync(c->h_red, res, 12 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double* r = c->h_red;
    out->sum_phi = r[0];
    out->sum_rho = r[1];
    out->kinetic = r[2];
    out->max_u = r[3];
    out->min_rho = r[4];
    out->min_phi = r[5];
    out->max_phi = r[6];
    out->p_in = r[7];
    out->p_out = r[8];
    out->interface_crossings = r[9];
    out->spread_radius = r[10];
    out->nonfinite = (int64_t)r[11];
    out->step = c->step;
    return LBM_OK;
}

int lbm_get_state(lbm_ctx* c, void* buf, size_t* bytes) {
    if (!c) return fail(nullptr, LBM_ERR_PARAM, "context is NULL");
    if (!bytes) return fail(c, LBM_ERR_PARAM, "bytes is NULL");
    const uint64_t bd = c->dist_elems * c->esize, bq = c->q_elems * sizeof(double);
    const uint64_t bp = c->mp_elems * sizeof(float);
    const uint64_t total = sizeof(StateHeader) + 2 * bd + bq + bp;
    if (!buf) {
        *bytes = total;
        return LBM_OK;
    }
    if (*bytes < total) return fail(c, LBM_ERR_RANGE, "state buffer too small");
    StateHeader h;
    memset(&h, 0, sizeof h);
    h.magic = STATE_MAGIC;
    h.version = STATE_VERSION;
    h.storage = c->storage;
    h.n_inst = (int32_t)c->inst.size();
    h.streamed = c->streamed ? 1 : 0;
    h.step = c->step;
    h.bytes_dist = bd;
    h.bytes_q = bq;
    h.bytes_mp = bp;
    h.total = total;
    h.layout = state_layout(c);
    char* b = (char*)buf;
    memcpy(b, &h, sizeof h);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(b + sizeof h, c->f[c->cur], bd, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(b + sizeof h + bd, c->g[c->cur], bd, hipMemcpyDeviceToHost));
    HIPCHK(c, copy_n(b + sizeof h + 2 * bd, c->q, bq, hipMemcpyDeviceToHost));
    HIPCHK(c, copy_n(b + sizeof h + 2 * bd + bq, c->rplane[c->cur], bp, hipMemcpyDeviceToHost));
    *bytes = total;
    return LBM_OK;
}

int lbm_set_state(lbm_ctx* c, const void* buf, size_t bytes) {
    if (!c) return fail(nullptr, LBM_ERR_PARAM, "context is NULL");
    if (!buf || bytes < sizeof(StateHeader)) return fail(c, LBM_ERR_PARAM, "state buffer too small");
    StateHeader h;
    memcpy(&h, buf, sizeof h);
    const uint64_t bd = c->dist_elems * c->esize, bq = c->q_elems * sizeof(double);
    const uint64_t bp = c->mp_elems * sizeof(float);
    if (h.magic != STATE_MAGIC || h.version != STATE_VERSION)
        return fail(c, LBM_ERR_PARAM, "not a state of this library");
    if (h.storage != c->storage || h.n_inst != (int32_t)c->inst.size() || h.bytes_dist != bd ||
        h.bytes_q != bq || h.bytes_mp != bp || h.total != bytes)
        return fail(c, LBM_ERR_PARAM, "state does not match this context");
    if (h.layout != state_layout(c))
        return fail(c, LBM_ERR_PARAM,
                    "state does not match this context (grid sizes, lattice or storage scales)");
    const char* b = (const char*)buf;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->f[0], b + sizeof h, bd, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->g[0], b + sizeof h + bd, bd, hipMemcpyHostToDevice));
    HIPCHK(c, copy_n(c->q, b + sizeof h + 2 * bd, bq, hipMemcpyHostToDevice));
    HIPCHK(c, copy_n(c->rplane[0], b + sizeof h + 2 * bd + bq, bp, hipMemcpyHostToDevice));
    c->cur = 0;
    c->streamed = h.streamed != 0;
    c->step = h.step;
    return LBM_OK;
}

int lbm_info(const lbm_ctx* c, int64_t* step, int32_t* kernel, int32_t* tile_rows,
             int32_t* stores, int32_t* grid, int32_t* strip, int32_t* narrow_tiles,
             int32_t* deal) {
    if (!c) return fail(nullptr, LBM_ERR_PARAM, "context is NULL");
    if (step) *step = c->step;
    if (kernel) *kernel = c->kernel;
    if (tile_rows) *tile_rows = c->tile_rows;
    if (stores) *stores = c->nt_store ? LBM_STORES_STREAMING : LBM_STORES_CACHED;
    if (grid) *grid = runs_persistent(c) ? LBM_GRID_PERSISTENT : LBM_GRID_TILES;
    if (strip) *strip = c->strip == 0 ? LBM_STRIP_ROWS : STRIP_TILES[c->strip];
    if (narrow_tiles) *narrow_tiles = c->narrow ? LBM_NARROW_ON : LBM_NARROW_OFF;
    if (deal) {
        // what the steps run with: a chunk shorter than an XCD's band, else one band per XCD
        const int per =
            (c->lists[list_index(c->tile_rows)][c->strip][c->narrow].count + NXCD - 1) / NXCD;
        *deal = (c->chunk > 0 && c->chunk < per && !runs_persistent(c)) ? c->chunk
                                                                          : LBM_DEAL_BANDS;
    }
    return LBM_OK;
}

const char* lbm_build_id(void) { return LBM_SOURCE_SHA256; }

const char* lbm_last_error(const lbm_ctx* c) {
    return c ? c->err.c_str() : g_thread_err.c_str();
}

void lbm_destroy(lbm_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);   // nothing to report to
    free_all(c);
    delete c;
}

}  // extern "C"
