// bgk_api.hip -- host side of libbgk.so: validation, layout, launches.
// The C ABI is declared in include/bgk.h.
#include "bgk_adjoint.h"
#include "bgk_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bgk.h"

using namespace bgk;

// Start value of the rounding counter (a vector store by one lane).
__global__ void k_set_pass(uint32_t *pass, uint32_t v)
{
    if (threadIdx.x == 0) pass[0] = v;
}


struct bgk_ctx {
    int precision = BGK_FP64;
    int dim = 1;
    int ninst = 0;
    int device = 0;
    std::vector<bgk_problem> probs;
    std::vector<Inst> h_inst;
    std::vector<int> h_cell_prefix, h_pseudo_prefix;
    Geo geo{};
    int ncells = 0, npseudo = 0;
    size_t f_elems = 0;
    int vsplit = 1;            // jz chunks per cell (one workgroup each)
    int vsplit_max = 1;        // largest vsplit the partial-sum buffer holds
    int vec = 1;               // streaming kernel: jx per lane task
    int zr = 1;                // streaming kernel: jz residues per workgroup
    int sblock = 256;          // streaming kernel: threads per workgroup
    int unroll = 1;            // streaming kernel: jz values whose loads are issued together
    int persist = 0;           // streaming kernel: 0 one workgroup per item, else resident workgroups per CU
    bool shift = false;        // every instance streams in the translation form (k_shift)
    // translation form in row tiles (k_shift_rows, the shape's unroll = 2):
    // cells per tile, log2 lanes per cell, window cells, tiles, LDS bytes
    bool row_ok = false, row_pcache = false;  // row_pcache: v_x table values in the source list
    int row_tt = 0, row_lg = 0, row_wmax = 0, row_ntiles = 0;
    size_t row_lds_bytes = 0;
    bool conservative = false; // some instance relaxes with the effective Maxwellian parameters
    // hipGraph replay of whole bgk_step calls (every launch after the one that
    // sets the rounding counter); key: (f_in, f_out, workspace, steps).
    bool use_graph = false;
    struct Chunk {
        const void *f_in, *f_out, *ws;
        int n;
        hipGraphExec_t exec;
        unsigned long long used;  // last use, for eviction
    };
    std::vector<Chunk> chunks;
    unsigned long long graph_clock = 0;
    int ncu = 256;             // compute units of the device
    double tuned_us = 0.0;     // streaming-kernel time of the chosen shape when autotuned
    // current streaming pass: table parity it reads
    int pass_parity = 0;
    size_t esize = 8;
    // device memory owned by the context (per-cell and per-entry data only;
    // every f-sized buffer is the caller's)
    Inst *d_inst = nullptr;
    int *d_cell_prefix = nullptr, *d_pseudo_prefix = nullptr;
    void *work = nullptr;      // the caller's workspace during a bgk_step call (ping-pong buffer)
    void *params = nullptr;    // 2 x (ncells + npseudo) * pe elements (parity buffers)
    double *partial = nullptr; // ncells * vsplit_max * NQ
    double *mom = nullptr;     // ncells * 5 (bgk_check)
    // reverse sweep (allocated at the first bgk_step_adjoint / bgk_lid_shear call)
    bool adj_ready = false;
    bool mixed = false;        // instances of different dimensions
    int lds_max = 65536;       // device LDS per workgroup (bytes)
    void *adj_h = nullptr, *adj_hb = nullptr;                     // during a reverse step: h = S(R_a f), abar
    void *adj_rec = nullptr;                                      // and the branch record of h's streaming pass
                                                                  // (the two halves of the caller's workspace)
    double *info_f = nullptr, *info_h = nullptr;                  // ncells * NINFO
    double *adj_sums = nullptr, *adj_wsum = nullptr;              // ncells * vsplit_max * (NSUM, NWALL)
    double *adj_coef = nullptr;                                   // ncells * NCOEF
    double *adj_dw = nullptr;                                     // ninst * 4 walls * (D, D')
    int *wall_cells = nullptr;                                    // perimeter cells of the cavities
    int n_wall_cells = 0;
    double *gk = nullptr, *gt = nullptr, *lid = nullptr;          // ncells, ncells, 2 * ncells
    double *lid_L = nullptr;                                      // ninst (bgk_cavity_metrics)
    int *flags = nullptr;
    // stochastic rounding of FP32 stores: device pass counter and the value
    // the next bgk_step starts it from
    uint32_t *pass = nullptr;
    uint32_t seed = 0;
    // timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t ev_used = 0;
    std::string err;
};

static thread_local std::string g_init_error;

static int fail(bgk_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    else g_init_error = msg;
    return code;
}

#define HIP_TRY(ctx, call)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ctx, BGK_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

static const double kGamma = 5.0 / 3.0;

// Spatial dimension of a problem kind.
static int kind_dim(int k)
{
    if (k == BGK_CAVITY_3D || k == BGK_PERIODIC_3D) return 3;
    if (k == BGK_CAVITY_2D || k == BGK_PERIODIC_2D) return 2;
    return 1;
}

static Args make_args(const bgk_ctx *c)
{
    Args a;
    a.inst = c->d_inst;
    a.cell_prefix = c->d_cell_prefix;
    a.pseudo_prefix = c->d_pseudo_prefix;
    a.ninst = c->ninst;
    a.ncells = c->ncells;
    a.npseudo = c->npseudo;
    a.vsplit = c->vsplit;
    a.zr = c->zr;
    a.nparts = c->vsplit;
    a.ntiles = c->row_ntiles;
    a.pass = c->pass;
    a.rec = nullptr;
    a.g = c->geo;
    return a;
}

// LDS of the streaming kernel after its tables: 8 bytes of alignment, the
// per-thread moment sums (NQ doubles per thread in 3D, 9 without the z half
// fluxes otherwise) and the node tables (v_z and v_z^2 per plane, v_x, v_y).
static size_t stream_acc_bytes(const Geo &g, int dim, int block)
{
    const size_t nacc = dim == 3 ? NQ : 9;
    return 8 + (nacc * block + 2 * g.nvz + g.nvx + g.nvy) * sizeof(double);
}

static void drop_graphs(bgk_ctx *c);

static void release(bgk_ctx *c)
{
    if (!c) return;
    (void)hipFree(c->d_inst);
    (void)hipFree(c->d_cell_prefix);
    (void)hipFree(c->d_pseudo_prefix);
    (void)hipFree(c->params);
    (void)hipFree(c->partial);
    (void)hipFree(c->mom);
    for (double *q : {c->info_f, c->info_h, c->adj_sums, c->adj_wsum, c->adj_coef, c->adj_dw, c->gk, c->gt, c->lid})
        (void)hipFree(q);
    (void)hipFree(c->lid_L);
    (void)hipFree(c->wall_cells);
    (void)hipFree(c->flags);
    (void)hipFree(c->pass);
    for (auto &e : c->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    drop_graphs(c);
    delete c;
}

// Time step from the Courant rule: dt = cfl / max_j sum_d |v_d(j)| / dx_d
// over the streaming directions.
static double courant_rate(const bgk_problem &p, int dim)
{
    const double len[3] = {p.x1 - p.x0, dim >= 2 ? p.y1 - p.y0 : 1.0, dim == 3 ? p.z1 - p.z0 : 1.0};
    const int n[3] = {p.nx, p.ny, p.nz};
    double r = 0.0;
    for (int a = 0; a < dim; ++a) {
        double m = 0.0;
        for (int k = 0; k < p.nv[a]; ++k)
            m = std::max(m, std::fabs(p.vlo[a] + (k + 0.5) * (p.vhi[a] - p.vlo[a]) / p.nv[a]));
        r += m / (len[a] / n[a]);
    }
    return r;
}

// Planes of the velocity grid with v_z < 0 (they come first).
static int negative_planes(const bgk_problem &p)
{
    int n = 0;
    for (int k = 0; k < p.nv[2]; ++k)
        if (p.vlo[2] + (k + 0.5) * (p.vhi[2] - p.vlo[2]) / p.nv[2] < 0.0) ++n;
    return n;
}

static int validate(const bgk_problem &p, int idx, std::string &msg)
{
    char b[256];
    auto bad = [&](const char *what) {
        snprintf(b, sizeof b, "problem %d: %s", idx, what);
        msg = b;
        return BGK_E_INVALID;
    };
    if (p.kind < 0 || p.kind > 5) return bad("unknown kind");
    const int dim = kind_dim(p.kind);
    if (p.nx < 1 || (dim >= 2 && p.ny < 1) || (dim == 3 && p.nz < 1)) return bad("nx, ny, nz must be >= 1");
    if (p.kind == BGK_PERIODIC_1D && p.nx < 2) return bad("periodic boxes need nx >= 2");
    if (p.kind == BGK_PERIODIC_2D && (p.nx < 2 || p.ny < 2)) return bad("periodic boxes need nx, ny >= 2");
    if (p.kind == BGK_PERIODIC_3D && (p.nx < 2 || p.ny < 2 || p.nz < 2))
        return bad("periodic boxes need nx, ny, nz >= 2");
    if (!(p.x1 > p.x0) || (dim >= 2 && !(p.y1 > p.y0)) || (dim == 3 && !(p.z1 > p.z0)))
        return bad("empty spatial box");
    for (int a = 0; a < 3; ++a) {
        if (a == 1 && p.reduced && dim == 1 && p.nv[1] == 1) continue;  // the single node v_y = 0
        if (p.nv[a] < 2 || p.nv[a] > NVMAX) {
            msg = "velocity cells per component must be in [2, 128]";
            return BGK_E_UNSUPPORTED;
        }
        if (!(p.vhi[a] > p.vlo[a])) return bad("empty velocity box");
    }
    if (!(p.kn > 0.0) || !std::isfinite(p.kn)) return bad("Kn must be > 0");
    if (!std::isfinite(p.omega)) return bad("omega must be finite");
    if (p.splitting != BGK_STRANG && p.splitting != BGK_LIE) return bad("unknown splitting");
    if (p.limiter != BGK_MINMOD && p.limiter != BGK_NOLIMIT && p.limiter != BGK_SHIFT) return bad("unknown limiter");
    if (p.maxwellian != BGK_POINT && p.maxwellian != BGK_CONSERVATIVE) return bad("unknown Maxwellian form");
    if (p.reduced != 0 && p.reduced != 1) return bad("reduced must be 0 or 1");
    if (p.reduced && (p.nv[2] != 2 || (dim == 1 && p.nv[1] != 1))) {
        snprintf(b, sizeof b, "problem %d: the reduced velocity space takes nv[2] = 2 (and nv[1] = 1 for "
                              "one-dimensional kinds)", idx);
        msg = b;
        return BGK_E_UNSUPPORTED;
    }
    if (dim == 3 && p.reduced) {
        snprintf(b, sizeof b, "problem %d: three-dimensional kinds stream along v_z (no reduced space)", idx);
        msg = b;
        return BGK_E_UNSUPPORTED;
    }
    if (dim == 3 && negative_planes(p) % 2) {
        snprintf(b, sizeof b, "problem %d: v_z must change sign at an even plane (nv[2] divisible by 4 on a "
                              "symmetric box)", idx);
        msg = b;
        return BGK_E_UNSUPPORTED;
    }
    if (p.limiter == BGK_SHIFT && dim >= 2) {
        snprintf(b, sizeof b, "problem %d: shift streaming is one-dimensional", idx);
        msg = b;
        return BGK_E_UNSUPPORTED;
    }
    if (p.kind == BGK_SHOCK_1D && !(p.mach > 1.0)) return bad("shock needs Mach > 1");
    if ((p.kind == BGK_CAVITY_2D || p.kind == BGK_CAVITY_3D) && !(p.t_wall > 0.0))
        return bad("wall temperature must be > 0");
    if (!(p.dt > 0.0) && !(p.cfl > 0.0)) return bad("need dt > 0 or cfl > 0");
    const double rate = courant_rate(p, dim);
    const double dt = p.dt > 0.0 ? p.dt : p.cfl / rate;
    if (p.limiter != BGK_SHIFT && dt * rate > 2.0 / 3.0 * (1.0 + 1e-12)) {
        snprintf(b, sizeof b, "problem %d: Courant sum %.6g exceeds 2/3", idx, dt * rate);
        msg = b;
        return BGK_E_CFL;
    }
    return BGK_OK;
}

// Launch shape of the streaming kernel.
//  vec:    jx values per lane task (16-byte loads where the grid allows);
//          valid when it divides Nvx and every group of vec consecutive v_x
//          has one sign;
//  vsplit: jz chunks per cell, one workgroup each;
//  unroll: jz values per software-pipeline stage;
//  zr, sblock: lane tasks = (Nvx/vec) * Nvy * zr fill whole waves; the block is
//          the largest multiple of 64 up to 256 dividing the task count.
static bool vec_valid(const bgk_ctx *c, int v)
{
    const Geo &g = c->geo;
    if (v == 1) return true;
    if (c->shift) return false;  // the translation-form kernel takes one jx per lane task
    if (g.red) return false;     // reduced: the column fold needs one jx per lane task
    if (v == 4 && c->precision == BGK_FP64) return false;
    if (c->dim == 3) return false;  // ten taps per lane: one jx per lane task
    if (g.nvx % v) return false;
    for (int k = 0; k < g.nvx; k += v) {
        const double a = g.lo[0] + (k + 0.5) * g.dv[0], b = g.lo[0] + (k + v - 0.5) * g.dv[0];
        if (!((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0))) return false;
    }
    return true;
}

static void drop_chunk(bgk_ctx::Chunk &k)
{
    if (k.exec) (void)hipGraphExecDestroy(k.exec);
    k.exec = nullptr;
}

static void drop_graphs(bgk_ctx *c)
{
    for (auto &k : c->chunks) drop_chunk(k);
    c->chunks.clear();
}

// Smallest jz residue count zr that makes the lane tasks (Nvx/vec) * Nvy * zr
// fill whole waves, and the largest block (a multiple of 64 up to 256)
// dividing the task count.
static void task_shape(const Geo &g, int vec, int zchunk, int *zr_out, int *block_out)
{
    const int groups = g.npl / vec;
    *zr_out = 1;
    *block_out = 256;
    for (int zr = 1; zr <= std::max(1, zchunk / 2); ++zr) {
        const int t = groups * zr;
        if (t % 64) continue;
        *zr_out = zr;
        for (int b = 256; b >= 64; b -= 64)
            if (t % b == 0) { *block_out = b; break; }
        return;
    }
    // reduced velocity space with planes of fewer than 64 lane groups (one-
    // dimensional problems: N_vx values per plane): one wave per workgroup,
    // filled with as many jz residues as the chunk has
    if (g.red && groups < 64) {
        *zr_out = std::max(1, std::min(zchunk, (64 + groups - 1) / groups));
        *block_out = 64;
    }
}

static void set_shape(bgk_ctx *c, int vec, int unroll, int vsplit, int persist = 0)
{
    drop_graphs(c);
    const Geo &g = c->geo;
    c->vec = vec;
    c->unroll = unroll;
    c->persist = persist;
    c->vsplit = std::max(1, std::min(c->vsplit_max, vsplit));
    if (c->shift && unroll == 2) c->vsplit = g.nvz;  // row tiles: one plane per work item
    task_shape(g, c->vec, g.nvz / c->vsplit, &c->zr, &c->sblock);
}

static int vsplit_for(const bgk_ctx *c, int target_wg)
{
    return std::max(1, std::min(c->geo.nvz, (target_wg + c->ncells - 1) / c->ncells));
}

// Translation form in row tiles: lanes per cell G = 2^lg >= N_vx (at most
// 64), 4 (cell, jx) pairs per lane of a ROW_THREADS-lane workgroup, TT = 4 ROW_THREADS / G - 1
// cells per tile; per instance the first tile and the reach of its sources
// below and above a tile (the largest shift m + 1 of each sign, plus one
// cell of margin); the window (TT + both reaches, at most ROW_THREADS
// cells) and the list of its needed sources set the LDS size, the list
// holding the sources' v_x table values too when they fit.
static void plan_rows(bgk_ctx *c)
{
    const Geo &g = c->geo;
    c->row_ok = false;
    if (g.nvx > 64) return;
    int lg = 0;
    while ((1 << lg) < g.nvx) ++lg;
    const int tt = ((4 * ROW_THREADS) >> lg) - 1;  // (tt + 1) N_vx sources fill ROW_EPL = 4 per lane
    int reach = 0, tiles = 0;
    for (Inst &I : c->h_inst) {
        int lo = 0, hi = 0;
        for (int k = 0; k < g.nvx; ++k) {
            const double vx = g.lo[0] + (k + 0.5) * g.dv[0];
            const int m = (int)std::floor(std::fabs(vx) * I.cx);
            if (vx > 0.0) lo = std::max(lo, m + 2);
            else hi = std::max(hi, m + 2);
        }
        I.reach_lo = lo;
        I.reach_hi = hi;
        I.tile0 = tiles;
        tiles += (I.nx + tt - 1) / tt;
        reach = std::max(reach, lo + hi);
    }
    const int wmax = tt + reach;
    if (wmax > ROW_THREADS) return;  // one window cell per lane
    // the v_x table values kept in the source list when they fit
    size_t lds = c->esize == 4 ? row_lds<float, true>(g.nvx, tt, wmax).total : row_lds<double, true>(g.nvx, tt, wmax).total;
    bool pc = true;
    if (lds > (size_t)c->lds_max) {
        pc = false;
        lds = c->esize == 4 ? row_lds<float, false>(g.nvx, tt, wmax).total : row_lds<double, false>(g.nvx, tt, wmax).total;
    }
    if (lds > (size_t)c->lds_max) return;
    c->row_ok = true;
    c->row_pcache = pc;
    c->row_tt = tt;
    c->row_lg = lg;
    c->row_wmax = wmax;
    c->row_ntiles = tiles;
    c->row_lds_bytes = lds;
}

// Default shape (measured on MI355X for the paper's grids; bgk_autotune refines it).
static void choose_launch(bgk_ctx *c)
{
    // up to 4 jz chunks per cell even on large grids: smaller work items keep
    // the y-neighbour rows of the cells in flight resident in each XCD's L2
    c->vsplit_max = std::max(vsplit_for(c, 8192), std::min(c->geo.nvz, 4));
    if (c->row_ok) c->vsplit_max = std::max(c->vsplit_max, c->geo.nvz);
    int vec = 1;
    for (int v : {4, 2})
        if (vec_valid(c, v)) { vec = v; break; }
    if (c->dim >= 2) vec = 1;
    int unroll = (c->dim == 1 && c->precision == BGK_FP32 && !c->shift) ? 2 : 1;
    // translation form: row tiles when their plane-by-tile items fill the device
    if (c->shift && c->row_ok && c->row_ntiles * c->geo.nvz >= c->ncu) unroll = 2;
    const int target = c->dim == 1 ? (c->precision == BGK_FP32 ? 1024 : 512) : 2048;
    set_shape(c, vec, unroll, vsplit_for(c, target));
}

// Host-side set-up of a context: validation, geometry, instance tables,
// time steps and the default launch shape.  No device memory is touched.
// Returns a status code and sets msg on failure.
static int plan_ctx(const bgk_problem *probs, int n_probs, int precision, bgk_ctx *c, std::string &msg)
{
    if (!probs || n_probs < 1) {
        msg = "need at least one problem";
        return BGK_E_INVALID;
    }
    if (precision != BGK_FP64 && precision != BGK_FP32) {
        msg = "unknown precision";
        return BGK_E_INVALID;
    }
    for (int i = 0; i < n_probs; ++i) {
        int rc = validate(probs[i], i, msg);
        if (rc) return rc;
        const bgk_problem &p = probs[i], &q = probs[0];
        const char *why = nullptr;
        if (p.reduced != q.reduced) why = "all instances must share the velocity space (reduced or not)";
        else if (p.reduced && kind_dim(p.kind) != kind_dim(q.kind))
            why = "the reduced velocity space differs by dimension: no mixed-dimension batch";
        else if ((p.limiter == BGK_SHIFT) != (q.limiter == BGK_SHIFT))
            why = "shift streaming cannot share a context with other limiters";
        for (int a = 0; a < 3 && !why; ++a)
            if (p.nv[a] != q.nv[a] || p.vlo[a] != q.vlo[a] || p.vhi[a] != q.vhi[a])
                why = "all instances must share the velocity grid";
        if (why) {
            msg = why;
            return BGK_E_UNSUPPORTED;
        }
    }
    c->precision = precision;
    c->esize = precision == BGK_FP64 ? 8 : 4;
    c->ninst = n_probs;
    // a batch mixing dimensions runs the kernels of the highest one
    c->dim = 1;
    for (int i = 0; i < n_probs; ++i) {
        c->dim = std::max(c->dim, kind_dim(probs[i].kind));
        if (kind_dim(probs[i].kind) != kind_dim(probs[0].kind)) c->mixed = true;
    }
    c->shift = probs[0].limiter == BGK_SHIFT;
    c->probs.assign(probs, probs + n_probs);
    (void)hipGetDevice(&c->device);
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && ncu > 0)
            c->ncu = ncu;
    }

    Geo &g = c->geo;
    g.nvx = probs[0].nv[0];
    g.nvy = probs[0].nv[1];
    g.nvz = probs[0].nv[2];
    g.npl = g.nvx * g.nvy;
    g.nv = (long long)g.npl * g.nvz;
    g.dV = 1.0;
    g.red = probs[0].reduced ? (c->dim == 2 ? 1 : 2) : 0;
    g.zneg = g.red ? 0 : negative_planes(probs[0]);
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = probs[0].vlo[a];
        g.dv[a] = (probs[0].vhi[a] - probs[0].vlo[a]) / probs[0].nv[a];
        if (a == 2 && g.red) {  // the two planes are integrals over v_z (and v_y)
            g.lo[a] = 0.0;
            g.dv[a] = 1.0;
        }
        if (a == 1 && g.red == 2) {  // the single node v_y = 0
            g.lo[a] = -0.5;
            g.dv[a] = 1.0;
        }
        g.dV *= g.dv[a];
    }
    g.tx1 = 4;
    g.ty1 = g.tx1 + g.nvx;
    g.tx2 = g.ty1 + g.nvy;
    g.ty2 = g.tx2 + g.nvx;
    g.tz = (g.ty2 + g.nvy + 1) & ~1;
    g.pe = (g.tz + 2 * g.nvz + 3) & ~3;
    {
        // LDS per workgroup: the table entries of every stencil slot (1 + 6
        // dim for the step; 17 and 9 for the reverse sweep of 2D and 1D
        // kinds) plus a few KB of static buffers
        int lds_max = 0;
        if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess ||
            lds_max <= 0)
            lds_max = 65536;
        const size_t entry = (size_t)g.pe * c->esize, slack = 4096;
        const size_t fwd = (size_t)(1 + 6 * c->dim) * entry + slack + stream_acc_bytes(g, c->dim, 256);
        c->lds_max = lds_max;
        if (fwd > (size_t)lds_max) {
            char b[160];
            snprintf(b, sizeof b, "velocity grid needs %zu bytes of LDS per workgroup; the device allows %d", fwd,
                     lds_max);
            msg = b;
            return BGK_E_UNSUPPORTED;
        }
    }

    c->h_cell_prefix.push_back(0);
    c->h_pseudo_prefix.push_back(0);
    long long f_off = 0;
    for (int i = 0; i < n_probs; ++i) {
        const bgk_problem &p = probs[i];
        const int dim = kind_dim(p.kind);
        Inst I{};
        I.kind = p.kind;
        I.nx = p.nx;
        I.ny = dim >= 2 ? p.ny : 1;
        I.nz = dim == 3 ? p.nz : 1;
        if ((long long)I.nx * I.ny * I.nz >= (1LL << 30)) {
            msg = "one instance must have fewer than 2^30 cells";
            return BGK_E_UNSUPPORTED;
        }
        I.ncell = I.nx * I.ny * I.nz;
        I.cell0 = c->h_cell_prefix.back();
        I.strang = p.splitting == BGK_STRANG;
        I.minmod = p.limiter == BGK_MINMOD;
        I.shift = p.limiter == BGK_SHIFT;
        I.conservative = p.maxwellian == BGK_CONSERVATIVE;
        if (I.conservative) c->conservative = true;
        I.f0 = f_off;
        const double dx = (p.x1 - p.x0) / p.nx, dy = dim >= 2 ? (p.y1 - p.y0) / p.ny : 1.0,
                     dz = dim == 3 ? (p.z1 - p.z0) / p.nz : 1.0;
        I.dt = p.dt > 0.0 ? p.dt : p.cfl / courant_rate(p, dim);
        I.cx = I.dt / dx;
        I.cy = dim >= 2 ? I.dt / dy : 0.0;
        I.cz = dim == 3 ? I.dt / dz : 0.0;
        I.kn = p.kn;
        I.omega = p.omega;
        I.tw = p.t_wall;
        I.uw = p.lid_mach * std::sqrt(kGamma / 2.0);
        I.x0 = p.x0;
        I.dx = dx;
        if (p.kind == BGK_SHOCK_1D) {
            // Eq. (RH) with upstream n = T = 1, V = M sqrt(gamma / 2).
            const double m2 = p.mach * p.mach, r = 4.0 * m2 / (m2 + 3.0);
            I.up[0] = 1.0;
            I.up[1] = p.mach * std::sqrt(kGamma / 2.0);
            I.up[2] = 1.0;
            I.dn[0] = r;
            I.dn[1] = I.up[1] / r;
            I.dn[2] = (5.0 * m2 - 1.0) * (m2 + 3.0) / (16.0 * m2);
        }
        // ghost entries: the two far fields, or one per face cell of each wall
        const int np = p.kind == BGK_SHOCK_1D    ? 2
                       : p.kind == BGK_CAVITY_2D ? 2 * I.nx + 2 * I.ny
                       : p.kind == BGK_CAVITY_3D ? 2 * (I.ny * I.nz + I.nx * I.nz + I.nx * I.ny)
                                                 : 0;
        if ((long long)I.ncell * g.nv * (long long)c->esize >= (1LL << 31) * 2LL) {
            msg = "one instance must hold fewer than 2^32 bytes of f";
            return BGK_E_UNSUPPORTED;
        }
        c->h_inst.push_back(I);
        c->h_cell_prefix.push_back(I.cell0 + I.ncell);
        c->h_pseudo_prefix.push_back(c->h_pseudo_prefix.back() + np);
        f_off += (long long)I.ncell * g.nv;
    }
    c->ncells = c->h_cell_prefix.back();
    c->npseudo = c->h_pseudo_prefix.back();
    for (int i = 0; i < n_probs; ++i) c->h_inst[i].pseudo0 = c->ncells + c->h_pseudo_prefix[i];
    c->f_elems = (size_t)f_off;
    if (c->shift) plan_rows(c);

    choose_launch(c);
    return BGK_OK;
}

extern "C" int bgk_init(const bgk_problem *probs, int n_probs, int precision, bgk_ctx **out)
{
    if (!out) return fail(nullptr, BGK_E_INVALID, "out is NULL");
    *out = nullptr;
    bgk_ctx *c = new bgk_ctx;
    {
        std::string msg;
        const int rc = plan_ctx(probs, n_probs, precision, c, msg);
        if (rc) {
            delete c;
            return fail(nullptr, rc, msg);
        }
    }
    const Geo &g = c->geo;

#define ALLOC(ptr, bytes)                                                         \
    do {                                                                          \
        hipError_t e_ = hipMalloc((void **)&(ptr), (bytes));                      \
        if (e_ != hipSuccess) {                                                   \
            std::string m_ = std::string("hipMalloc: ") + hipGetErrorString(e_); \
            release(c);                                                           \
            return fail(nullptr, BGK_E_HIP, m_);                                  \
        }                                                                         \
    } while (0)
    ALLOC(c->d_inst, sizeof(Inst) * n_probs);
    ALLOC(c->d_cell_prefix, sizeof(int) * (n_probs + 1));
    ALLOC(c->d_pseudo_prefix, sizeof(int) * (n_probs + 1));
    ALLOC(c->params, 2 * (size_t)(c->ncells + c->npseudo) * g.pe * c->esize);
    ALLOC(c->partial, sizeof(double) * (size_t)c->ncells * c->vsplit_max * NQ);
    ALLOC(c->mom, sizeof(double) * (size_t)c->ncells * 5);
    ALLOC(c->flags, sizeof(int));
    ALLOC(c->pass, sizeof(uint32_t));
#undef ALLOC
    hipError_t e1 = hipMemcpy(c->d_inst, c->h_inst.data(), sizeof(Inst) * n_probs, hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(c->d_cell_prefix, c->h_cell_prefix.data(), sizeof(int) * (n_probs + 1), hipMemcpyHostToDevice);
    hipError_t e3 = hipMemcpy(c->d_pseudo_prefix, c->h_pseudo_prefix.data(), sizeof(int) * (n_probs + 1), hipMemcpyHostToDevice);
    hipError_t e4 = hipMemset(c->pass, 0, sizeof(uint32_t));
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
        release(c);
        return fail(nullptr, BGK_E_HIP, "hipMemcpy of instance tables failed");
    }
    *out = c;
    return BGK_OK;
}

extern "C" int bgk_free(bgk_ctx *ctx)
{
    if (!ctx) return BGK_E_INVALID;
    (void)hipDeviceSynchronize();
    release(ctx);
    return BGK_OK;
}

extern "C" const char *bgk_last_error(const bgk_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

// Reverse-step workspace: h = S(R_a f_n), the streamed adjoint (f-sized
// each) and the branch record of h's streaming pass (one byte per element,
// rounded up to 256 bytes).
static size_t adjoint_ws_bytes(const bgk_ctx *c)
{
    return 2 * c->f_elems * c->esize + ((c->f_elems + 255) & ~(size_t)255);
}

extern "C" int bgk_sizes(const bgk_ctx *ctx, size_t *f_elems, size_t *n_cells, size_t *ws_step_bytes,
                         size_t *ws_adjoint_bytes)
{
    if (!ctx) return BGK_E_INVALID;
    const size_t fb = ctx->f_elems * ctx->esize;
    if (f_elems) *f_elems = ctx->f_elems;
    if (n_cells) *n_cells = (size_t)ctx->ncells;
    if (ws_step_bytes) *ws_step_bytes = fb;  // the ping-pong buffer of bgk_step
    if (ws_adjoint_bytes) *ws_adjoint_bytes = adjoint_ws_bytes(ctx);
    return BGK_OK;
}

extern "C" int bgk_instance_info(const bgk_ctx *ctx, int inst, size_t *f_offset, size_t *cell_offset, double *dt)
{
    if (!ctx || inst < 0 || inst >= ctx->ninst) return BGK_E_INVALID;
    const Inst &I = ctx->h_inst[inst];
    if (f_offset) *f_offset = (size_t)I.f0;
    if (cell_offset) *cell_offset = (size_t)I.cell0;
    if (dt) *dt = I.dt;
    return BGK_OK;
}

// ------------------------------------------------------------- launches

template <typename real>
static real *params_buf(bgk_ctx *c, int parity)
{
    return (real *)c->params + (size_t)parity * (c->ncells + c->npseudo) * c->geo.pe;
}

// Jx values per lane of the pointwise kernels (16-byte loads where Nvx allows).
// Threads per workgroup of a kernel whose threads stride over `ntask` tasks
// of one plane: the multiple of 64 up to 256 that leaves the fewest idle
// lanes in the last round (the larger on a tie), e.g. 192 for 144 or 576.
static int fit_block(int ntask)
{
    int best = 256, idle = 1 << 30;
    for (int b = 256; b >= 64; b -= 64) {
        const int w = (ntask + b - 1) / b * b - ntask;
        if (w < idle) { best = b; idle = w; }
    }
    return best;
}

static int pointwise_vec(const bgk_ctx *c)
{
    const int want = c->precision == BGK_FP32 ? 4 : 2;
    for (int v = want; v > 1; v /= 2)
        if (c->geo.nvx % v == 0) return v;
    return 1;
}

// Workgroup of the moment and closing-relaxation kernels (VEC jx per task).
static int pointwise_block(const bgk_ctx *c) { return fit_block(c->geo.npl / pointwise_vec(c)); }

// Arguments of the pointwise kernels (moments, initial state, closing
// relaxation): their own jz chunk count, the streaming one except for the
// row-tile translation form, whose one chunk per plane would leave these
// kernels mostly empty workgroups; the moment sums still fill every one of
// the nparts slots per cell that the table preparation adds up.
static Args pointwise_args(const bgk_ctx *c)
{
    Args a = make_args(c);
    if (c->shift && c->unroll == 2) a.vsplit = std::min(c->vsplit, vsplit_for(c, 2048));
    return a;
}

template <typename real>
static int launch_moments(bgk_ctx *c, const void *f, hipStream_t s)
{
    const Args a = pointwise_args(c);
    const int nb = c->ncells * a.vsplit;
    if (pointwise_vec(c) == 4)
        hipLaunchKernelGGL((k_moments<real, 4>), dim3(nb), dim3(pointwise_block(c)), 0, s, a, (const real *)f, c->partial);
    else if (pointwise_vec(c) == 2)
        hipLaunchKernelGGL((k_moments<real, 2>), dim3(nb), dim3(pointwise_block(c)), 0, s, a, (const real *)f, c->partial);
    else
        hipLaunchKernelGGL((k_moments<real, 1>), dim3(nb), dim3(pointwise_block(c)), 0, s, a, (const real *)f, c->partial);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

template <typename real>
static int launch_prep(bgk_ctx *c, int mode, int nparts, int parity, hipStream_t s)
{
    const int ne = c->ncells + (mode == MODE_FINAL ? 0 : c->npseudo);
    Args a = make_args(c);
    a.nparts = nparts;
    real *copy = mode == MODE_FIRST ? params_buf<real>(c, 1 - parity) : nullptr;
    // lanes per entry: the smallest of 16, 32, 64 that holds the largest velocity axis
    const int nvmax = std::max(c->geo.nvx, std::max(c->geo.nvy, c->geo.nvz));
    const int w = nvmax <= 16 ? 16 : nvmax <= 32 ? 32 : 64;
    const int per_block = 4 * (64 / w);
    real *pb = params_buf<real>(c, parity);
    // cells, then (with their own kernel) the ghost sources
    auto go = [&](auto kern, int first, int count) {
        if (count > 0)
            hipLaunchKernelGGL(kern, dim3((count + per_block - 1) / per_block), dim3(256), 0, s, a, c->partial, pb,
                               mode, ne, copy);
    };
    auto both = [&](auto cells, auto ghosts) {
        go(cells, 0, c->ncells);
        go(ghosts, c->ncells, ne - c->ncells);
    };
    if (c->conservative) {
        if (w == 16) both(k_prep<real, 16, false, true>, k_prep<real, 16, true, true>);
        else if (w == 32) both(k_prep<real, 32, false, true>, k_prep<real, 32, true, true>);
        else both(k_prep<real, 64, false, true>, k_prep<real, 64, true, true>);
    } else {
        if (w == 16) both(k_prep<real, 16, false, false>, k_prep<real, 16, true, false>);
        else if (w == 32) both(k_prep<real, 32, false, false>, k_prep<real, 32, true, false>);
        else both(k_prep<real, 64, false, false>, k_prep<real, 64, true, false>);
    }
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

// The next pass reads what this one writes.  While both f buffers fit in the
// 256 MB last-level cache (MALL) plain stores leave the output there (the
// 256 x 32^3 FP64 shock runs 30 us instead of 43 us per pass); larger working
// sets use non-temporal stores, measured faster for them.
// LDS of the role-ordered z-tables of the one-residue kernels:
// [sign combination][jz][tap role][2] values; roles: 7 (2D) or 4 for the
// streaming kernel, 9 or 5 for the reverse sweep's gather kernel.
static size_t role_table_bytes(const bgk_ctx *c)
{
    const int combos = c->dim >= 2 ? 4 : 2;
    const int roles = 1 + 3 * c->dim;
    return (size_t)combos * c->geo.nvz * roles * 2 * c->esize;
}

// The one-residue form needs every lane of a wave on one plane (zr = 1) and
// its role tables to fit in LDS next to the slot entries (and, for the
// streaming kernel, the moment sums).
static bool use_roles(const bgk_ctx *c, int zr, size_t lds, int block)
{
    return zr == 1 && lds + role_table_bytes(c) + stream_acc_bytes(c->geo, c->dim, block) + 4096 <=
                          (size_t)c->lds_max;
}

static bool stream_nt(const bgk_ctx *c)
{
    return 2.0 * (double)c->f_elems * (double)c->esize > 192.0 * (1 << 20);
}

// Pipeline modes of the per-cell kernel (the shape's `unroll`): 1 and 2 jz
// planes per stage with one stage in flight; 3 and 4 one plane per stage
// with 2 and 3 planes in flight.  The deeper modes exist in the one-residue
// form only (elsewhere they run as mode 1).
template <typename real, int DIM, int VEC, int UNR, int PD, bool NTS>
static void stream_kernel_z(bgk_ctx *c, int nb, size_t lds, const void *src, void *dst, hipStream_t s)
{
    const real *p = (const real *)params_buf<real>(c, c->pass_parity);
    const size_t acc = stream_acc_bytes(c->geo, DIM, c->sblock);
    if (use_roles(c, c->zr, lds, c->sblock))  // one plane per wave: role-ordered z-tables after the slots
        hipLaunchKernelGGL((k_stream<real, DIM, VEC, UNR, PD, NTS, true>), dim3(nb), dim3(c->sblock),
                           lds + role_table_bytes(c) + acc, s, make_args(c), (const real *)src, (real *)dst,
                           p, c->partial);
    else
        hipLaunchKernelGGL((k_stream<real, DIM, VEC, UNR, 1, NTS, false>), dim3(nb), dim3(c->sblock), lds + acc, s,
                           make_args(c), (const real *)src, (real *)dst, p, c->partial);
}

template <typename real, int DIM, int VEC, int UNR, int PD>
static void stream_kernel_u(bgk_ctx *c, int nb, size_t lds, const void *src, void *dst, hipStream_t s)
{
    if (stream_nt(c)) stream_kernel_z<real, DIM, VEC, UNR, PD, true>(c, nb, lds, src, dst, s);
    else stream_kernel_z<real, DIM, VEC, UNR, PD, false>(c, nb, lds, src, dst, s);
}

template <typename real, int DIM, int VEC>
static void stream_kernel(bgk_ctx *c, int nb, size_t lds, const void *src, void *dst, hipStream_t s)
{
    if constexpr (DIM == 3) {  // 3D: one or two planes per stage, one stage in flight
        if (c->unroll == 2) stream_kernel_u<real, DIM, VEC, 2, 1>(c, nb, lds, src, dst, s);
        else stream_kernel_u<real, DIM, VEC, 1, 1>(c, nb, lds, src, dst, s);
    } else {
        switch (c->unroll) {
        case 2: stream_kernel_u<real, DIM, VEC, 2, 1>(c, nb, lds, src, dst, s); break;
        case 3: stream_kernel_u<real, DIM, VEC, 1, 2>(c, nb, lds, src, dst, s); break;
        case 4: stream_kernel_u<real, DIM, VEC, 1, 3>(c, nb, lds, src, dst, s); break;
        default: stream_kernel_u<real, DIM, VEC, 1, 1>(c, nb, lds, src, dst, s); break;
        }
    }
}

template <typename real, int DIM>
static void stream_dispatch(bgk_ctx *c, int nb, size_t lds, const void *src, void *dst, hipStream_t s)
{
    if constexpr (DIM == 3) {  // one jx per lane task
        stream_kernel<real, DIM, 1>(c, nb, lds, src, dst, s);
    } else {
        if constexpr (sizeof(real) == 4) {
            if (c->vec == 4) {
                stream_kernel<real, DIM, 4>(c, nb, lds, src, dst, s);
                return;
            }
        }
        if (c->vec == 2) stream_kernel<real, DIM, 2>(c, nb, lds, src, dst, s);
        else stream_kernel<real, DIM, 1>(c, nb, lds, src, dst, s);
    }
}

template <typename real>
static int launch_stream(bgk_ctx *c, const void *src, void *dst, hipStream_t s)
{
    const int items = c->ncells * c->vsplit;
    const int nb = c->persist ? std::min(items, c->persist * c->ncu) : items;
    const int nslot = 1 + 6 * c->dim;
    const size_t lds = (size_t)nslot * c->geo.pe * sizeof(real);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        if (c->ev_used == c->events.size()) {
            hipEvent_t a, b;
            HIP_TRY(c, hipEventCreate(&a));
            HIP_TRY(c, hipEventCreate(&b));
            c->events.push_back({a, b});
        }
        e0 = c->events[c->ev_used].first;
        e1 = c->events[c->ev_used].second;
        c->ev_used++;
        HIP_TRY(c, hipEventRecord(e0, s));
    }
    if (c->shift && c->unroll == 2) {
        const real *p = (const real *)params_buf<real>(c, c->pass_parity);
        const int items = c->row_ntiles * c->geo.nvz;
        const int nbr = c->persist ? std::min(items, c->persist * c->ncu) : items;
        const Args a = make_args(c);
        const size_t l = c->row_lds_bytes;
        // plain stores (measured faster than non-temporal ones here even when
        // the f buffers exceed the last-level cache)
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(nbr), dim3(ROW_THREADS), l, s, a, (const real *)src, (real *)dst, p, c->partial,
                               c->row_tt, c->row_wmax, c->row_lg);
        };
        if (c->row_pcache) go(k_shift_rows<real, 4, true, false>);
        else go(k_shift_rows<real, 4, false, false>);
    } else if (c->shift) {
        const real *p = (const real *)params_buf<real>(c, c->pass_parity);
        // the v_z tables of a cell's 2 Nvx source entries, staged in LDS when they fit in 64 KB
        const size_t st = (size_t)4 * c->geo.nvx * c->geo.nvz * sizeof(real);
        const bool stage = st <= 65536 && (int)st <= c->lds_max / 2;
        const bool nt = stream_nt(c);
        const Args a = make_args(c);
        if (stage && nt)
            hipLaunchKernelGGL((k_shift<real, true, true>), dim3(nb), dim3(c->sblock), st, s, a, (const real *)src,
                               (real *)dst, p, c->partial);
        else if (stage)
            hipLaunchKernelGGL((k_shift<real, false, true>), dim3(nb), dim3(c->sblock), st, s, a, (const real *)src,
                               (real *)dst, p, c->partial);
        else if (nt)
            hipLaunchKernelGGL((k_shift<real, true, false>), dim3(nb), dim3(c->sblock), 0, s, a, (const real *)src,
                               (real *)dst, p, c->partial);
        else
            hipLaunchKernelGGL((k_shift<real, false, false>), dim3(nb), dim3(c->sblock), 0, s, a, (const real *)src,
                               (real *)dst, p, c->partial);
    } else if (c->dim == 3) stream_dispatch<real, 3>(c, nb, lds, src, dst, s);
    else if (c->dim == 2) stream_dispatch<real, 2>(c, nb, lds, src, dst, s);
    else stream_dispatch<real, 1>(c, nb, lds, src, dst, s);
    HIP_TRY(c, hipGetLastError());
    if (c->timing) HIP_TRY(c, hipEventRecord(e1, s));
    return BGK_OK;
}

template <typename real>
static int launch_final(bgk_ctx *c, const void *src, void *dst, int parity, hipStream_t s)
{
    const Args a = pointwise_args(c);
    const int nb = c->ncells * a.vsplit;
    const real *p = (const real *)params_buf<real>(c, parity);
    if (pointwise_vec(c) == 4)
        hipLaunchKernelGGL((k_final<real, 4>), dim3(nb), dim3(pointwise_block(c)), 0, s, a, (const real *)src, (real *)dst, p);
    else if (pointwise_vec(c) == 2)
        hipLaunchKernelGGL((k_final<real, 2>), dim3(nb), dim3(pointwise_block(c)), 0, s, a, (const real *)src, (real *)dst, p);
    else
        hipLaunchKernelGGL((k_final<real, 1>), dim3(nb), dim3(pointwise_block(c)), 0, s, a, (const real *)src, (real *)dst, p);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

#define TRY(x)                   \
    do {                         \
        int rc_ = (x);           \
        if (rc_) return rc_;     \
    } while (0)

// Launch sequence of n >= 1 steps.  Tables alternate between two parity
// buffers: pass k reads buffer (k - 1) % 2 and the preparation after it fills
// buffer k % 2.  Pass k writes X_k = f_out when n - k is even, else the work
// buffer, so the last pass lands in f_out.
template <typename real>
static int one_pass(bgk_ctx *c, int k, int n, const void *src, void *dst, hipStream_t s)
{
    c->pass_parity = (k - 1) % 2;
    TRY(launch_stream<real>(c, src, dst, s));
    return launch_prep<real>(c, k < n ? MODE_MID : MODE_FINAL, c->vsplit, k % 2, s);
}

// Every launch of n >= 1 steps after the rounding counter is set: the
// moments of f_in, the opening tables, n streaming passes each followed by
// the next tables, and the closing relaxation into f_out.
template <typename real>
static int step_launches(bgk_ctx *c, const void *f_in, void *f_out, int n, hipStream_t s)
{
    TRY(launch_moments<real>(c, f_in, s));
    TRY(launch_prep<real>(c, MODE_FIRST, c->vsplit, 0, s));
    auto X = [&](int k) -> void * { return k == 0 ? const_cast<void *>(f_in) : ((n - k) % 2 == 0 ? f_out : c->work); };
    for (int k = 1; k <= n; ++k) TRY(one_pass<real>(c, k, n, X(k - 1), X(k), s));
    return launch_final<real>(c, f_out, f_out, n % 2, s);
}

constexpr size_t MAX_GRAPHS = 4;  // whole-call graphs kept per context (least recently used dropped)

// Capture step_launches for (f_in, f_out, workspace, n) into a graph.
template <typename real>
static int capture_step(bgk_ctx *c, const void *f_in, void *f_out, int n, hipStream_t s, bgk_ctx::Chunk &ch)
{
    ch.f_in = f_in;
    ch.f_out = f_out;
    ch.ws = c->work;
    ch.n = n;
    ch.exec = nullptr;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(c, BGK_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    const int rc = step_launches<real>(c, f_in, f_out, n, s);
    e = hipStreamEndCapture(s, &graph);
    if (rc || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc ? rc : fail(c, BGK_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&ch.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(c, BGK_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return BGK_OK;
}

template <typename real>
static int do_step(bgk_ctx *c, const void *f_in, void *f_out, int n, hipStream_t s)
{
    // rounding counter of pass k (1-based) is seed + k - 1; the tables after
    // each pass advance it on the device.  Set outside any graph: its value
    // changes from call to call.
    hipLaunchKernelGGL(k_set_pass, dim3(1), dim3(64), 0, s, c->pass, c->seed);
    HIP_TRY(c, hipGetLastError());
    c->seed += (uint32_t)n;
    // graphs step aside while kernel timing is on (HIP reports no elapsed
    // time for events recorded by graph nodes) and on the legacy default
    // stream, which cannot be captured
    if (!c->use_graph || c->timing || s == nullptr) return step_launches<real>(c, f_in, f_out, n, s);
    bgk_ctx::Chunk *ch = nullptr;
    for (auto &k : c->chunks)
        if (k.f_in == f_in && k.f_out == f_out && k.ws == c->work && k.n == n) ch = &k;
    if (!ch) {
        if (c->chunks.size() >= MAX_GRAPHS) {
            size_t lru = 0;
            for (size_t i = 1; i < c->chunks.size(); ++i)
                if (c->chunks[i].used < c->chunks[lru].used) lru = i;
            drop_chunk(c->chunks[lru]);
            c->chunks.erase(c->chunks.begin() + (long)lru);
        }
        bgk_ctx::Chunk nc;
        const int rc = capture_step<real>(c, f_in, f_out, n, s, nc);
        if (rc) {
            drop_chunk(nc);
            return rc;
        }
        c->chunks.push_back(std::move(nc));
        ch = &c->chunks.back();
    }
    ch->used = ++c->graph_clock;
    HIP_TRY(c, hipGraphLaunch(ch->exec, s));
    return BGK_OK;
}

// ------------------------------------------------------------- reverse sweep

// Per-cell lid sums of bgk_lid_shear (allocated at its first call).
static int ensure_lid(bgk_ctx *c)
{
    if (!c->lid) HIP_TRY(c, hipMalloc((void **)&c->lid, sizeof(double) * 2 * (size_t)c->ncells));
    return BGK_OK;
}

static int ensure_adjoint(bgk_ctx *c)
{
    if (c->adj_ready) return BGK_OK;
    const size_t nc = (size_t)c->ncells, np = nc * c->vsplit_max;
    HIP_TRY(c, hipMalloc((void **)&c->info_f, sizeof(double) * nc * NINFO));
    HIP_TRY(c, hipMalloc((void **)&c->info_h, sizeof(double) * nc * NINFO));
    HIP_TRY(c, hipMalloc((void **)&c->adj_sums, sizeof(double) * np * NSUM));
    HIP_TRY(c, hipMalloc((void **)&c->adj_wsum, sizeof(double) * np * NWALL));
    HIP_TRY(c, hipMalloc((void **)&c->adj_coef, sizeof(double) * nc * NCOEF));
    HIP_TRY(c, hipMalloc((void **)&c->adj_dw, sizeof(double) * c->ninst * 8));
    HIP_TRY(c, hipMalloc((void **)&c->gk, sizeof(double) * nc));
    HIP_TRY(c, hipMalloc((void **)&c->gt, sizeof(double) * nc));
    TRY(ensure_lid(c));
    std::vector<int> wc;
    for (const Inst &I : c->h_inst) {
        if (I.kind != KIND_CAVITY) continue;
        for (int iy = 0; iy < I.ny; ++iy)
            for (int ix = 0; ix < I.nx; ++ix)
                if (ix == 0 || ix == I.nx - 1 || iy == 0 || iy == I.ny - 1) wc.push_back(I.cell0 + iy * I.nx + ix);
    }
    c->n_wall_cells = (int)wc.size();
    if (!wc.empty()) {
        HIP_TRY(c, hipMalloc((void **)&c->wall_cells, sizeof(int) * wc.size()));
        HIP_TRY(c, hipMemcpy(c->wall_cells, wc.data(), sizeof(int) * wc.size(), hipMemcpyHostToDevice));
    }
    c->adj_ready = true;
    return BGK_OK;
}

static int fill(bgk_ctx *c, double *x, long long n, double v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, v);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

// Coefficients (c->adj_coef) of the transpose of a relaxation at x applied
// to mu, with the per-cell relaxation data in info; adds dL/dKn to c->gk.
template <typename real>
static int relax_coef(bgk_ctx *c, const void *x, const void *mu, const double *info, hipStream_t s)
{
    const int nb = c->ncells * c->vsplit;
    hipLaunchKernelGGL(k_adj_sums<real>, dim3(nb), dim3(fit_block(c->geo.npl)), 0, s, make_args(c), (const real *)x,
                       (const real *)mu, info, c->adj_sums);
    HIP_TRY(c, hipGetLastError());
    hipLaunchKernelGGL(k_adj_coef, dim3((c->ncells + 255) / 256), dim3(256), 0, s, make_args(c), info, c->adj_sums,
                       c->adj_coef, c->gk);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

template <typename real>
static int relax_info(bgk_ctx *c, double *info, int which, hipStream_t s)
{
    hipLaunchKernelGGL(k_relax_info, dim3((c->ncells + 255) / 256), dim3(256), 0, s, make_args(c), c->partial, info,
                       which);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

// The recording form of the step's first streaming pass (h = S(R_a f) with
// the opening tables of parity 0): the plain pass plus one branch byte per
// element into rec.  One jx per lane task and two planes per pipeline stage
// whatever the context's tuned shape; stores as the plain pass's.
template <typename real, int DIM, bool NTS>
static void stream_rec_kernel(bgk_ctx *c, const Args &a, int nb, int block, size_t lds, const void *src, void *dst,
                              hipStream_t s)
{
    const size_t acc = stream_acc_bytes(c->geo, DIM, block);
    const real *p = (const real *)params_buf<real>(c, 0);
    if (use_roles(c, a.zr, lds, block))
        hipLaunchKernelGGL((k_stream<real, DIM, 1, 2, 1, NTS, true, true>), dim3(nb), dim3(block),
                           lds + role_table_bytes(c) + acc, s, a, (const real *)src, (real *)dst, p, c->partial);
    else
        hipLaunchKernelGGL((k_stream<real, DIM, 1, 2, 1, NTS, false, true>), dim3(nb), dim3(block), lds + acc, s, a,
                           (const real *)src, (real *)dst, p, c->partial);
}

template <typename real, int DIM>
static int launch_stream_rec(bgk_ctx *c, const void *src, void *dst, unsigned char *rec, hipStream_t s)
{
    Args a = make_args(c);
    a.rec = rec;
    int block = 256;
    task_shape(c->geo, 1, c->geo.nvz / c->vsplit, &a.zr, &block);
    const int nb = c->ncells * c->vsplit;
    const size_t lds = (size_t)(1 + 6 * DIM) * c->geo.pe * sizeof(real);
    if (stream_nt(c)) stream_rec_kernel<real, DIM, true>(c, a, nb, block, lds, src, dst, s);
    else stream_rec_kernel<real, DIM, false>(c, a, nb, block, lds, src, dst, s);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

template <typename real, int DIM>
static void adj_stream_dispatch(bgk_ctx *c, const unsigned char *rec, const void *lam, hipStream_t s)
{
    const int nb = c->ncells * c->vsplit;
    const size_t lds = (size_t)(2 * DIM) * c->geo.pe * sizeof(real);  // the emitted ghosts' entries
    const real *p0 = params_buf<real>(c, 0);
    const real *lr = (const real *)lam;
    real *o = (real *)c->adj_hb;
    // its own lane-task shape: two jx per lane task for double where the grid allows
    const int vec = (sizeof(real) == 8 && vec_valid(c, 2)) ? 2 : 1;
    Args a = make_args(c);
    int block = 256;
    task_shape(c->geo, vec, c->geo.nvz / c->vsplit, &a.zr, &block);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(nb), dim3(block), lds, s, a, rec, p0, lr, c->adj_coef, o, c->adj_wsum);
    };
    if (a.zr == 1) {
        if (vec == 2) go(k_adj_stream<real, DIM, 2, true>);
        else go(k_adj_stream<real, DIM, 1, true>);
    } else {
        if (vec == 2) go(k_adj_stream<real, DIM, 2, false>);
        else go(k_adj_stream<real, DIM, 1, false>);
    }
}

// abar = S^T(R_b^T lambda^{n+1}): the gather pass with the step's branch
// record and the diffuse-wall returns (R_b^T coefficients in place).
template <typename real>
static int adj_gather_wall(bgk_ctx *c, const unsigned char *br, const void *lam_next, hipStream_t s)
{
    if (c->dim == 1) adj_stream_dispatch<real, 1>(c, br, lam_next, s);
    else adj_stream_dispatch<real, 2>(c, br, lam_next, s);
    HIP_TRY(c, hipGetLastError());
    if (c->n_wall_cells > 0) {
        const real *p0 = params_buf<real>(c, 0);
        hipLaunchKernelGGL(k_adj_wall_flux<real>, dim3(4 * c->ninst), dim3(256), 0, s, make_args(c), p0, c->adj_dw);
        HIP_TRY(c, hipGetLastError());
        hipLaunchKernelGGL(k_adj_wall<real>, dim3(c->n_wall_cells), dim3(256), 0, s, make_args(c), c->wall_cells, p0,
                           c->adj_dw, c->adj_wsum, (real *)c->adj_hb, c->gt);
        HIP_TRY(c, hipGetLastError());
    }
    return BGK_OK;
}

// lambda^n = R_a^T(abar) at f (relaxation data info_f).
template <typename real>
static int adj_close(bgk_ctx *c, const void *f, void *lam_n, hipStream_t s)
{
    if (c->vsplit == 1) {
        // one workgroup per cell: sums, coefficients and lambda^n in one pass
        hipLaunchKernelGGL((k_adj_close<real, false>), dim3(c->ncells), dim3(fit_block(c->geo.npl)), 0, s,
                           make_args(c), (const real *)f, (const real *)c->adj_hb, c->info_f, c->gk, (real *)lam_n,
                           (const real *)nullptr, (const double *)nullptr, (double *)nullptr);
        HIP_TRY(c, hipGetLastError());
    } else {
        TRY(relax_coef<real>(c, f, c->adj_hb, c->info_f, s));
        const int nb = c->ncells * c->vsplit;
        hipLaunchKernelGGL(k_adj_apply<real>, dim3(nb), dim3(fit_block(c->geo.npl)), 0, s, make_args(c),
                           (const real *)c->adj_hb, c->adj_coef, (real *)lam_n);
        HIP_TRY(c, hipGetLastError());
    }
    return BGK_OK;
}

// The reverse step once its forward data are in place -- the relaxation
// data of f and h (info_f, info_h), the opening tables in parity buffer 0,
// h = S(R_a f) and the branch record of that streaming pass:
//   abar = S^T(R_b^T lambda^{n+1})   (k_adj_sums/coef at h, k_adj_stream, k_adj_wall),
//   lambda^n = R_a^T(abar)           (k_adj_close, or k_adj_sums, k_adj_coef, k_adj_apply).
template <typename real>
static int adjoint_tail(bgk_ctx *c, const void *f, const void *h, const unsigned char *br, const void *lam_next,
                        void *lam_n, double *grad, hipStream_t s)
{
    TRY(relax_coef<real>(c, h, lam_next, c->info_h, s));
    TRY(adj_gather_wall<real>(c, br, lam_next, s));
    TRY(adj_close<real>(c, f, lam_n, s));
    hipLaunchKernelGGL(k_grad_reduce, dim3(c->ninst), dim3(256), 0, s, make_args(c), c->gk, c->gt, grad);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

// One reverse step from f^n alone: the step's first streaming pass is
// recomputed in its recording form into the workspace.
template <typename real>
static int do_adjoint(bgk_ctx *c, const void *f, const void *lam_next, void *lam_n, double *grad, hipStream_t s)
{
    TRY(ensure_adjoint(c));
    TRY(fill(c, c->gk, c->ncells, 0.0, s));
    TRY(fill(c, c->gt, c->ncells, 0.0, s));
    TRY(launch_moments<real>(c, f, s));
    TRY(relax_info<real>(c, c->info_f, 0, s));
    TRY(launch_prep<real>(c, MODE_FIRST, c->vsplit, 0, s));
    c->pass_parity = 0;
    unsigned char *br = (unsigned char *)c->adj_rec;
    if (c->dim == 1) TRY((launch_stream_rec<real, 1>(c, f, c->adj_h, br, s)));
    else TRY((launch_stream_rec<real, 2>(c, f, c->adj_h, br, s)));
    TRY(relax_info<real>(c, c->info_h, 1, s));
    return adjoint_tail<real>(c, f, c->adj_h, br, lam_next, lam_n, grad, s);
}

// Step record (bgk_step_record): h = S(R_a f_n) as the step stored it, the
// per-cell totals of the moment sums of f_n and of h, and the branch record
// of the streaming pass; each part 256-byte aligned.
struct RecordLayout {
    size_t h, tot_f, tot_h, br, bytes;
};

static RecordLayout record_layout(const bgk_ctx *c)
{
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    RecordLayout r;
    r.h = 0;
    r.tot_f = up(c->f_elems * c->esize);
    r.tot_h = r.tot_f + up(sizeof(double) * (size_t)c->ncells * NQ);
    r.br = r.tot_h + up(sizeof(double) * (size_t)c->ncells * NQ);
    r.bytes = r.br + up(c->f_elems);
    return r;
}

static int part_totals(bgk_ctx *c, double *tot, hipStream_t s)
{
    const long long n = (long long)c->ncells * NQ;
    hipLaunchKernelGGL(k_part_totals, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, make_args(c), c->partial, tot);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

static int part_restore(bgk_ctx *c, const double *tot, hipStream_t s)
{
    const long long n = (long long)c->ncells * c->vsplit * NQ;
    hipLaunchKernelGGL(k_part_restore, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, make_args(c), tot,
                       c->partial);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

// One step that keeps its record: the launch sequence of a one-step
// bgk_step with the streaming pass in its recording form writing h into the
// record, and the closing relaxation reading it from there.
template <typename real>
static int do_step_record(bgk_ctx *c, const void *f_in, void *f_out, char *rec, hipStream_t s)
{
    const RecordLayout L = record_layout(c);
    hipLaunchKernelGGL(k_set_pass, dim3(1), dim3(64), 0, s, c->pass, c->seed);
    HIP_TRY(c, hipGetLastError());
    c->seed += 1u;
    TRY(launch_moments<real>(c, f_in, s));
    TRY(launch_prep<real>(c, MODE_FIRST, c->vsplit, 0, s));
    TRY(part_totals(c, (double *)(rec + L.tot_f), s));
    c->pass_parity = 0;
    unsigned char *br = (unsigned char *)(rec + L.br);
    if (c->dim == 1) TRY((launch_stream_rec<real, 1>(c, f_in, rec + L.h, br, s)));
    else TRY((launch_stream_rec<real, 2>(c, f_in, rec + L.h, br, s)));
    TRY(part_totals(c, (double *)(rec + L.tot_h), s));
    TRY(launch_prep<real>(c, MODE_FINAL, c->vsplit, 1, s));
    return launch_final<real>(c, rec + L.h, f_out, 1, s);
}

// One reverse step from f^n and its step record: nothing is recomputed.
template <typename real>
static int do_adjoint_record(bgk_ctx *c, const void *f, const char *rec, const void *lam_next, void *lam_n,
                             double *grad, hipStream_t s)
{
    const RecordLayout L = record_layout(c);
    TRY(ensure_adjoint(c));
    TRY(fill(c, c->gk, c->ncells, 0.0, s));
    TRY(fill(c, c->gt, c->ncells, 0.0, s));
    TRY(part_restore(c, (const double *)(rec + L.tot_f), s));
    TRY(relax_info<real>(c, c->info_f, 0, s));
    TRY(launch_prep<real>(c, MODE_FIRST, c->vsplit, 0, s));
    TRY(part_restore(c, (const double *)(rec + L.tot_h), s));
    TRY(relax_info<real>(c, c->info_h, 1, s));
    return adjoint_tail<real>(c, f, rec + L.h, (const unsigned char *)(rec + L.br), lam_next, lam_n, grad, s);
}

// A reverse sweep over n recorded steps: lambda^0 from lambda^n with the
// states f[i] and records rec[i] of steps i = 0 .. n-1, one step after the
// other from the last.  With one chunk per cell the close pass of step i also
// forms step i-1's sums at h (k_adj_close<real, true>), so only the last step
// runs a separate sums pass; the parameter gradients are reduced once.
// lambda^i lands in lam_0 for even i and in lam_tmp for odd i.
template <typename real>
static int do_adjoint_sweep(bgk_ctx *c, int n, const void *const *f, const void *const *rec, const void *lam_N,
                            void *lam_0, double *grad, void *lam_tmp, hipStream_t s)
{
    const RecordLayout L = record_layout(c);
    TRY(ensure_adjoint(c));
    TRY(fill(c, c->gk, c->ncells, 0.0, s));
    TRY(fill(c, c->gt, c->ncells, 0.0, s));
    const bool fuse = c->vsplit == 1;
    auto R = [&](int i) { return (const char *)rec[i]; };
    auto lam_out = [&](int i) -> void * { return i % 2 == 0 ? lam_0 : lam_tmp; };
    auto lam_in = [&](int i) -> const void * { return i + 1 == n ? lam_N : (const void *)lam_out(i + 1); };
    for (int i = n - 1; i >= 0; --i) {
        // step i's opening relaxation data and tables
        TRY(part_restore(c, (const double *)(R(i) + L.tot_f), s));
        TRY(relax_info<real>(c, c->info_f, 0, s));
        TRY(launch_prep<real>(c, MODE_FIRST, c->vsplit, 0, s));
        if (i == n - 1 || !fuse) {
            // R_b^T coefficients of step i from its own sums at h
            TRY(part_restore(c, (const double *)(R(i) + L.tot_h), s));
            TRY(relax_info<real>(c, c->info_h, 1, s));
            TRY(relax_coef<real>(c, R(i) + L.h, lam_in(i), c->info_h, s));
        }
        TRY(adj_gather_wall<real>(c, (const unsigned char *)(R(i) + L.br), lam_in(i), s));
        if (fuse && i > 0) {
            // lambda^i, and with it step i-1's sums at h and its R_b^T coefficients
            TRY(part_restore(c, (const double *)(R(i - 1) + L.tot_h), s));
            TRY(relax_info<real>(c, c->info_h, 1, s));
            hipLaunchKernelGGL((k_adj_close<real, true>), dim3(c->ncells), dim3(fit_block(c->geo.npl)), 0, s,
                               make_args(c), (const real *)f[i], (const real *)c->adj_hb, c->info_f, c->gk,
                               (real *)lam_out(i), (const real *)(R(i - 1) + L.h), (const double *)c->info_h,
                               c->adj_sums);
            HIP_TRY(c, hipGetLastError());
            hipLaunchKernelGGL(k_adj_coef, dim3((c->ncells + 255) / 256), dim3(256), 0, s, make_args(c), c->info_h,
                               c->adj_sums, c->adj_coef, c->gk);
            HIP_TRY(c, hipGetLastError());
        } else {
            TRY(adj_close<real>(c, f[i], lam_out(i), s));
        }
    }
    hipLaunchKernelGGL(k_grad_reduce, dim3(c->ninst), dim3(256), 0, s, make_args(c), c->gk, c->gt, grad);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

// Does [a, a + na) overlap [b, b + nb)?
static bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

// Contexts with a reverse sweep: one- and two-dimensional kinds of one
// dimension, the per-cell streaming, the point-value Maxwellian, the full
// velocity space.
static int adjoint_kinds(bgk_ctx *ctx, const char *who)
{
    const std::string w(who);
    if (ctx->dim == 3) return fail(ctx, BGK_E_UNSUPPORTED, w + ": one- and two-dimensional kinds only");
    if (ctx->mixed) return fail(ctx, BGK_E_UNSUPPORTED, w + ": instances of one dimension only");
    if (ctx->shift) return fail(ctx, BGK_E_UNSUPPORTED, w + ": no reverse sweep of shift streaming");
    if (ctx->conservative)
        return fail(ctx, BGK_E_UNSUPPORTED, w + ": no reverse sweep of the effective Maxwellian parameters");
    if (ctx->geo.red) return fail(ctx, BGK_E_UNSUPPORTED, w + ": no reverse sweep in the reduced velocity space");
    return BGK_OK;
}

extern "C" int bgk_record_bytes(const bgk_ctx *ctx, size_t *bytes)
{
    if (!ctx || !bytes) return BGK_E_INVALID;
    *bytes = record_layout(ctx).bytes;
    return BGK_OK;
}

extern "C" int bgk_step_record(bgk_ctx *ctx, const void *f_in, void *f_out, void *rec, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (!f_in || !f_out || !rec) return fail(ctx, BGK_E_INVALID, "bgk_step_record: NULL buffer");
    const size_t fb = ctx->f_elems * ctx->esize, rb = record_layout(ctx).bytes;
    if (overlaps(f_in, fb, f_out, fb)) return fail(ctx, BGK_E_ALIAS, "bgk_step_record: f_in and f_out must not overlap");
    if (overlaps(rec, rb, f_in, fb) || overlaps(rec, rb, f_out, fb))
        return fail(ctx, BGK_E_ALIAS, "bgk_step_record: the record must not overlap f_in or f_out");
    TRY(adjoint_kinds(ctx, "bgk_step_record"));
    hipStream_t s = (hipStream_t)stream;
    return ctx->precision == BGK_FP64 ? do_step_record<double>(ctx, f_in, f_out, (char *)rec, s)
                                      : do_step_record<float>(ctx, f_in, f_out, (char *)rec, s);
}

extern "C" int bgk_step_adjoint_record(bgk_ctx *ctx, const void *f_n, const void *rec, const void *lam_next,
                                       void *lam_n, double *grad_params, void *ws, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (!f_n || !rec || !lam_next || !lam_n || !grad_params || !ws)
        return fail(ctx, BGK_E_INVALID, "bgk_step_adjoint_record: NULL buffer");
    const size_t fb = ctx->f_elems * ctx->esize, rb = record_layout(ctx).bytes;
    if (overlaps(lam_n, fb, f_n, fb) || overlaps(lam_n, fb, lam_next, fb) || overlaps(lam_n, fb, rec, rb))
        return fail(ctx, BGK_E_ALIAS, "bgk_step_adjoint_record: lam_n must not overlap f_n, rec or lam_next");
    for (const void *q : {f_n, lam_next, (const void *)lam_n})
        if (overlaps(ws, fb, q, fb))
            return fail(ctx, BGK_E_ALIAS, "bgk_step_adjoint_record: the workspace must not overlap f_n, lam_next or lam_n");
    if (overlaps(ws, fb, rec, rb))
        return fail(ctx, BGK_E_ALIAS, "bgk_step_adjoint_record: the workspace must not overlap the record");
    TRY(adjoint_kinds(ctx, "bgk_step_adjoint_record"));
    hipStream_t s = (hipStream_t)stream;
    ctx->adj_hb = ws;
    const int rc = ctx->precision == BGK_FP64
                       ? do_adjoint_record<double>(ctx, f_n, (const char *)rec, lam_next, lam_n, grad_params, s)
                       : do_adjoint_record<float>(ctx, f_n, (const char *)rec, lam_next, lam_n, grad_params, s);
    ctx->adj_hb = nullptr;
    return rc;
}

extern "C" int bgk_adjoint_sweep_record(bgk_ctx *ctx, int n, const void *const *f, const void *const *rec,
                                        const void *lam_N, void *lam_0, double *grad_params, void *ws, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (n < 0) return fail(ctx, BGK_E_INVALID, "bgk_adjoint_sweep_record: n < 0");
    if ((n > 0 && (!f || !rec)) || !lam_N || !lam_0 || !grad_params || !ws)
        return fail(ctx, BGK_E_INVALID, "bgk_adjoint_sweep_record: NULL buffer");
    const size_t fb = ctx->f_elems * ctx->esize, rb = record_layout(ctx).bytes;
    if (overlaps(lam_0, fb, lam_N, fb) || overlaps(ws, 2 * fb, lam_N, fb) || overlaps(ws, 2 * fb, lam_0, fb))
        return fail(ctx, BGK_E_ALIAS, "bgk_adjoint_sweep_record: lam_0, lam_N and the workspace must not overlap");
    for (int i = 0; i < n; ++i) {
        if (!f[i] || !rec[i]) return fail(ctx, BGK_E_INVALID, "bgk_adjoint_sweep_record: NULL state or record");
        if (overlaps(lam_0, fb, f[i], fb) || overlaps(lam_0, fb, rec[i], rb) || overlaps(ws, 2 * fb, f[i], fb) ||
            overlaps(ws, 2 * fb, rec[i], rb))
            return fail(ctx, BGK_E_ALIAS, "bgk_adjoint_sweep_record: lam_0 and the workspace must not overlap a "
                                          "state or record");
    }
    TRY(adjoint_kinds(ctx, "bgk_adjoint_sweep_record"));
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        HIP_TRY(ctx, hipMemcpyAsync(lam_0, lam_N, fb, hipMemcpyDeviceToDevice, s));
        return BGK_OK;
    }
    ctx->adj_hb = ws;
    void *tmp = (char *)ws + fb;
    const int rc = ctx->precision == BGK_FP64
                       ? do_adjoint_sweep<double>(ctx, n, f, rec, lam_N, lam_0, grad_params, tmp, s)
                       : do_adjoint_sweep<float>(ctx, n, f, rec, lam_N, lam_0, grad_params, tmp, s);
    ctx->adj_hb = nullptr;
    return rc;
}

extern "C" int bgk_step_adjoint(bgk_ctx *ctx, const void *f_n, const void *lam_next, void *lam_n, double *grad_params,
                                void *ws, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (!f_n || !lam_next || !lam_n || !grad_params || !ws)
        return fail(ctx, BGK_E_INVALID, "bgk_step_adjoint: NULL buffer");
    if (lam_n == f_n || lam_n == lam_next) return fail(ctx, BGK_E_ALIAS, "bgk_step_adjoint: lam_n must not alias inputs");
    const size_t fb = ctx->f_elems * ctx->esize;
    for (const void *q : {f_n, lam_next, (const void *)lam_n})
        if (overlaps(ws, adjoint_ws_bytes(ctx), q, fb))
            return fail(ctx, BGK_E_ALIAS, "bgk_step_adjoint: the workspace must not overlap f_n, lam_next or lam_n");
    TRY(adjoint_kinds(ctx, "bgk_step_adjoint"));
    hipStream_t s = (hipStream_t)stream;
    ctx->adj_h = ws;
    ctx->adj_hb = (char *)ws + fb;
    ctx->adj_rec = (char *)ws + 2 * fb;
    const int rc = ctx->precision == BGK_FP64 ? do_adjoint<double>(ctx, f_n, lam_next, lam_n, grad_params, s)
                                              : do_adjoint<float>(ctx, f_n, lam_next, lam_n, grad_params, s);
    ctx->adj_h = ctx->adj_hb = ctx->adj_rec = nullptr;
    return rc;
}

template <typename real>
static int lid(bgk_ctx *c, const void *f, double *L, void *lam, double *grad, hipStream_t s)
{
    TRY(ensure_lid(c));
    hipLaunchKernelGGL(k_lid_sums<real>, dim3(c->ncells), dim3(256), 0, s, make_args(c), (const real *)f, c->lid);
    HIP_TRY(c, hipGetLastError());
    hipLaunchKernelGGL(k_lid_finish, dim3(c->ninst), dim3(64), 0, s, make_args(c), c->lid, L, grad);
    HIP_TRY(c, hipGetLastError());
    if (lam) {
        hipLaunchKernelGGL(k_lid_seed<real>, dim3(c->ncells), dim3(256), 0, s, make_args(c), (real *)lam);
        HIP_TRY(c, hipGetLastError());
    }
    return BGK_OK;
}

extern "C" int bgk_lid_shear(bgk_ctx *ctx, const void *f, double *L, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (!f || !L) return fail(ctx, BGK_E_INVALID, "bgk_lid_shear: NULL buffer");
    if (ctx->dim == 3) return fail(ctx, BGK_E_UNSUPPORTED, "bgk_lid_shear: two-dimensional cavities only");
    hipStream_t s = (hipStream_t)stream;
    return ctx->precision == BGK_FP64 ? lid<double>(ctx, f, L, nullptr, nullptr, s)
                                      : lid<float>(ctx, f, L, nullptr, nullptr, s);
}

extern "C" int bgk_lid_shear_grad(bgk_ctx *ctx, const void *f, void *lam, double *grad_params, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (!f || !lam || !grad_params) return fail(ctx, BGK_E_INVALID, "bgk_lid_shear_grad: NULL buffer");
    if (lam == f) return fail(ctx, BGK_E_ALIAS, "bgk_lid_shear_grad: lam must not alias f");
    if (ctx->geo.red) return fail(ctx, BGK_E_UNSUPPORTED, "bgk_lid_shear_grad: not in the reduced velocity space");
    if (ctx->dim == 3) return fail(ctx, BGK_E_UNSUPPORTED, "bgk_lid_shear_grad: two-dimensional cavities only");
    hipStream_t s = (hipStream_t)stream;
    return ctx->precision == BGK_FP64 ? lid<double>(ctx, f, nullptr, lam, grad_params, s)
                                      : lid<float>(ctx, f, nullptr, lam, grad_params, s);
}

// Steady-cavity metrics (Table of Sec. 5.2), computed on the host from the
// lid shear and the moments of the centre line.
//   D = -L / (p0 U_W W): mean lid shear stress in units of p0 U_W, with
//       p0 = 1/2 (n = T = 1) and W the lid width;
//   G = 1 / H * int u dy, u = V_x / U_W on the line x = (x0 + x1) / 2 (the
//       middle column, or the mean of the two middle columns), from the
//       first zero of u below the lid (the main vortex's centre; linear
//       between cell centres) to the lid (u extrapolated linearly over the
//       top half cell); from the bottom wall when u has no zero.
static void centre_line_metrics(const Inst &I, const bgk_problem &p, const double *mom, double L, double *out)
{
    const int nx = I.nx, ny = I.ny;
    const double uw = I.uw, W = p.x1 - p.x0, H = p.y1 - p.y0, h = H / ny;
    out[0] = -L / (0.5 * uw * W);
    std::vector<double> u(ny);
    for (int iy = 0; iy < ny; ++iy) {
        const double *row = mom + 5 * (size_t)iy * nx;
        const double vx = (nx & 1) ? row[5 * (nx / 2) + 1] : 0.5 * (row[5 * (nx / 2 - 1) + 1] + row[5 * (nx / 2) + 1]);
        u[iy] = vx / uw;
    }
    // lowest row of the run of positive u that reaches the lid
    int lo = ny - 1;
    while (lo > 0 && u[lo - 1] > 0.0) --lo;
    double area = 0.0;
    if (lo == 0) {
        const double ub = ny > 1 ? 1.5 * u[0] - 0.5 * u[1] : u[0];
        area += 0.25 * h * (ub + u[0]);
    } else if (u[lo] > 0.0) {
        area += 0.5 * h * u[lo] * u[lo] / (u[lo] - u[lo - 1]);
    }
    for (int iy = lo; iy + 1 < ny; ++iy) area += 0.5 * h * (u[iy] + u[iy + 1]);
    const double ut = ny > 1 ? 1.5 * u[ny - 1] - 0.5 * u[ny - 2] : u[ny - 1];
    area += 0.25 * h * (u[ny - 1] + ut);
    out[1] = area / H;
}

extern "C" int bgk_cavity_metrics(bgk_ctx *ctx, const void *f, double *out, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (!f || !out) return fail(ctx, BGK_E_INVALID, "bgk_cavity_metrics: NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    if (!ctx->lid_L) HIP_TRY(ctx, hipMalloc((void **)&ctx->lid_L, sizeof(double) * ctx->ninst));
    TRY(ctx->precision == BGK_FP64 ? lid<double>(ctx, f, ctx->lid_L, nullptr, nullptr, s)
                                   : lid<float>(ctx, f, ctx->lid_L, nullptr, nullptr, s));
    TRY(bgk_moments(ctx, f, ctx->mom, stream));
    std::vector<double> L(ctx->ninst), mom((size_t)ctx->ncells * 5);
    HIP_TRY(ctx, hipMemcpyAsync(L.data(), ctx->lid_L, sizeof(double) * L.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(mom.data(), ctx->mom, sizeof(double) * mom.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    for (int i = 0; i < ctx->ninst; ++i) {
        const Inst &I = ctx->h_inst[i];
        if (I.kind != KIND_CAVITY || !(I.uw != 0.0)) {
            out[2 * i] = out[2 * i + 1] = std::nan("");
            continue;
        }
        centre_line_metrics(I, ctx->probs[i], mom.data() + 5 * (size_t)I.cell0, L[i], out + 2 * i);
    }
    return BGK_OK;
}

// ------------------------------------------------------------- autotuning

// Time of one step in the steady part of bgk_step: ((2 + n) steps - 2 steps)
// / n, so the once-per-call passes (moments of the input, closing relaxation)
// cancel, after `warm` untimed steps; f -> tmp, with graph replay, timing and
// the rounding seed saved and restored.
template <typename real>
static int time_steps(bgk_ctx *c, const void *f, void *tmp, hipStream_t s, double *us, int n = 8, int warm = 0)
{
    hipEvent_t e[3];
    for (auto &x : e) HIP_TRY(c, hipEventCreate(&x));
    const bool timing = c->timing, graph = c->use_graph;
    const uint32_t seed = c->seed;
    c->timing = false;
    c->use_graph = false;
    // untimed first: a shape's first launch loads its code object
    int rc = do_step<real>(c, f, tmp, 1, s);
    if (!rc && warm > 0) rc = do_step<real>(c, f, tmp, warm, s);
    if (!rc) rc = hipEventRecord(e[0], s) == hipSuccess ? 0 : BGK_E_HIP;
    if (!rc) rc = do_step<real>(c, f, tmp, 2, s);
    if (!rc) rc = hipEventRecord(e[1], s) == hipSuccess ? 0 : BGK_E_HIP;
    if (!rc) rc = do_step<real>(c, f, tmp, 2 + n, s);
    if (!rc) rc = hipEventRecord(e[2], s) == hipSuccess ? 0 : BGK_E_HIP;
    float a = 0.0f, b = 0.0f;
    if (!rc) rc = hipEventSynchronize(e[2]) == hipSuccess ? 0 : BGK_E_HIP;
    if (!rc) rc = hipEventElapsedTime(&a, e[0], e[1]) == hipSuccess ? 0 : BGK_E_HIP;
    if (!rc) rc = hipEventElapsedTime(&b, e[1], e[2]) == hipSuccess ? 0 : BGK_E_HIP;
    c->timing = timing;
    c->use_graph = graph;
    c->seed = seed;
    for (auto &x : e) (void)hipEventDestroy(x);
    if (rc) return fail(c, rc, "autotune: timing failed");
    *us = 1e3 * (double)(b - a) / (double)n;
    return BGK_OK;
}

// Try the candidate shapes on f and keep the fastest by the steady step time
// of real steps (f -> tmp, the caller's scratch state; the ping-pong buffer
// is the caller's workspace, already in c->work).  The sweep times 8 steps
// per shape; such short runs vary by up to ~10% (the clock state of a short
// burst differs from a sustained run), so the four fastest are timed twice
// more over 32 steps after 16 untimed ones and ranked by the better of those
// two timings alone.
template <typename real>
static int autotune(bgk_ctx *c, const void *f, void *tmp, hipStream_t s)
{
    TRY(launch_moments<real>(c, f, s));
    TRY(launch_prep<real>(c, MODE_FIRST, c->vsplit, 0, s));
    struct Cand { double us; int vec, unroll, vsplit, persist; };
    const Cand start{0.0, c->vec, c->unroll, c->vsplit, c->persist};
    std::vector<Cand> cands;
    std::vector<int> splits;
    for (int t : {256, 512, 1024, 2048, 4096, 8192}) {
        const int v = std::min(vsplit_for(c, t), c->vsplit_max);
        if (std::find(splits.begin(), splits.end(), v) == splits.end()) splits.push_back(v);
    }
    for (int v : {2, 4})
        if (v <= c->vsplit_max && std::find(splits.begin(), splits.end(), v) == splits.end()) splits.push_back(v);
    auto measure = [&](const Cand &k, double *us, int n, int warm) {
        set_shape(c, k.vec, k.unroll, k.vsplit, k.persist);
        return time_steps<real>(c, f, tmp, s, us, n, warm);
    };
    int rc = BGK_OK;
    {
        // untimed warm-up: the first shapes of a cold device otherwise time slow
        double us = 0.0;
        for (int r = 0; r < 3 && !rc; ++r) rc = time_steps<real>(c, f, tmp, s, &us);
    }
    for (int vec : {4, 2, 1}) {
        if (!vec_valid(c, vec)) continue;
        for (int unroll : {1, 2, 3, 4})
            for (int vs : splits)
                for (int ps : {0, 2, 4}) {
                    if (rc) break;
                    if (c->shift && unroll > (c->row_ok ? 2 : 1)) continue;  // per-cell or row tiles
                    if (c->dim == 3 && unroll > 2) continue;  // 3D: modes 1 and 2 only
                    if (ps && c->ncells * vs <= ps * c->ncu) continue;  // grid already resident
                    Cand k{0.0, vec, unroll, vs, ps};
                    rc = measure(k, &k.us, 8, 0);
                    if (!rc) cands.push_back(k);
                }
    }
    std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.us < b.us; });
    if (cands.size() > 4) cands.resize(4);
    for (Cand &k : cands) k.us = HUGE_VAL;
    for (int rep = 0; rep < 2 && !rc; ++rep)
        for (Cand &k : cands) {
            double us = 0.0;
            if (!rc) rc = measure(k, &us, 32, 16);
            if (!rc) k.us = std::min(k.us, us);
        }
    (void)hipStreamSynchronize(s);
    if (rc || cands.empty()) {
        set_shape(c, start.vec, start.unroll, start.vsplit, start.persist);
        return rc ? rc : fail(c, BGK_E_INVALID, "autotune: no valid shape");
    }
    const Cand *best = &cands[0];
    for (const Cand &k : cands)
        if (k.us < best->us) best = &k;
    set_shape(c, best->vec, best->unroll, best->vsplit, best->persist);
    c->tuned_us = best->us;
    return BGK_OK;
}

extern "C" int bgk_autotune(bgk_ctx *ctx, const void *f, void *scratch, void *ws, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (!f || !scratch || !ws) return fail(ctx, BGK_E_INVALID, "bgk_autotune: NULL buffer");
    const size_t fb = ctx->f_elems * ctx->esize;
    if (overlaps(scratch, fb, f, fb) || overlaps(ws, fb, f, fb) || overlaps(ws, fb, scratch, fb))
        return fail(ctx, BGK_E_ALIAS, "bgk_autotune: f, scratch and the workspace must not overlap");
    hipStream_t s = (hipStream_t)stream;
    ctx->work = ws;
    const int rc = ctx->precision == BGK_FP64 ? autotune<double>(ctx, f, scratch, s)
                                              : autotune<float>(ctx, f, scratch, s);
    ctx->work = nullptr;
    return rc;
}

extern "C" int bgk_get_launch(const bgk_ctx *ctx, int *vec, int *unroll, int *vsplit, int *persist, double *tuned_us)
{
    if (!ctx) return BGK_E_INVALID;
    if (vec) *vec = ctx->vec;
    if (unroll) *unroll = ctx->unroll;
    if (vsplit) *vsplit = ctx->vsplit;
    if (persist) *persist = ctx->persist;
    if (tuned_us) *tuned_us = ctx->tuned_us;
    return BGK_OK;
}

extern "C" int bgk_set_launch(bgk_ctx *ctx, int vec, int unroll, int vsplit, int persist)
{
    if (!ctx) return BGK_E_INVALID;
    if (!(vec == 1 || vec == 2 || vec == 4) || !vec_valid(ctx, vec) || unroll < 1 || unroll > 4 ||
        (ctx->shift && unroll > (ctx->row_ok ? 2 : 1)) || (ctx->dim == 3 && unroll > 2) || vsplit < 1 || vsplit > ctx->vsplit_max ||
        persist < 0 || persist > 64)
        return fail(ctx, BGK_E_INVALID, "bgk_set_launch: shape not valid for this context");
    set_shape(ctx, vec, unroll, vsplit, persist);
    return BGK_OK;
}

extern "C" int bgk_step(bgk_ctx *ctx, const void *f_in, void *f_out, int n_steps, void *ws, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (!f_in || !f_out) return fail(ctx, BGK_E_INVALID, "bgk_step: NULL buffer");
    if (n_steps < 0) return fail(ctx, BGK_E_INVALID, "bgk_step: n_steps < 0");
    const size_t fb = ctx->f_elems * ctx->esize;
    if (overlaps(f_in, fb, f_out, fb)) return fail(ctx, BGK_E_ALIAS, "bgk_step: f_in and f_out must not overlap");
    if (n_steps >= 2 && !ws) return fail(ctx, BGK_E_INVALID, "bgk_step: n_steps >= 2 needs the workspace");
    if (n_steps >= 2 && (overlaps(ws, fb, f_in, fb) || overlaps(ws, fb, f_out, fb)))
        return fail(ctx, BGK_E_ALIAS, "bgk_step: the workspace must not overlap f_in or f_out");
    hipStream_t s = (hipStream_t)stream;
    if (n_steps == 0) {
        HIP_TRY(ctx, hipMemcpyAsync(f_out, f_in, fb, hipMemcpyDeviceToDevice, s));
        return BGK_OK;
    }
    ctx->work = n_steps >= 2 ? ws : nullptr;
    const int rc = ctx->precision == BGK_FP64 ? do_step<double>(ctx, f_in, f_out, n_steps, s)
                                              : do_step<float>(ctx, f_in, f_out, n_steps, s);
    ctx->work = nullptr;
    return rc;
}

extern "C" int bgk_moments(bgk_ctx *ctx, const void *f, double *mom, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (!f || !mom) return fail(ctx, BGK_E_INVALID, "bgk_moments: NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    TRY(ctx->precision == BGK_FP64 ? launch_moments<double>(ctx, f, s) : launch_moments<float>(ctx, f, s));
    hipLaunchKernelGGL(k_macro, dim3((ctx->ncells + 255) / 256), dim3(256), 0, s, make_args(ctx), ctx->partial, mom);
    HIP_TRY(ctx, hipGetLastError());
    return BGK_OK;
}

extern "C" int bgk_initial_state(bgk_ctx *ctx, void *f, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (!f) return fail(ctx, BGK_E_INVALID, "bgk_initial_state: NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    const Args a = pointwise_args(ctx);
    const int nb = ctx->ncells * a.vsplit;
    if (ctx->precision == BGK_FP64)
        hipLaunchKernelGGL(k_init<double>, dim3(nb), dim3(fit_block(ctx->geo.npl)), 0, s, a, (double *)f);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(nb), dim3(fit_block(ctx->geo.npl)), 0, s, a, (float *)f);
    HIP_TRY(ctx, hipGetLastError());
    return BGK_OK;
}

extern "C" int bgk_check(bgk_ctx *ctx, const void *f, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    TRY(bgk_moments(ctx, f, ctx->mom, stream));
    HIP_TRY(ctx, hipMemsetAsync(ctx->flags, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_check, dim3((ctx->ncells + 255) / 256), dim3(256), 0, s, ctx->ncells, ctx->mom, ctx->flags);
    HIP_TRY(ctx, hipGetLastError());
    int flags = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&flags, ctx->flags, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (flags & 1) return fail(ctx, BGK_E_NONFINITE, "bgk_check: non-finite moment");
    if (flags & 2) return fail(ctx, BGK_E_NEGATIVE, "bgk_check: density or temperature <= 0");
    return BGK_OK;
}

extern "C" int bgk_set_rounding_seed(bgk_ctx *ctx, unsigned int seed)
{
    if (!ctx) return BGK_E_INVALID;
    ctx->seed = seed;
    return BGK_OK;
}

extern "C" int bgk_get_rounding_seed(const bgk_ctx *ctx, unsigned int *seed)
{
    if (!ctx || !seed) return BGK_E_INVALID;
    *seed = ctx->seed;
    return BGK_OK;
}

extern "C" int bgk_set_graph(bgk_ctx *ctx, int on)
{
    if (!ctx) return BGK_E_INVALID;
    ctx->use_graph = on != 0;
    if (!ctx->use_graph) drop_graphs(ctx);
    return BGK_OK;
}

extern "C" int bgk_set_timing(bgk_ctx *ctx, int capacity)
{
    if (!ctx || capacity < 0) return BGK_E_INVALID;
    ctx->timing = capacity > 0;
    ctx->ev_used = 0;
    while (ctx->events.size() < (size_t)capacity) {
        hipEvent_t a, b;
        HIP_TRY(ctx, hipEventCreate(&a));
        HIP_TRY(ctx, hipEventCreate(&b));
        ctx->events.push_back({a, b});
    }
    return BGK_OK;
}

extern "C" int bgk_timing(bgk_ctx *ctx, double *ms, int *launches)
{
    if (!ctx) return BGK_E_INVALID;
    double tot = 0.0;
    int count = 0;
    auto add = [&](const std::pair<hipEvent_t, hipEvent_t> &e) -> int {
        HIP_TRY(ctx, hipEventSynchronize(e.second));
        float t = 0.0f;
        HIP_TRY(ctx, hipEventElapsedTime(&t, e.first, e.second));
        tot += t;
        count++;
        return BGK_OK;
    };
    for (size_t i = 0; i < ctx->ev_used; ++i) TRY(add(ctx->events[i]));
    if (ms) *ms = tot;
    if (launches) *launches = count;
    ctx->ev_used = 0;
    return BGK_OK;
}

// ------------------------------------------------------------- allocation-free step
// bgk_step_noalloc: the step of bgk_step for callers that cannot allocate
// device memory.  The per-call device data a context would own (instance
// tables, the Maxwellian table entries of both parities, the moment partial
// sums, the rounding counter) is carved from one static device array of
// NOALLOC_SCRATCH_BYTES; each device holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel: its device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)BGK_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::vector<void *> g_scratch_ptr;  // device address of `scratch`, per device

static int scratch_address(int dev, void **out, std::string &msg)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return BGK_E_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BGK_OK;
}

// Host data reaches the device through kernel arguments (copied when the
// launch is enqueued), so no staging buffer has to outlive the call.
constexpr int UPLOAD_CHUNK = 2048;
struct UploadChunk { unsigned char b[UPLOAD_CHUNK]; };

__global__ void k_upload(UploadChunk c, int n, unsigned char *__restrict__ dst)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = c.b[i];
}

static int upload(const void *src, size_t n, void *dst, hipStream_t s, std::string &msg)
{
    const unsigned char *p = (const unsigned char *)src;
    for (size_t o = 0; o < n; o += UPLOAD_CHUNK) {
        UploadChunk c;
        const int k = (int)std::min<size_t>(UPLOAD_CHUNK, n - o);
        memcpy(c.b, p + o, (size_t)k);
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, c, k, (unsigned char *)dst + o);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            msg = std::string("k_upload: ") + hipGetErrorString(e);
            return BGK_E_HIP;
        }
    }
    return BGK_OK;
}

extern "C" int bgk_step_noalloc(const bgk_problem *probs, int n_probs, int precision, const void *f_in, void *f_out,
                                int n_steps, void *ws, void *stream)
{
    bgk_ctx c;  // host-side plan; its device pointers are carved from the scratch array
    std::string msg;
    int rc = plan_ctx(probs, n_probs, precision, &c, msg);
    if (rc) return fail(nullptr, rc, msg);
    // layout of the scratch array, 256-byte aligned pieces
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t b_inst = up(sizeof(Inst) * n_probs), b_pre = up(sizeof(int) * (n_probs + 1));
    const size_t b_par = up(2 * (size_t)(c.ncells + c.npseudo) * c.geo.pe * c.esize);
    const size_t b_part = up(sizeof(double) * (size_t)c.ncells * c.vsplit_max * NQ), b_pass = 256;
    const size_t total = b_inst + 2 * b_pre + b_par + b_part + b_pass;
    if (total > NOALLOC_SCRATCH_BYTES) {
        char b[200];
        snprintf(b, sizeof b, "bgk_step_noalloc: the problems need %.1f MiB of device scratch; the static array holds %d MiB",
                 (double)total / (1 << 20), BGK_NOALLOC_SCRATCH_MIB);
        return fail(nullptr, BGK_E_UNSUPPORTED, b);
    }
    if (!f_in || !f_out) return fail(nullptr, BGK_E_INVALID, "bgk_step_noalloc: NULL buffer");
    if (n_steps < 0) return fail(nullptr, BGK_E_INVALID, "bgk_step_noalloc: n_steps < 0");
    const size_t fb = c.f_elems * c.esize;
    if (overlaps(f_in, fb, f_out, fb))
        return fail(nullptr, BGK_E_ALIAS, "bgk_step_noalloc: f_in and f_out must not overlap");
    if (n_steps >= 2 && !ws) return fail(nullptr, BGK_E_INVALID, "bgk_step_noalloc: n_steps >= 2 needs the workspace");
    if (n_steps >= 2 && (overlaps(ws, fb, f_in, fb) || overlaps(ws, fb, f_out, fb)))
        return fail(nullptr, BGK_E_ALIAS, "bgk_step_noalloc: the workspace must not overlap f_in or f_out");
    hipStream_t s = (hipStream_t)stream;
    if (n_steps == 0) {
        const hipError_t e = hipMemcpyAsync(f_out, f_in, fb, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(nullptr, BGK_E_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
        return BGK_OK;
    }
    void *base = nullptr;
    rc = scratch_address(c.device, &base, msg);
    if (rc) return fail(nullptr, rc, msg);
    unsigned char *q = (unsigned char *)base;
    c.d_inst = (Inst *)q;
    q += b_inst;
    c.d_cell_prefix = (int *)q;
    q += b_pre;
    c.d_pseudo_prefix = (int *)q;
    q += b_pre;
    c.params = q;
    q += b_par;
    c.partial = (double *)q;
    q += b_part;
    c.pass = (uint32_t *)q;
    rc = upload(c.h_inst.data(), sizeof(Inst) * n_probs, c.d_inst, s, msg);
    if (!rc) rc = upload(c.h_cell_prefix.data(), sizeof(int) * (n_probs + 1), c.d_cell_prefix, s, msg);
    if (!rc) rc = upload(c.h_pseudo_prefix.data(), sizeof(int) * (n_probs + 1), c.d_pseudo_prefix, s, msg);
    if (rc) return fail(nullptr, rc, msg);
    c.work = n_steps >= 2 ? ws : nullptr;
    rc = precision == BGK_FP64 ? do_step<double>(&c, f_in, f_out, n_steps, s) : do_step<float>(&c, f_in, f_out, n_steps, s);
    if (rc) return fail(nullptr, rc, c.err);
    return BGK_OK;
}
