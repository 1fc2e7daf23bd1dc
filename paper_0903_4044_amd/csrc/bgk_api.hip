// bgk_api.hip -- host side of libbgk.so: validation, layout, launches.
// The C ABI is declared in include/bgk.h.
#include "bgk_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bgk.h"

using namespace bgk;

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
    int vsplit = 1;
    int block = 256;
    size_t esize = 8;
    // device memory owned by the context
    Inst *d_inst = nullptr;
    int *d_cell_prefix = nullptr, *d_pseudo_prefix = nullptr;
    void *work = nullptr;      // one f-sized buffer for the ping-pong
    void *params = nullptr;    // (ncells + npseudo) * pe elements
    double *partial = nullptr; // ncells * vsplit * NQ
    double *mom = nullptr;     // ncells * 5 (bgk_check)
    int *flags = nullptr;
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

static bool is2d_kind(int k) { return k == BGK_CAVITY_2D || k == BGK_PERIODIC_2D; }

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
    a.g = c->geo;
    return a;
}

static void release(bgk_ctx *c)
{
    if (!c) return;
    (void)hipFree(c->d_inst);
    (void)hipFree(c->d_cell_prefix);
    (void)hipFree(c->d_pseudo_prefix);
    (void)hipFree(c->work);
    (void)hipFree(c->params);
    (void)hipFree(c->partial);
    (void)hipFree(c->mom);
    (void)hipFree(c->flags);
    for (auto &e : c->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    delete c;
}

// Time step from the Courant rule: dt = cfl / max_j sum_d |v_d(j)| / dx_d.
static double courant_rate(const bgk_problem &p, bool two)
{
    const double dx = (p.x1 - p.x0) / p.nx, dy = two ? (p.y1 - p.y0) / p.ny : 1.0;
    double mx = 0.0, my = 0.0;
    for (int k = 0; k < p.nv[0]; ++k)
        mx = std::max(mx, std::fabs(p.vlo[0] + (k + 0.5) * (p.vhi[0] - p.vlo[0]) / p.nv[0]));
    for (int k = 0; k < p.nv[1]; ++k)
        my = std::max(my, std::fabs(p.vlo[1] + (k + 0.5) * (p.vhi[1] - p.vlo[1]) / p.nv[1]));
    return mx / dx + (two ? my / dy : 0.0);
}

static int validate(const bgk_problem &p, int idx, std::string &msg)
{
    char b[256];
    auto bad = [&](const char *what) {
        snprintf(b, sizeof b, "problem %d: %s", idx, what);
        msg = b;
        return BGK_E_INVALID;
    };
    if (p.kind < 0 || p.kind > 3) return bad("unknown kind");
    const bool two = is2d_kind(p.kind);
    if (p.nx < 1 || (two && p.ny < 1)) return bad("nx, ny must be >= 1");
    if (p.kind == BGK_PERIODIC_1D && p.nx < 2) return bad("periodic boxes need nx >= 2");
    if (p.kind == BGK_PERIODIC_2D && (p.nx < 2 || p.ny < 2)) return bad("periodic boxes need nx, ny >= 2");
    if (!(p.x1 > p.x0) || (two && !(p.y1 > p.y0))) return bad("empty spatial box");
    for (int a = 0; a < 3; ++a) {
        if (p.nv[a] < 2 || p.nv[a] > NVMAX) {
            msg = "velocity cells per component must be in [2, 128]";
            return BGK_E_UNSUPPORTED;
        }
        if (!(p.vhi[a] > p.vlo[a])) return bad("empty velocity box");
    }
    if (!(p.kn > 0.0) || !std::isfinite(p.kn)) return bad("Kn must be > 0");
    if (!std::isfinite(p.omega)) return bad("omega must be finite");
    if (p.splitting != BGK_STRANG && p.splitting != BGK_LIE) return bad("unknown splitting");
    if (p.limiter != BGK_MINMOD && p.limiter != BGK_NOLIMIT) return bad("unknown limiter");
    if (p.kind == BGK_SHOCK_1D && !(p.mach > 1.0)) return bad("shock needs Mach > 1");
    if (p.kind == BGK_CAVITY_2D && !(p.t_wall > 0.0)) return bad("wall temperature must be > 0");
    if (!(p.dt > 0.0) && !(p.cfl > 0.0)) return bad("need dt > 0 or cfl > 0");
    const double rate = courant_rate(p, two);
    const double dt = p.dt > 0.0 ? p.dt : p.cfl / rate;
    if (dt * rate > 2.0 / 3.0 * (1.0 + 1e-12)) {
        snprintf(b, sizeof b, "problem %d: Courant sum %.6g exceeds 2/3", idx, dt * rate);
        msg = b;
        return BGK_E_CFL;
    }
    return BGK_OK;
}

extern "C" int bgk_init(const bgk_problem *probs, int n_probs, int precision, bgk_ctx **out)
{
    if (!out) return fail(nullptr, BGK_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!probs || n_probs < 1) return fail(nullptr, BGK_E_INVALID, "need at least one problem");
    if (precision != BGK_FP64 && precision != BGK_FP32) return fail(nullptr, BGK_E_INVALID, "unknown precision");
    for (int i = 0; i < n_probs; ++i) {
        std::string msg;
        int rc = validate(probs[i], i, msg);
        if (rc) return fail(nullptr, rc, msg);
        const bgk_problem &p = probs[i], &q = probs[0];
        if (is2d_kind(p.kind) != is2d_kind(q.kind))
            return fail(nullptr, BGK_E_UNSUPPORTED, "all instances must have the same dimension");
        for (int a = 0; a < 3; ++a)
            if (p.nv[a] != q.nv[a] || p.vlo[a] != q.vlo[a] || p.vhi[a] != q.vhi[a])
                return fail(nullptr, BGK_E_UNSUPPORTED, "all instances must share the velocity grid");
    }
    bgk_ctx *c = new bgk_ctx;
    c->precision = precision;
    c->esize = precision == BGK_FP64 ? 8 : 4;
    c->ninst = n_probs;
    c->dim = is2d_kind(probs[0].kind) ? 2 : 1;
    c->probs.assign(probs, probs + n_probs);
    (void)hipGetDevice(&c->device);

    Geo &g = c->geo;
    g.nvx = probs[0].nv[0];
    g.nvy = probs[0].nv[1];
    g.nvz = probs[0].nv[2];
    g.npl = g.nvx * g.nvy;
    g.nv = (long long)g.npl * g.nvz;
    g.dV = 1.0;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = probs[0].vlo[a];
        g.dv[a] = (probs[0].vhi[a] - probs[0].vlo[a]) / probs[0].nv[a];
        g.dV *= g.dv[a];
    }
    g.tx1 = 4;
    g.ty1 = g.tx1 + g.nvx;
    g.tx2 = g.ty1 + g.nvy;
    g.ty2 = g.tx2 + g.nvx;
    g.tz = (g.ty2 + g.nvy + 1) & ~1;
    g.pe = (g.tz + 2 * g.nvz + 3) & ~3;

    c->h_cell_prefix.push_back(0);
    c->h_pseudo_prefix.push_back(0);
    long long f_off = 0;
    for (int i = 0; i < n_probs; ++i) {
        const bgk_problem &p = probs[i];
        const bool two = is2d_kind(p.kind);
        Inst I{};
        I.kind = p.kind;
        I.nx = p.nx;
        I.ny = two ? p.ny : 1;
        I.ncell = I.nx * I.ny;
        I.cell0 = c->h_cell_prefix.back();
        I.strang = p.splitting == BGK_STRANG;
        I.minmod = p.limiter == BGK_MINMOD;
        I.f0 = f_off;
        const double dx = (p.x1 - p.x0) / p.nx, dy = two ? (p.y1 - p.y0) / p.ny : 1.0;
        I.dt = p.dt > 0.0 ? p.dt : p.cfl / courant_rate(p, two);
        I.cx = I.dt / dx;
        I.cy = two ? I.dt / dy : 0.0;
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
        const int np = p.kind == BGK_SHOCK_1D ? 2 : p.kind == BGK_CAVITY_2D ? 2 * I.nx + 2 * I.ny : 0;
        if ((long long)I.ncell * g.nv * (long long)c->esize >= (1LL << 31) * 2LL) {
            release(c);
            return fail(nullptr, BGK_E_UNSUPPORTED, "one instance must hold fewer than 2^32 bytes of f");
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

    // Velocity chunks per cell: enough workgroups to fill 256 CUs several times.
    const int target = 4096;
    c->vsplit = std::max(1, std::min(g.nvz, (target + c->ncells - 1) / c->ncells));
    c->block = 256;

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
    ALLOC(c->work, c->f_elems * c->esize);
    ALLOC(c->params, (size_t)(c->ncells + c->npseudo) * g.pe * c->esize);
    ALLOC(c->partial, sizeof(double) * (size_t)c->ncells * c->vsplit * NQ);
    ALLOC(c->mom, sizeof(double) * (size_t)c->ncells * 5);
    ALLOC(c->flags, sizeof(int));
#undef ALLOC
    hipError_t e1 = hipMemcpy(c->d_inst, c->h_inst.data(), sizeof(Inst) * n_probs, hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(c->d_cell_prefix, c->h_cell_prefix.data(), sizeof(int) * (n_probs + 1), hipMemcpyHostToDevice);
    hipError_t e3 = hipMemcpy(c->d_pseudo_prefix, c->h_pseudo_prefix.data(), sizeof(int) * (n_probs + 1), hipMemcpyHostToDevice);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
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

extern "C" int bgk_sizes(const bgk_ctx *ctx, size_t *f_elems, size_t *n_cells)
{
    if (!ctx) return BGK_E_INVALID;
    if (f_elems) *f_elems = ctx->f_elems;
    if (n_cells) *n_cells = (size_t)ctx->ncells;
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
static int launch_moments(bgk_ctx *c, const void *f, hipStream_t s)
{
    const int nb = c->ncells * c->vsplit;
    hipLaunchKernelGGL(k_moments<real>, dim3(nb), dim3(c->block), 0, s, make_args(c), (const real *)f, c->partial);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

template <typename real>
static int launch_prep(bgk_ctx *c, int mode, hipStream_t s)
{
    const int nb = c->ncells + (mode == MODE_FINAL ? 0 : c->npseudo);
    hipLaunchKernelGGL(k_prep<real>, dim3(nb), dim3(64), 0, s, make_args(c), c->partial, (real *)c->params, mode);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

template <typename real>
static int launch_stream(bgk_ctx *c, const void *src, void *dst, hipStream_t s)
{
    const int nb = c->ncells * c->vsplit;
    const int nslot = c->dim == 1 ? 7 : 13;
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
    if (c->dim == 1)
        hipLaunchKernelGGL((k_stream<real, 1>), dim3(nb), dim3(c->block), lds, s, make_args(c), (const real *)src,
                           (real *)dst, (const real *)c->params, c->partial);
    else
        hipLaunchKernelGGL((k_stream<real, 2>), dim3(nb), dim3(c->block), lds, s, make_args(c), (const real *)src,
                           (real *)dst, (const real *)c->params, c->partial);
    HIP_TRY(c, hipGetLastError());
    if (c->timing) HIP_TRY(c, hipEventRecord(e1, s));
    return BGK_OK;
}

template <typename real>
static int launch_final(bgk_ctx *c, const void *src, void *dst, hipStream_t s)
{
    const int nb = c->ncells * c->vsplit;
    hipLaunchKernelGGL(k_final<real>, dim3(nb), dim3(c->block), 0, s, make_args(c), (const real *)src, (real *)dst,
                       (const real *)c->params);
    HIP_TRY(c, hipGetLastError());
    return BGK_OK;
}

#define TRY(x)                   \
    do {                         \
        int rc_ = (x);           \
        if (rc_) return rc_;     \
    } while (0)

template <typename real>
static int do_step(bgk_ctx *c, const void *f_in, void *f_out, int n, hipStream_t s)
{
    TRY(launch_moments<real>(c, f_in, s));
    TRY(launch_prep<real>(c, MODE_FIRST, s));
    const void *src = f_in;
    for (int k = 1; k <= n; ++k) {
        // The last streaming pass lands in f_out; earlier ones alternate with the work buffer.
        void *dst = ((n - k) % 2 == 0) ? f_out : c->work;
        TRY(launch_stream<real>(c, src, dst, s));
        TRY(launch_prep<real>(c, k < n ? MODE_MID : MODE_FINAL, s));
        src = dst;
    }
    return launch_final<real>(c, f_out, f_out, s);
}

extern "C" int bgk_step(bgk_ctx *ctx, const void *f_in, void *f_out, int n_steps, void *stream)
{
    if (!ctx) return BGK_E_INVALID;
    if (!f_in || !f_out) return fail(ctx, BGK_E_INVALID, "bgk_step: NULL buffer");
    if (n_steps < 0) return fail(ctx, BGK_E_INVALID, "bgk_step: n_steps < 0");
    if (f_in == f_out) return fail(ctx, BGK_E_ALIAS, "bgk_step: f_in and f_out must differ");
    hipStream_t s = (hipStream_t)stream;
    if (n_steps == 0) {
        HIP_TRY(ctx, hipMemcpyAsync(f_out, f_in, ctx->f_elems * ctx->esize, hipMemcpyDeviceToDevice, s));
        return BGK_OK;
    }
    return ctx->precision == BGK_FP64 ? do_step<double>(ctx, f_in, f_out, n_steps, s)
                                      : do_step<float>(ctx, f_in, f_out, n_steps, s);
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
    const int nb = ctx->ncells * ctx->vsplit;
    if (ctx->precision == BGK_FP64)
        hipLaunchKernelGGL(k_init<double>, dim3(nb), dim3(ctx->block), 0, s, make_args(ctx), (double *)f);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(nb), dim3(ctx->block), 0, s, make_args(ctx), (float *)f);
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
    for (size_t i = 0; i < ctx->ev_used; ++i) {
        HIP_TRY(ctx, hipEventSynchronize(ctx->events[i].second));
        float t = 0.0f;
        HIP_TRY(ctx, hipEventElapsedTime(&t, ctx->events[i].first, ctx->events[i].second));
        tot += t;
    }
    if (ms) *ms = tot;
    if (launches) *launches = (int)ctx->ev_used;
    ctx->ev_used = 0;
    return BGK_OK;
}
