// bgk_device.h -- gfx950 kernels of the BGK discrete-velocity step.
//
// State between launches.  A time step is R2 S R1 (Strang: R1 = R2 = R_{dt/2};
// Lie: R1 = identity, R2 = R_dt).  Composing k steps,
//     f^k = R2 S (R1 R2) S (R1 R2) ... S R1 f^0,
// so the streaming kernel works on the streamed-but-not-yet-relaxed state
// h^n = S(...) and applies, on the fly, the relaxations that sit between two
// streaming passes: g = R1(R2(h^n)), h^{n+1} = S(g).  f is never materialised
// between steps; the last launch of bgk_step applies R2 pointwise.  Each
// streaming launch therefore reads h^n once and writes h^{n+1} once.
//
// Relaxation (Eq. relaxation of Sec. 2.1) is affine in f once the Maxwellian
// parameters are fixed: R(x) = a Phi(m(x)) + (1 - a) x, a = 1 - exp(-nu tau).
// The moments of R2(h) follow from those of h without touching f again:
//     m(R2(h)) = a2 m(Phi2) + (1 - a2) m(h),
// where m(Phi2) is a product of 1D sums because the discrete Maxwellian
// factorises over velocity components.  So the pair R1 R2 reduces, per cell,
// to   g = c0 h + c1 Phi2 + c2 Phi1   with three scalars and six 1D tables,
// prepared once per cell per launch by k_prep from the FP64 moment sums of h
// that the previous streaming launch reduced.
//
// Table entries ("params").  One entry per spatial cell and one per ghost
// source ("pseudo" entry: the two far-field Maxwellians of a shock, one
// emitted wall Maxwellian n_W Phi_W per wall face of a cavity).  An entry holds
//     c0, TX1[Nvx], TY1[Nvy], TX2[Nvx], TY2[Nvy], TZ[Nvz][2]
// and evaluates to   g(j) = c0 h(j) + TX1[jx] TY1[jy] TZ[jz][0]
//                                 + TX2[jx] TY2[jy] TZ[jz][1].
// For a pseudo entry c0 = 0, so the ghost value is a pure Maxwellian.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bgk {

constexpr int NVMAX = 128;        // per velocity component
constexpr int KIND_SHOCK = 0, KIND_CAVITY = 1, KIND_PER1 = 2, KIND_PER2 = 3;
constexpr int MODE_FIRST = 0, MODE_MID = 1, MODE_FINAL = 2;
constexpr int NQ = 9;             // moment sums per cell: 1, vx, vy, vz, |v|^2, 4 half fluxes

struct Inst {
    int kind, nx, ny, ncell;
    int cell0;      // first global cell index of the instance
    int pseudo0;    // first global params entry of its ghost sources
    int strang, minmod;
    long long f0;   // element offset of the instance in f
    double cx, cy;  // dt / dx, dt / dy
    double dt, kn, omega;
    double tw, uw;  // wall temperature, lid speed
    double x0, dx;  // spatial origin and cell size along x
    double up[3], dn[3];  // shock far-field (n, V, T)
};

struct Geo {
    int nvx, nvy, nvz;
    int npl;                    // nvx * nvy
    long long nv;               // nvx * nvy * nvz
    double lo[3], dv[3];
    double dV;
    int pe;                     // params entry stride (elements)
    int tx1, ty1, tx2, ty2, tz; // entry offsets
};

struct Args {
    const Inst *inst;
    const int *cell_prefix;     // ninst + 1
    const int *pseudo_prefix;   // ninst + 1 (global params index of pseudo entries)
    int ninst;
    int ncells;                 // total cells
    int npseudo;                // total pseudo entries
    int vsplit;                 // velocity chunks (along jz) per cell
    Geo g;
};

__device__ __forceinline__ int find_inst(const int *prefix, int n, int x)
{
    int lo = 0, hi = n;  // prefix[lo] <= x < prefix[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (prefix[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// Work-group placement.  Consecutive workgroup ids land on the eight XCDs
// round-robin, and each XCD has its own L2.  Remap so that XCD x processes a
// contiguous block of logical work items (neighbouring cells share L2).
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    constexpr int X = 8;
    int q = nb / X, r = nb % X;
    int x = b % X, k = b / X;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ double vnode(const Geo &g, int a, int k) { return g.lo[a] + (k + 0.5) * g.dv[a]; }

__device__ __forceinline__ float minmod3(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double minmod3(double a, double b) { return fmax(fmin(a, b), fmin(fmax(a, b), 0.0)); }

// Deterministic block reduction of NQ doubles; thread q < NQ writes out[q].
template <int N>
__device__ __forceinline__ void block_sum_store(double (&acc)[N], double *out)
{
    __shared__ double red[16][N];
#pragma unroll
    for (int q = 0; q < N; ++q)
        for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < N; ++q) red[w][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < N) {
        double s = 0.0;
        for (int k = 0; k < nw; ++k) s += red[k][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Per-p (one (jx, jy) column, summed over its jz range) contribution to the
// nine moment sums: A0 = sum h, Az = sum vz h, Azz = sum vz^2 h.
__device__ __forceinline__ void fold_column(double (&acc)[NQ], double vx, double vy, double A0, double Az, double Azz)
{
    acc[0] += A0;
    acc[1] += vx * A0;
    acc[2] += vy * A0;
    acc[3] += Az;
    acc[4] += (vx * vx + vy * vy) * A0 + Azz;
    acc[5] += vx < 0.0 ? -vx * A0 : 0.0;
    acc[6] += vx > 0.0 ? vx * A0 : 0.0;
    acc[7] += vy < 0.0 ? -vy * A0 : 0.0;
    acc[8] += vy > 0.0 ? vy * A0 : 0.0;
}

// ---------------------------------------------------------------- moments
// Partial moment sums of f over one jz chunk of one cell:
// partial[(cell * vsplit + split) * NQ + q] (without the dV factor).
template <typename real>
__global__ void __launch_bounds__(256) k_moments(Args A, const real *__restrict__ f, double *__restrict__ partial)
{
    const Geo &g = A.g;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int gc = L / A.vsplit, split = L % A.vsplit;
    const int ii = find_inst(A.cell_prefix, A.ninst, gc);
    const Inst &I = A.inst[ii];
    const real *fc = f + I.f0 + (long long)(gc - I.cell0) * g.nv;
    const int z0 = split * g.nvz / A.vsplit, z1 = (split + 1) * g.nvz / A.vsplit;
    double acc[NQ] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int p = threadIdx.x; p < g.npl; p += blockDim.x) {
        const int jx = p % g.nvx, jy = p / g.nvx;
        double A0 = 0, Az = 0, Azz = 0;
        for (int jz = z0; jz < z1; ++jz) {
            const double h = (double)fc[(long long)jz * g.npl + p];
            const double vz = vnode(g, 2, jz);
            A0 += h;
            Az += vz * h;
            Azz += vz * vz * h;
        }
        fold_column(acc, vnode(g, 0, jx), vnode(g, 1, jy), A0, Az, Azz);
    }
    block_sum_store<NQ>(acc, partial + (long long)L * NQ);
}

// Per-cell macroscopic moments (n, Vx, Vy, Vz, T) from the partial sums.
__global__ void k_macro(Args A, const double *__restrict__ partial, double *__restrict__ mom)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= A.ncells) return;
    double s[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < A.vsplit; ++k)
        for (int q = 0; q < 5; ++q) s[q] += partial[((long long)c * A.vsplit + k) * NQ + q];
    const double n = s[0] * A.g.dV;
    const double vx = s[1] / s[0], vy = s[2] / s[0], vz = s[3] / s[0];
    const double T = 2.0 / 3.0 * (s[4] / s[0] - (vx * vx + vy * vy + vz * vz));
    mom[5 * c + 0] = n;
    mom[5 * c + 1] = vx;
    mom[5 * c + 2] = vy;
    mom[5 * c + 3] = vz;
    mom[5 * c + 4] = T;
}

// Flags: bit 0 non-finite moment, bit 1 n <= 0 or T <= 0.
__global__ void k_check(int ncells, const double *__restrict__ mom, int *__restrict__ flags)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    int bad = 0;
    for (int q = 0; q < 5; ++q)
        if (!isfinite(mom[5 * c + q])) bad |= 1;
    if (!(mom[5 * c] > 0.0) || !(mom[5 * c + 4] > 0.0)) bad |= 2;
    if (bad) atomicOr(flags, bad);
}

// ---------------------------------------------------------------- prep
// One 64-thread workgroup per params entry.

// Relaxation times of the two relaxations folded into a table entry.
//   FIRST: g = R1(f0)        (Strang: R_{dt/2}; Lie: identity)
//   MID:   g = R1(R2(h))     (Strang: R_{dt/2} R_{dt/2}; Lie: R_dt)
//   FINAL: f = R2(h)         (Strang: R_{dt/2}; Lie: R_dt)
// Returned in application order: ta is applied first, tb second; nr relaxations.
__device__ __forceinline__ int relax_times(const Inst &I, int mode, double *ta, double *tb)
{
    const double h = 0.5 * I.dt;
    if (I.strang) {
        *ta = h;
        *tb = h;
        return mode == MODE_MID ? 2 : 1;
    }
    *ta = I.dt;
    *tb = 0.0;
    return mode == MODE_FIRST ? 0 : 1;
}

struct Relax {          // Maxwellian parameters of one relaxation
    double n, V[3], T, a, P;
};

__device__ __forceinline__ void moments_from_raw(const double *raw, Relax *r)
{
    r->n = raw[0];
    r->V[0] = raw[1] / raw[0];
    r->V[1] = raw[2] / raw[0];
    r->V[2] = raw[3] / raw[0];
    r->T = 2.0 / 3.0 * (raw[4] / raw[0] - (r->V[0] * r->V[0] + r->V[1] * r->V[1] + r->V[2] * r->V[2]));
}

__device__ __forceinline__ void finish_relax(const Inst &I, double tau, Relax *r)
{
    const double nu = r->n * pow(r->T, 1.0 - I.omega) / I.kn;
    r->a = -expm1(-nu * tau);
    r->P = r->n * pow(M_PI * r->T, -1.5);
}

// e[a * NVMAX + k] = exp(-(v_a(k) - V_a)^2 / T) for all three components.
__device__ __forceinline__ void exp_tables(const Geo &g, const double V[3], double T, double *e)
{
    const int n = g.nvx + g.nvy + g.nvz;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        int a, k;
        if (t < g.nvx) { a = 0; k = t; }
        else if (t < g.nvx + g.nvy) { a = 1; k = t - g.nvx; }
        else { a = 2; k = t - g.nvx - g.nvy; }
        const double d = vnode(g, a, k) - V[a];
        e[a * NVMAX + k] = exp(-d * d / T);
    }
}

// Serial 1D sums of a table (one thread per component, fixed order):
// s[a][0] = sum e, s[a][1] = sum v e, s[a][2] = sum v^2 e,
// s[a][3] = sum_{v<0} |v| e, s[a][4] = sum_{v>0} v e.
__device__ __forceinline__ void table_sums(const Geo &g, const double *e, double (*s)[5])
{
    const int a = threadIdx.x;
    if (a < 3) {
        const int n = a == 0 ? g.nvx : (a == 1 ? g.nvy : g.nvz);
        double s0 = 0, s1 = 0, s2 = 0, sm = 0, sp = 0;
        for (int k = 0; k < n; ++k) {
            const double v = vnode(g, a, k), x = e[a * NVMAX + k];
            s0 += x;
            s1 += v * x;
            s2 += v * v * x;
            if (v < 0.0) sm += -v * x;
            else if (v > 0.0) sp += v * x;
        }
        s[a][0] = s0; s[a][1] = s1; s[a][2] = s2; s[a][3] = sm; s[a][4] = sp;
    }
}

// Raw moments (with dV) of the discrete Maxwellian P * e_x e_y e_z.
__device__ __forceinline__ void maxwell_raw(double P, double dV, const double (*s)[5], double *m)
{
    const double w = P * dV;
    m[0] = w * s[0][0] * s[1][0] * s[2][0];
    m[1] = w * s[0][1] * s[1][0] * s[2][0];
    m[2] = w * s[0][0] * s[1][1] * s[2][0];
    m[3] = w * s[0][0] * s[1][0] * s[2][1];
    m[4] = w * (s[0][2] * s[1][0] * s[2][0] + s[0][0] * s[1][2] * s[2][0] + s[0][0] * s[1][0] * s[2][2]);
}

// Shared state of one prep workgroup.
struct PrepShared {
    double raw[NQ];
    double e1[3 * NVMAX], e2[3 * NVMAX];
    double s1[3][5], s2[3][5];
    Relax r1, r2;       // r1 applied first, r2 second
    double c0, cA, cB;  // g = c0 h + cA * Phi_1 + cB * Phi_2 (cA, cB include P)
    int nr;
};

// Coefficients of the relaxations folded into one cell's entry, from that
// cell's partial moment sums.  All threads of the workgroup take part.
__device__ void cell_coefficients(const Args &A, const Inst &I, int gc, int mode, const double *partial, PrepShared &S,
                                  bool want_sums)
{
    const Geo &g = A.g;
    if (threadIdx.x < NQ) {
        double s = 0.0;
        for (int k = 0; k < A.vsplit; ++k) s += partial[((long long)gc * A.vsplit + k) * NQ + threadIdx.x];
        S.raw[threadIdx.x] = s * g.dV;
    }
    __syncthreads();
    double ta, tb;
    const int nr = relax_times(I, mode, &ta, &tb);
    if (threadIdx.x == 0) {
        S.nr = nr;
        S.c0 = 1.0; S.cA = 0.0; S.cB = 0.0;
        if (nr >= 1) { moments_from_raw(S.raw, &S.r1); finish_relax(I, ta, &S.r1); }
    }
    __syncthreads();
    if (nr >= 1) {
        exp_tables(g, S.r1.V, S.r1.T, S.e1);
        __syncthreads();
        if (nr == 2 || want_sums) { table_sums(g, S.e1, S.s1); __syncthreads(); }
        if (nr == 2) {
            if (threadIdx.x == 0) {
                double mp[5], m2[5];
                maxwell_raw(S.r1.P, g.dV, S.s1, mp);
                for (int q = 0; q < 5; ++q) m2[q] = S.r1.a * mp[q] + (1.0 - S.r1.a) * S.raw[q];
                moments_from_raw(m2, &S.r2);
                finish_relax(I, tb, &S.r2);
            }
            __syncthreads();
            exp_tables(g, S.r2.V, S.r2.T, S.e2);
            __syncthreads();
            if (want_sums) { table_sums(g, S.e2, S.s2); __syncthreads(); }
        }
        if (threadIdx.x == 0) {
            if (nr == 2) {
                S.c0 = (1.0 - S.r1.a) * (1.0 - S.r2.a);
                S.cA = S.r1.a * (1.0 - S.r2.a) * S.r1.P;
                S.cB = S.r2.a * S.r2.P;
            } else {
                S.c0 = 1.0 - S.r1.a;
                S.cA = S.r1.a * S.r1.P;
            }
        }
        __syncthreads();
    }
}

template <typename real>
__device__ void write_entry(const Geo &g, real *E, double c0, double cA, const double *eA, double cB, const double *eB,
                            bool hasA, bool hasB)
{
    for (int t = threadIdx.x; t < g.pe; t += blockDim.x) {
        double v = 0.0;
        if (t == 0) v = c0;
        else if (t >= g.tx1 && t < g.tx1 + g.nvx) v = hasA ? cA * eA[t - g.tx1] : 0.0;
        else if (t >= g.ty1 && t < g.ty1 + g.nvy) v = hasA ? eA[NVMAX + t - g.ty1] : 0.0;
        else if (t >= g.tx2 && t < g.tx2 + g.nvx) v = hasB ? cB * eB[t - g.tx2] : 0.0;
        else if (t >= g.ty2 && t < g.ty2 + g.nvy) v = hasB ? eB[NVMAX + t - g.ty2] : 0.0;
        else if (t >= g.tz && t < g.tz + 2 * g.nvz) {
            const int k = (t - g.tz) >> 1;
            if ((t - g.tz) & 1) v = hasB ? eB[2 * NVMAX + k] : 0.0;
            else v = hasA ? eA[2 * NVMAX + k] : 0.0;
        }
        E[t] = (real)v;
    }
}

// Wall geometry: wall w = 0 left (+x inward), 1 right (-x), 2 bottom (+y), 3 top (-y).
__device__ __forceinline__ int wall_of_entry(const Inst &I, int k, int *pos)
{
    if (k < I.ny) { *pos = k; return 0; }
    k -= I.ny;
    if (k < I.ny) { *pos = k; return 1; }
    k -= I.ny;
    if (k < I.nx) { *pos = k; return 2; }
    *pos = k - I.nx;
    return 3;
}

template <typename real>
__global__ void __launch_bounds__(64) k_prep(Args A, const double *__restrict__ partial, real *__restrict__ params, int mode)
{
    __shared__ PrepShared S;
    __shared__ double ew[3 * NVMAX];
    __shared__ double sw[3][5];
    const Geo &g = A.g;
    const int e = blockIdx.x;
    if (e < A.ncells) {
        const int ii = find_inst(A.cell_prefix, A.ninst, e);
        const Inst &I = A.inst[ii];
        cell_coefficients(A, I, e, mode, partial, S, false);
        write_entry<real>(g, params + (long long)e * g.pe, S.c0, S.cA, S.e1, S.cB, S.e2, S.nr >= 1, S.nr == 2);
        return;
    }
    // ghost sources
    const int pe = e - A.ncells;
    const int ii = find_inst(A.pseudo_prefix, A.ninst, pe);
    const Inst &I = A.inst[ii];
    const int k = pe - A.pseudo_prefix[ii];
    real *E = params + (long long)e * g.pe;
    if (I.kind == KIND_SHOCK) {
        // Far-field Maxwellian of Eq. (bc_shock): k = 0 upstream (x < x0), 1 downstream.
        const double *st = k == 0 ? I.up : I.dn;
        const double V[3] = {st[1], 0.0, 0.0};
        exp_tables(g, V, st[2], S.e1);
        __syncthreads();
        write_entry<real>(g, E, 0.0, st[0] * pow(M_PI * st[2], -1.5), S.e1, 0.0, S.e2, true, false);
        return;
    }
    // Diffuse wall face, Eq. (bc_cavity): ghost = n_W Phi_W for velocities
    // leaving the wall.  n_W makes the discrete net mass flux zero:
    //   n_W = sum_{v.n<0} |v.n| g0 / sum_{v.n>0} v.n Phi_W,
    // g0 being the wall-adjacent cell of the streaming input, g0 = c0 h + cA Phi_1 + cB Phi_2.
    int pos;
    const int w = wall_of_entry(I, k, &pos);
    const int axis = w < 2 ? 0 : 1;
    const int adj = w == 0 ? pos * I.nx : w == 1 ? pos * I.nx + I.nx - 1 : w == 2 ? pos : (I.ny - 1) * I.nx + pos;
    cell_coefficients(A, I, I.cell0 + adj, mode, partial, S, true);
    const double VW[3] = {w == 3 ? I.uw : 0.0, 0.0, 0.0};
    exp_tables(g, VW, I.tw, ew);
    __syncthreads();
    table_sums(g, ew, sw);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int b1 = axis == 0 ? 1 : 0;  // the two other components
        const int b2 = 2;
        // incident: v_axis < 0 for walls 0, 2 (index 3 of the sums), v_axis > 0 for walls 1, 3 (index 4)
        const int in = (w == 0 || w == 2) ? 3 : 4, out = (w == 0 || w == 2) ? 4 : 3;
        const double hraw = S.raw[5 + (w == 0 ? 0 : w == 1 ? 1 : w == 2 ? 2 : 3)];
        double flux = S.c0 * hraw;
        if (S.nr >= 1) flux += S.cA * g.dV * S.s1[axis][in] * S.s1[b1][0] * S.s1[b2][0];
        if (S.nr == 2) flux += S.cB * g.dV * S.s2[axis][in] * S.s2[b1][0] * S.s2[b2][0];
        const double pw = pow(M_PI * I.tw, -1.5);
        const double den = pw * g.dV * sw[axis][out] * sw[b1][0] * sw[b2][0];
        S.r2.n = flux / den;  // n_W (r2 is free here)
        S.r2.P = S.r2.n * pw;
    }
    __syncthreads();
    write_entry<real>(g, E, 0.0, S.r2.P, ew, 0.0, S.e2, true, false);
}

// ---------------------------------------------------------------- stream
// One workgroup per (cell, jz chunk).  Thread lanes run over the (jx, jy)
// plane, each lane loops over jz.  Per lane and velocity the upwind stencil
// in each direction is {i - 2s, i - s, i, i + s} with s = sign(v_d); a slot
// table resolves every stencil position (interior cell, periodic image,
// far-field Maxwellian, wall-adjacent cell or emitted wall Maxwellian) once
// per workgroup, so the inner loop is branch-free.
//
// Slots: 0 centre; 1 + 3*si + m (x direction), 7 + 3*si + m (y direction),
// si = 0 for s = +1, 1 for s = -1; m = 0, 1, 2 for k = -2, -1, +1.

struct SlotInfo { int cell[13]; int par[13]; };

__device__ __forceinline__ void resolve_slot(const Inst &I, int axis, int pos, int other, int sgn, int own, int *cell, int *par)
{
    const int N = axis == 0 ? I.nx : I.ny;
    auto at = [&](int q) { return axis == 0 ? other * I.nx + q : q * I.nx + other; };
    if (pos >= 0 && pos < N) { *cell = at(pos); *par = I.cell0 + *cell; return; }
    if (I.kind == KIND_PER1 || I.kind == KIND_PER2) {
        const int q = ((pos % N) + N) % N;
        *cell = at(q); *par = I.cell0 + *cell; return;
    }
    if (I.kind == KIND_SHOCK) { *cell = own; *par = I.pseudo0 + (pos < 0 ? 0 : 1); return; }
    const bool low = pos < 0;
    const bool emitted = low ? (sgn > 0) : (sgn < 0);
    if (emitted) {
        const int w = axis == 0 ? (low ? 0 : 1) : (low ? 2 : 3);
        const int off = w == 0 ? 0 : w == 1 ? I.ny : w == 2 ? 2 * I.ny : 2 * I.ny + I.nx;
        *cell = own;
        *par = I.pseudo0 + off + other;
    } else {
        *cell = at(low ? 0 : N - 1);
        *par = I.cell0 + *cell;
    }
}

template <typename real>
struct Tap {           // one stencil input for the current lane
    const real *src;   // h at (slot cell, jz = 0, this p)
    const real *tz;    // TZ of the slot entry (LDS)
    real c0, l1, l2;
    __device__ __forceinline__ real eval(int jz, long long zoff) const
    {
        const real h = src[zoff];
        const real a = tz[2 * jz], b = tz[2 * jz + 1];
        return c0 * h + (l1 * a + l2 * b);
    }
};

template <typename real>
__device__ __forceinline__ Tap<real> make_tap(const Geo &g, const real *sp, const SlotInfo &SI, int slot, const real *base,
                                              int p, int jx, int jy)
{
    Tap<real> t;
    const real *E = sp + slot * g.pe;
    t.src = base + (long long)SI.cell[slot] * g.nv + p;
    t.tz = E + g.tz;
    t.c0 = E[0];
    t.l1 = E[g.tx1 + jx] * E[g.ty1 + jy];
    t.l2 = E[g.tx2 + jx] * E[g.ty2 + jy];
    return t;
}

// Upwind flux difference along one direction, values in upwind order
// (u_{-2}, u_{-1}, u_0, u_1) for Courant magnitude C and slope factor k = (1 - C)/2.
template <typename real>
__device__ __forceinline__ real flux_diff(real um2, real um1, real u0, real u1, real C, real k)
{
    const real fp = u0 + k * minmod3(u1 - u0, u0 - um1);
    const real fm = um1 + k * minmod3(u0 - um1, um1 - um2);
    return C * (fp - fm);
}

template <typename real, int DIM>
__global__ void __launch_bounds__(256) k_stream(Args A, const real *__restrict__ src, real *__restrict__ dst,
                                                const real *__restrict__ params, double *__restrict__ partial)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NSLOT = DIM == 1 ? 7 : 13;
    real *sp = reinterpret_cast<real *>(smem);
    __shared__ SlotInfo SI;
    const Geo &g = A.g;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int gc = L / A.vsplit, split = L % A.vsplit;
    const int ii = find_inst(A.cell_prefix, A.ninst, gc);
    const Inst &I = A.inst[ii];
    const int c = gc - I.cell0;
    const int ix = c % I.nx, iy = c / I.nx;

    if (threadIdx.x < NSLOT) {
        const int s = threadIdx.x;
        int cell, par;
        if (s == 0) { cell = c; par = gc; }
        else {
            const int d = (s - 1) / 6, r = (s - 1) % 6, si = r / 3, m = r % 3;
            const int sgn = si == 0 ? 1 : -1, k = m == 0 ? -2 : (m == 1 ? -1 : 1);
            if (d == 0) resolve_slot(I, 0, ix + sgn * k, iy, sgn, c, &cell, &par);
            else resolve_slot(I, 1, iy + sgn * k, ix, sgn, c, &cell, &par);
        }
        SI.cell[s] = cell;
        SI.par[s] = par;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NSLOT * g.pe; t += blockDim.x) {
        const int s = t / g.pe, o = t - s * g.pe;
        sp[t] = params[(long long)SI.par[s] * g.pe + o];
    }
    __syncthreads();

    const real *base = src + I.f0;
    real *out = dst + I.f0 + (long long)c * g.nv;
    const int z0 = split * g.nvz / A.vsplit, z1 = (split + 1) * g.nvz / A.vsplit;
    const bool lim = I.minmod != 0;
    double acc[NQ] = {0, 0, 0, 0, 0, 0, 0, 0, 0};

    for (int p = threadIdx.x; p < g.npl; p += blockDim.x) {
        const int jx = p % g.nvx, jy = p / g.nvx;
        const double vx = vnode(g, 0, jx), vy = vnode(g, 1, jy);
        const int sx = vx > 0.0 ? 0 : 1;
        const real Cx = (real)(fabs(vx) * I.cx);
        const real kx = lim ? (real)0.5 * ((real)1 - Cx) : (real)0;
        const Tap<real> tc = make_tap<real>(g, sp, SI, 0, base, p, jx, jy);
        const Tap<real> xa = make_tap<real>(g, sp, SI, 1 + 3 * sx + 0, base, p, jx, jy);
        const Tap<real> xb = make_tap<real>(g, sp, SI, 1 + 3 * sx + 1, base, p, jx, jy);
        const Tap<real> xd = make_tap<real>(g, sp, SI, 1 + 3 * sx + 2, base, p, jx, jy);
        Tap<real> ya, yb, yd;
        real Cy = 0, ky = 0;
        if constexpr (DIM == 2) {
            const int sy = vy > 0.0 ? 0 : 1;
            Cy = (real)(fabs(vy) * I.cy);
            ky = lim ? (real)0.5 * ((real)1 - Cy) : (real)0;
            ya = make_tap<real>(g, sp, SI, 7 + 3 * sy + 0, base, p, jx, jy);
            yb = make_tap<real>(g, sp, SI, 7 + 3 * sy + 1, base, p, jx, jy);
            yd = make_tap<real>(g, sp, SI, 7 + 3 * sy + 2, base, p, jx, jy);
        }
        double A0 = 0, Az = 0, Azz = 0;
        for (int jz = z0; jz < z1; ++jz) {
            const long long zo = (long long)jz * g.npl;
            const real u0 = tc.eval(jz, zo);
            real r = u0 - flux_diff<real>(xa.eval(jz, zo), xb.eval(jz, zo), u0, xd.eval(jz, zo), Cx, kx);
            if constexpr (DIM == 2)
                r -= flux_diff<real>(ya.eval(jz, zo), yb.eval(jz, zo), u0, yd.eval(jz, zo), Cy, ky);
            out[zo + p] = r;
            const double hd = (double)r, vz = vnode(g, 2, jz);
            A0 += hd;
            Az += vz * hd;
            Azz += vz * vz * hd;
        }
        fold_column(acc, vx, vy, A0, Az, Azz);
    }
    block_sum_store<NQ>(acc, partial + (long long)L * NQ);
}

// ---------------------------------------------------------------- final
// Pointwise f = R2(h) from the cell's own entry (MODE_FINAL tables).
template <typename real>
__global__ void __launch_bounds__(256) k_final(Args A, const real *src, real *dst, const real *__restrict__ params)
{
    const Geo &g = A.g;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int gc = L / A.vsplit, split = L % A.vsplit;
    const int ii = find_inst(A.cell_prefix, A.ninst, gc);
    const Inst &I = A.inst[ii];
    const long long off = I.f0 + (long long)(gc - I.cell0) * g.nv;
    const real *E = params + (long long)gc * g.pe;
    const int z0 = split * g.nvz / A.vsplit, z1 = (split + 1) * g.nvz / A.vsplit;
    const real c0 = E[0];
    for (int p = threadIdx.x; p < g.npl; p += blockDim.x) {
        const int jx = p % g.nvx, jy = p / g.nvx;
        const real l1 = E[g.tx1 + jx] * E[g.ty1 + jy];
        const real l2 = E[g.tx2 + jx] * E[g.ty2 + jy];
        for (int jz = z0; jz < z1; ++jz) {
            const long long i = off + (long long)jz * g.npl + p;
            dst[i] = c0 * src[i] + (l1 * E[g.tz + 2 * jz] + l2 * E[g.tz + 2 * jz + 1]);
        }
    }
}

// ---------------------------------------------------------------- initial state
template <typename real>
__global__ void __launch_bounds__(256) k_init(Args A, real *__restrict__ f)
{
    const Geo &g = A.g;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int gc = L / A.vsplit, split = L % A.vsplit;
    const int ii = find_inst(A.cell_prefix, A.ninst, gc);
    const Inst &I = A.inst[ii];
    const int c = gc - I.cell0;
    double n = 1.0, V = 0.0, T = 1.0;
    if (I.kind == KIND_SHOCK) {
        // Sec. 4.1: upstream state for x < 0, downstream state for x >= 0.
        const double x = I.x0 + (c + 0.5) * I.dx;
        const double *st = x < 0.0 ? I.up : I.dn;
        n = st[0]; V = st[1]; T = st[2];
    }
    const double P = n * pow(M_PI * T, -1.5);
    const long long off = I.f0 + (long long)c * g.nv;
    const int z0 = split * g.nvz / A.vsplit, z1 = (split + 1) * g.nvz / A.vsplit;
    for (int p = threadIdx.x; p < g.npl; p += blockDim.x) {
        const int jx = p % g.nvx, jy = p / g.nvx;
        const double dx = vnode(g, 0, jx) - V, vy = vnode(g, 1, jy);
        for (int jz = z0; jz < z1; ++jz) {
            const double vz = vnode(g, 2, jz);
            f[off + (long long)jz * g.npl + p] = (real)(P * exp(-(dx * dx + vy * vy + vz * vz) / T));
        }
    }
}

}  // namespace bgk
