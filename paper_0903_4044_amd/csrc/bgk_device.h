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

#include <type_traits>

namespace bgk {

constexpr int NVMAX = 128;        // per velocity component
constexpr int KIND_SHOCK = 0, KIND_CAVITY = 1, KIND_PER1 = 2, KIND_PER2 = 3, KIND_CAV3 = 4, KIND_PER3 = 5;
constexpr int MODE_FIRST = 0, MODE_MID = 1, MODE_FINAL = 2;
// moment sums per cell: 1, vx, vy, vz, |v|^2, and the half-range fluxes
// sum_{v_a < 0} |v_a| f, sum_{v_a > 0} v_a f of x (5, 6), y (7, 8), z (9, 10)
constexpr int NQ = 11;

struct Inst {
    int kind, nx, ny, nz, ncell;
    int cell0;      // first global cell index of the instance
    int pseudo0;    // first global params entry of its ghost sources
    int strang, minmod;
    int shift;      // translation form of the streaming step (k_shift)
    int conservative;  // relaxations use the effective Maxwellian parameters
    long long f0;   // element offset of the instance in f
    double cx, cy, cz;  // dt / dx, dt / dy, dt / dz
    double dt, kn, omega;
    double tw, uw;  // wall temperature, lid speed
    double x0, dx;  // spatial origin and cell size along x
    double up[3], dn[3];  // shock far-field (n, V, T)
    // translation-form streaming in row tiles: first tile of the instance,
    // and the sources' reach below and above a tile (cells, with a margin)
    int tile0, reach_lo, reach_hi;
};

// Streaming directions of an instance.
__device__ __forceinline__ int inst_dim(const Inst &I)
{
    return I.kind == KIND_CAV3 || I.kind == KIND_PER3 ? 3 : I.kind == KIND_CAVITY || I.kind == KIND_PER2 ? 2 : 1;
}

struct Geo {
    int nvx, nvy, nvz;
    int npl;                    // nvx * nvy
    long long nv;               // nvx * nvy * nvz
    double lo[3], dv[3];
    double dV;
    int red;                    // components integrated out: 1 v_z (2D kinds), 2 v_y and v_z (1D kinds)
    int zneg;                   // planes with v_z < 0 (they come first)
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
    int zr;                     // jz residues per streaming workgroup (lane tasks)
    int nparts;                 // partial moment sums per cell that consumers add up
    int ntiles;                 // row-tile translation streaming: tiles over all instances
    uint32_t *pass;             // rounding counter: advanced once per streaming pass
    unsigned char *rec;         // branch record of a recording streaming pass (else unused)
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

// Visiting order of the cells of one instance for the stencil kernels.  The
// columns of a 2D instance are cut into strips STRIP cells wide and each
// strip is walked row by row, so the cells in flight on one XCD and their
// y-neighbours (two rows either side) span a few strip widths of the visiting
// order and stay in that XCD's L2; row-major order would put the y-neighbours
// nx cells away and fetch every row from HBM several times.  1D instances
// (ny = 1) map to themselves.  Returns the instance-local cell of position q.
constexpr int STRIP = 16;

__device__ __forceinline__ int strip_cell(const Inst &I, int q)
{
    // 3D instances: the planes iz one after the other, each walked in strips
    const int pl = I.nx * I.ny, iz = q / pl;
    q -= iz * pl;
    const int W = I.nx < STRIP ? I.nx : STRIP;
    const int span = W * I.ny;
    const int nfull = I.nx / W;
    if (q < nfull * span) {
        const int k = q / span, r = q - k * span;
        const int iy = r / W;
        return iz * pl + iy * I.nx + k * W + (r - iy * W);
    }
    const int rem = I.nx - nfull * W;
    const int r = q - nfull * span;
    const int iy = r / rem;
    return iz * pl + iy * I.nx + nfull * W + (r - iy * rem);
}

// Order of the streaming kernel's (cell, jz chunk) items: superblocks of
// SUPER cells in the visiting order, each walked chunk by chunk.  The items
// in flight on one XCD are then one chunk of up to about SUPER consecutive
// cells, and the cells their stencils reach (two rows either side in the
// strip order) are the same chunk of nearby cells: a working set of one
// chunk per cell, where walking all chunks of a cell together would keep
// every chunk of all those cells in the XCD's L2 at once.
constexpr int SUPER = 128;

__device__ __forceinline__ void item_cell_chunk(int L, int ncells, int vsplit, int *cell, int *split)
{
    const int sb = L / (SUPER * vsplit), c0 = sb * SUPER;
    const int n = min(SUPER, ncells - c0), k = L - c0 * vsplit;
    *split = k / n;
    *cell = c0 + (k - *split * n);
}

__device__ __forceinline__ double vnode(const Geo &g, int a, int k) { return g.lo[a] + (k + 0.5) * g.dv[a]; }

// The jz planes [z0, z1) of chunk `split` of `vsplit`: chunks start on even
// planes (pairs of planes share one rounding hash), the last chunk takes an
// odd last plane.
__device__ __forceinline__ void chunk_bounds(int nvz, int vsplit, int split, int *z0, int *z1)
{
    const int npair = nvz >> 1;
    *z0 = 2 * (split * npair / vsplit);
    *z1 = split == vsplit - 1 ? nvz : 2 * ((split + 1) * npair / vsplit);
}

// The v_z axis.  Full velocity space: nodes v_z(k).  Reduced velocity space
// (the projection the paper cites in Sec. 3 and Sec. 6): the components a
// problem does not stream along are integrated out, v_z for two-dimensional
// problems (plane 0 holds g = int f dv_z, plane 1 h = int v_z^2 f dv_z) and
// v_y, v_z for one-dimensional ones (g = int f dv_y dv_z, h = int (v_y^2 +
// v_z^2) f dv_y dv_z, and the v_y axis is the single node v_y = 0), so V = 0
// along them and the integrals of Eq. (Maxw) are exact.  Per plane: its
// share m in mass and momentum, its v_z and its energy term zz beyond
// m |v|^2: (1, v_z, v_z^2) in full velocity space, (1, 0, 0) for g and
// (0, 0, 1) for h.
struct ZW { double m, z, zz; };

__device__ __forceinline__ ZW zweights(const Geo &g, int k)
{
    if (g.red) return k == 0 ? ZW{1.0, 0.0, 0.0} : ZW{0.0, 0.0, 1.0};
    const double vz = vnode(g, 2, k);
    return ZW{1.0, vz, vz * vz};
}

// The Maxwellian's factor on plane k: exp(-(v_z - V_z)^2 / T), or in reduced
// velocity space the integrals over the components out: sqrt(pi T) (g) and
// (T / 2) sqrt(pi T) (h) over v_z; pi T (g) and pi T^2 (h) over v_y, v_z.
__device__ __forceinline__ double zfactor(const Geo &g, int k, double Vz, double T)
{
    if (g.red == 2) return k == 0 ? M_PI * T : M_PI * T * T;
    if (g.red) {
        const double s = sqrt(M_PI * T);
        return k == 0 ? s : 0.5 * T * s;
    }
    const double d = vnode(g, 2, k) - Vz;
    return exp(-d * d / T);
}

__device__ __forceinline__ float minmod3(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }

// ---------------------------------------------------------------- rounding
// FP32 storage of f rounds each stored value stochastically: up or down to
// a neighbouring float with probabilities that make the rounding unbiased.
// Round-to-nearest would stall a near-equilibrium region: the change of f
// per step there is far below half an ulp, so every step rounds back to the
// same float and the slow drift of the FP64 dynamics is lost.  The random
// bits come from a counter-based hash of (element index within its
// instance, streaming pass), so they do not depend on launch shape or
// batching, and a run repeats exactly for the same rounding seed.

// 32-bit integer hash ("lowbias32", C. Wellons, Prospecting for Hash
// Functions, 2018): xorshift-multiply rounds with constants 0x7feb352d and
// 0x846ca68b.
__device__ __forceinline__ uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Key of one rounding pass; `stream` separates the streaming kernel (0) from
// the closing relaxation (1).
__device__ __forceinline__ uint32_t pass_key(const uint32_t *pass, uint32_t stream)
{
    return hash32(*pass * 2u + stream + 0x9e3779b9u);
}

// Stochastic rounding of x to float with 16 random bits r16, placed at the
// top of the 29 bits below the float's last mantissa bit (the lower 13 bits
// truncate: a bias under 2^-16 ulp).  One 32-bit hash serves two elements.
__device__ __forceinline__ float round_stochastic16(double x, uint32_t r16)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    b += (unsigned long long)r16 << 13;
    b &= ~((1ull << 29) - 1ull);
    return (float)__longlong_as_double((long long)b);
}

// Stochastic rounding of x to float: add 29 uniform bits below the float's
// last mantissa bit of |x| and truncate (sign-magnitude, so the magnitude
// rounds away from zero with probability equal to the dropped fraction).
__device__ __forceinline__ float round_stochastic(double x, uint32_t r)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    b += (unsigned long long)(r >> 3);
    b &= ~((1ull << 29) - 1ull);
    return (float)__longlong_as_double((long long)b);
}
__device__ __forceinline__ double minmod3(double a, double b) { return fmax(fmin(a, b), fmin(fmax(a, b), 0.0)); }

// Branch of a limited slope minmod(a, b), read off the limiter's own value
// m = median(a, b, 0): 0 when m = 0 (the differences disagree in sign or one
// is zero), 2 when m equals b (b the smaller magnitude, ties included), else
// 1 (a).  The reverse sweep differentiates the slope on this branch.
template <typename real>
__device__ __forceinline__ uint32_t mm_code(real a, real b)
{
    const real m = minmod3(a, b);
    return m == (real)0 ? 0u : (m == b ? 2u : 1u);
}

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
// moment sums: A0 = sum h, Az = sum vz h, Azz = sum vz^2 h, and the z
// half-range fluxes Azm = sum_{vz<0} |vz| h, Azp = sum_{vz>0} vz h.
__device__ __forceinline__ void fold_column(double (&acc)[NQ], double vx, double vy, double A0, double Az, double Azz,
                                            double Azm = 0.0, double Azp = 0.0)
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
    acc[9] += Azm;
    acc[10] += Azp;
}

// The same fold into this thread's slots of the workgroup's LDS accumulators
// (acc[q * stride]): the nine sums do not occupy registers across a task.
// The sums pass through fold_column itself, so the arithmetic (and its
// rounding) is that of the register form.
// NS: the sums kept (9 without the z half fluxes, 11 with them).
template <int NS = NQ>
__device__ __forceinline__ void fold_column_lds(double *acc, int stride, double vx, double vy, double A0, double Az,
                                                double Azz, double Azm = 0.0, double Azp = 0.0)
{
    double t[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) t[q] = q < NS ? acc[q * stride] : 0.0;
    fold_column(t, vx, vy, A0, Az, Azz, Azm, Azp);
#pragma unroll
    for (int q = 0; q < NS; ++q) acc[q * stride] = t[q];
}

template <typename T, int N>
using vec_t = T __attribute__((ext_vector_type(N)));

// Byte-offset load/store from a uniform base (SGPR base + 32-bit VGPR offset).
template <typename V>
__device__ __forceinline__ V ld(const void *base, uint32_t off)
{
    return *reinterpret_cast<const V *>(reinterpret_cast<const char *>(base) + off);
}

// Buffer loads: a descriptor (base, byte size) in scalar registers, a 32-bit
// per-lane byte offset and a wave-uniform byte offset added by the load
// itself, so no vector instruction forms a 64-bit address.  Reads past the
// size return zero instead of faulting.  Third descriptor word of this ISA
// family for raw (unformatted, stride 0) buffers.
constexpr int BUF_WORD3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    // The descriptor must sit in scalar registers (a descriptor the compiler
    // takes for divergent costs a loop per load); its inputs are wave-uniform,
    // and readfirstlane says so.
    const uint64_t a = (uint64_t)(uintptr_t)base;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    void *p = (void *)(uintptr_t)(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), BUF_WORD3);
}

template <typename V>
__device__ __forceinline__ V buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(V) == 4)
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    else if constexpr (sizeof(V) == 8)
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    else
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}

// ---------------------------------------------------------------- moments
// Partial moment sums of f over one jz chunk of one cell:
// partial[(cell * nparts + split) * NQ + q] (without the dV factor).  Each
// lane reads VEC consecutive jx at one jy (16-byte loads where the grid
// allows) down its jz chunk.
template <typename real, int VEC>
__global__ void __launch_bounds__(256) k_moments(Args A, const real *__restrict__ f, double *__restrict__ partial)
{
    using V = vec_t<real, VEC>;
    const Geo &g = A.g;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int gc = L / A.vsplit, split = L % A.vsplit;
    const int ii = find_inst(A.cell_prefix, A.ninst, gc);
    const Inst &I = A.inst[ii];
    const real *fc = f + I.f0 + (long long)(gc - I.cell0) * g.nv;
    int z0, z1;
    chunk_bounds(g.nvz, A.vsplit, split, &z0, &z1);
    const int ngrp = g.npl / VEC;
    double acc[NQ] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int q = threadIdx.x; q < ngrp; q += blockDim.x) {
        const int p0 = q * VEC, jx0 = p0 % g.nvx, jy = p0 / g.nvx;
        double A0[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) A0[e] = 0.0;
        double Az = 0, Azz = 0, Azm = 0, Azp = 0;
#pragma unroll 4
        for (int jz = z0; jz < z1; ++jz) {
            const V h = ld<V>(fc, (uint32_t)((jz * g.npl + p0) * (int)sizeof(real)));
            const ZW w = zweights(g, jz);
            double sh = 0.0;
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const double he = (double)h[e];
                A0[e] = __builtin_fma(w.m, he, A0[e]);
                sh += he;
            }
            Az += w.z * sh;
            Azz += w.zz * sh;
            if (w.z < 0.0) Azm -= w.z * sh;
            else Azp += w.z * sh;
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            fold_column(acc, vnode(g, 0, jx0 + e), vnode(g, 1, jy), A0[e], e == 0 ? Az : 0.0, e == 0 ? Azz : 0.0,
                        e == 0 ? Azm : 0.0, e == 0 ? Azp : 0.0);
    }
    // slot (cell, split) of the A.nparts per cell the consumers add up; a
    // launch with fewer chunks than slots zeroes the remaining ones
    block_sum_store<NQ>(acc, partial + ((long long)gc * A.nparts + split) * NQ);
    if (split == 0)
        for (int t = threadIdx.x; t < (A.nparts - A.vsplit) * NQ; t += blockDim.x)
            partial[((long long)gc * A.nparts + A.vsplit) * NQ + t] = 0.0;
}

// Per-cell macroscopic moments (n, Vx, Vy, Vz, T) from the partial sums.
__global__ void k_macro(Args A, const double *__restrict__ partial, double *__restrict__ mom)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= A.ncells) return;
    double s[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < A.nparts; ++k)
        for (int q = 0; q < 5; ++q) s[q] += partial[((long long)c * A.nparts + k) * NQ + q];
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
// One wave per table entry, four entries per 256-thread workgroup.  Each lane
// owns slots k = lane and k = lane + 64 of the 1D tables of every velocity
// component; the 1D sums the relaxations need are butterfly wave reductions,
// so the whole computation stays in registers (no LDS, no block barrier).

// Relaxation times of the relaxations folded into a table entry.
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

struct Relax {          // one relaxation: moments (n, V, T) of its input, a, and
    double n, V[3], T, a;  // the Maxwellian P e_x e_y e_z, e_c = exp(-(v_c - Vm_c)^2 / Tm)
    double P, Vm[3], Tm;   // (Vm, Tm = V, T unless the effective parameters are used)
};

__device__ __forceinline__ void moments_from_raw(const double *raw, Relax *r)
{
    r->n = raw[0];
    r->V[0] = raw[1] / raw[0];
    r->V[1] = raw[2] / raw[0];
    r->V[2] = raw[3] / raw[0];
    r->T = 2.0 / 3.0 * (raw[4] / raw[0] - (r->V[0] * r->V[0] + r->V[1] * r->V[1] + r->V[2] * r->V[2]));
    for (int c = 0; c < 3; ++c) r->Vm[c] = r->V[c];
    r->Tm = r->T;
}

// (pi T)^(-3/2) as a square root and a division (no pow).
__device__ __forceinline__ double pi_t_m32(double T)
{
    const double pt = M_PI * T;
    return 1.0 / (pt * sqrt(pt));
}

__device__ __forceinline__ void finish_relax(const Inst &I, double tau, Relax *r)
{
    // T^(1 - omega): a square root for omega = 1/2 (every workload), pow otherwise
    const double tp = I.omega == 0.5 ? sqrt(r->T) : pow(r->T, 1.0 - I.omega);
    const double nu = r->n * tp / I.kn;
    r->a = -expm1(-nu * tau);
    r->P = r->n * pi_t_m32(r->T);
}

// A double from another lane of the same 16-lane row (DPP move of both halves).
template <int CTRL>
__device__ __forceinline__ double dpp_double(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// A double from lane (this lane xor 16) within its 32-lane half (swizzle).
__device__ __forceinline__ double swizzle_xor16(double x)
{
    constexpr int PAT = 0x1F | (0x10 << 10);  // bit mode: and 0x1F, or 0, xor 0x10
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_ds_swizzle((int)b, PAT);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), PAT);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the W-lane segment of the wave that holds this lane.  Pairs of
// lanes exchange partial sums and add them, so every lane of the segment
// ends with the same bits: swaps within quads (DPP quad permutations), then
// quads (half-row mirror) and half rows (row mirror) of a 16-lane row, then
// rows through a swizzle and across the two halves through a permute.  Lanes
// beyond a segment's data hold zeros, so a segment's sum equals that of a
// wider one.
template <int W = 64>
__device__ __forceinline__ double wave_sum(double x)
{
    static_assert(W == 16 || W == 32 || W == 64, "segments of 16, 32 or 64 lanes");
    x += dpp_double<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dpp_double<0x4E>(x);   // quad_perm [2,3,0,1]
    x += dpp_double<0x141>(x);  // row_half_mirror
    x += dpp_double<0x140>(x);  // row_mirror
    if constexpr (W >= 32) x += swizzle_xor16(x);
    if constexpr (W == 64) x += __shfl_xor(x, 32, 64);
    return x;
}

__device__ __forceinline__ int nv_of(const Geo &g, int a) { return a == 0 ? g.nvx : (a == 1 ? g.nvy : g.nvz); }

// This lane's slots of e_a(k) = exp(-(v_a(k) - V_a)^2 / T).
struct Tables {
    double e[3][2];
};

template <int W = 64>
__device__ __forceinline__ void lane_tables(const Geo &g, const double V[3], double T, Tables &t)
{
    const int lane = threadIdx.x & (W - 1);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int k = lane + W * s;
            t.e[a][s] = 0.0;
            if (W * s >= nv_of(g, a)) continue;  // uniform: no second slot up to W points
            if (k >= nv_of(g, a)) continue;
            if (a == 2) {
                t.e[a][s] = zfactor(g, k, V[a], T);
            } else {
                const double d = vnode(g, a, k) - V[a];
                t.e[a][s] = exp(-d * d / T);
            }
        }
}

__device__ __forceinline__ void zero_tables(Tables &t)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) t.e[a][0] = t.e[a][1] = 0.0;
}

// Wave-reduced 1D sums of a table: s[a][0] = sum e, s[a][1] = sum v e,
// s[a][2] = sum v^2 e, s[a][3] = sum_{v<0} |v| e, s[a][4] = sum_{v>0} v e.
template <int W = 64>
__device__ __forceinline__ void wave_table_sums(const Geo &g, const Tables &t, double (*s)[5], bool half)
{
    const int lane = threadIdx.x & (W - 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double s0 = 0, s1 = 0, s2 = 0, sm = 0, sp = 0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double x = t.e[a][q];
            if (a == 2) {
                const ZW w = zweights(g, lane + W * q);
                s0 += w.m * x;
                s1 += w.z * x;
                s2 += w.zz * x;
                if (w.z < 0.0) sm += -w.z * x;
                else sp += w.z * x;
                continue;
            }
            const double v = vnode(g, a, lane + W * q);
            s0 += x;
            s1 += v * x;
            s2 += v * v * x;
            if (v < 0.0) sm += -v * x;
            else sp += v * x;
        }
        s[a][0] = wave_sum<W>(s0);
        s[a][1] = wave_sum<W>(s1);
        s[a][2] = wave_sum<W>(s2);
        if (half) {
            s[a][3] = wave_sum<W>(sm);
            s[a][4] = wave_sum<W>(sp);
        }
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

// Effective Maxwellian parameters (Sec. 2.1, the remark on conservation after
// Eq. (exact)): the (n~, V~, T~) whose discretized Maxwellian has exactly the
// grid moments (n, V, T) of the cell, so that the relaxation conserves mass,
// momentum and energy on the velocity grid.  The Maxwellian factorises, so
// with u = v_c - V~_c and e_c(u) = exp(-u^2 / T~) per component c and the
// normalised power sums  m_k = sum u^k e_c / sum e_c  (k = 1..4), the grid
// mean of v_c is V~_c + m_1 and its grid variance c2 = m_2 - m_1^2; the
// temperature condition couples the components: (2/3) sum_c c2_c = T.
// Newton's method on (V~, T~), started at (V, T), with the exact Jacobian
// (derivatives of weighted means by the score 2u/T~ resp. u^2/T~^2):
//   d mean_c / d V~_c = 2 c2_c / T~,     d mean_c / d T~ = (m_3 - m_1 m_2)_c / T~^2,
//   d c2_c / d V~_c   = 2 c3_c / T~,     d c2_c / d T~   = (c4 - c2^2 + 2 m_1 c3)_c / T~^2,
// c3, c4 being the central moments.  The 4x4 system has arrowhead form and is
// solved in closed form.  It stops after the first step that changes no
// parameter by more than 1e-14 of its scale (sqrt(T~), T~), or after 30.
// Then n~ needs no iteration: the grid density is linear in it, and the
// prefactor  P = n~ (pi T~)^(-3/2) = n / (dV prod_c sum e_c).  The final
// pass fills this lane's table slots with the e_c of the result.  All sums
// are butterflies inside the W-lane segment, so every lane holds the same
// values and the loop is uniform over the segment.
template <int W = 64>
__device__ __forceinline__ void effective_tables(const Geo &g, Relax *r, Tables &t)
{
    const int lane = threadIdx.x & (W - 1);
    double Vt[3] = {r->V[0], r->V[1], r->V[2]}, Tt = r->T;
    bool done = false;
    for (int it = 0;; ++it) {
        double res[3], jvv[3], jvt[3], jtv[3], jtt = 0.0, rt = -r->T, s0[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if ((c == 2 && g.red) || (c == 1 && g.red == 2)) {
                // reduced velocity space: V = 0 along the components out is no
                // unknown; h = (T~ / 2) g (v_z out) or h = T~ g (v_y, v_z out)
                // on every node, so their share of the temperature is exact;
                // a v_y axis taken out is the single node v_y = 0 (factor 1)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int k = lane + W * q;
                    t.e[c][q] = c == 1 ? (k == 0 ? 1.0 : 0.0) : (k < 2 ? zfactor(g, k, 0.0, Tt) : 0.0);
                }
                s0[c] = c == 1 ? 1.0 : zfactor(g, 0, 0.0, Tt);
                if (done) continue;
                res[c] = 0.0;
                jvv[c] = 1.0;
                jvt[c] = 0.0;
                jtv[c] = 0.0;
                if (c == 2) {
                    const double share = g.red == 2 ? 1.0 : 0.5;  // (h / g) / T~
                    jtt += 2.0 / 3.0 * share;
                    rt += 2.0 / 3.0 * share * Tt;
                }
                continue;
            }
            double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0, p4 = 0.0;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int k = lane + W * q;
                t.e[c][q] = 0.0;
                if (W * q >= nv_of(g, c)) continue;  // uniform: no second slot up to W points
                if (k < nv_of(g, c)) {
                    const double u = vnode(g, c, k) - Vt[c], u2 = u * u;
                    const double e = exp(-u2 / Tt);
                    t.e[c][q] = e;
                    p0 += e;
                    p1 += u * e;
                    p2 += u2 * e;
                    p3 += u2 * u * e;
                    p4 += u2 * u2 * e;
                }
            }
            s0[c] = wave_sum<W>(p0);
            if (done) continue;
            const double i0 = 1.0 / s0[c];
            const double a1 = wave_sum<W>(p1) * i0, a2 = wave_sum<W>(p2) * i0;
            const double a3 = wave_sum<W>(p3) * i0, a4 = wave_sum<W>(p4) * i0;
            const double c2 = a2 - a1 * a1;
            const double c3 = a3 - 3.0 * a1 * a2 + 2.0 * a1 * a1 * a1;
            const double c4 = a4 - 4.0 * a1 * a3 + 6.0 * a1 * a1 * a2 - 3.0 * a1 * a1 * a1 * a1;
            res[c] = Vt[c] + a1 - r->V[c];
            jvv[c] = 2.0 * c2 / Tt;
            jvt[c] = (a3 - a1 * a2) / (Tt * Tt);
            jtv[c] = 4.0 / 3.0 * c3 / Tt;
            jtt += 2.0 / 3.0 * (c4 - c2 * c2 + 2.0 * a1 * c3) / (Tt * Tt);
            rt += 2.0 / 3.0 * c2;
        }
        if (done) {
            r->P = r->n / (g.dV * s0[0] * s0[1] * s0[2]);
            break;
        }
        double num = rt, den = jtt;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            num -= jtv[c] * res[c] / jvv[c];
            den -= jtv[c] * jvt[c] / jvv[c];
        }
        const double dT = num / den;
        bool small = fabs(dT) <= 1e-14 * Tt;
        const double vs = sqrt(Tt);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double dV = (res[c] - jvt[c] * dT) / jvv[c];
            Vt[c] -= dV;
            small = small && fabs(dV) <= 1e-14 * vs;
        }
        Tt = fmax(Tt - dT, 0.5 * Tt);  // a step may not more than halve T~
        done = small || it == 29;
    }
    for (int c = 0; c < 3; ++c) r->Vm[c] = Vt[c];
    r->Tm = Tt;
}

// Everything one wave knows about the relaxations of one cell.
struct Coef {
    double raw[NQ];     // moment sums (with dV) of the cell's input
    Relax r1, r2;       // r1 applied first, r2 second
    double c0, cA, cB;  // g = c0 h + cA e1 + cB e2 (cA, cB include a and P)
    int nr;
    Tables t1, t2;
    double s1[3][5], s2[3][5];
};

// Coefficients of the relaxations folded into one cell's entry, from that
// cell's partial moment sums (A.nparts per cell).  Wave-uniform control flow.
template <int W = 64, bool CONS = true>
__device__ __forceinline__ void cell_coefficients(const Args &A, const Inst &I, int gc, int mode,
                                                  const double *partial, Coef &C, bool want_sums)
{
    const Geo &g = A.g;
    const int lane = threadIdx.x & (W - 1);
    double mine = 0.0;
    if (lane < NQ)
        for (int k = 0; k < A.nparts; ++k) mine += partial[((long long)gc * A.nparts + k) * NQ + lane];
#pragma unroll
    for (int q = 0; q < NQ; ++q) C.raw[q] = __shfl(mine, q, W) * g.dV;
    double ta, tb;
    C.nr = relax_times(I, mode, &ta, &tb);
    C.c0 = 1.0;
    C.cA = C.cB = 0.0;
    zero_tables(C.t1);
    zero_tables(C.t2);
    if (C.nr == 0) return;
    moments_from_raw(C.raw, &C.r1);
    finish_relax(I, ta, &C.r1);
    // CONS = false: no conservative instance in the launch (the point form
    // alone, far fewer registers)
    const bool cons = CONS && I.conservative;
    if (cons) effective_tables<W>(g, &C.r1, C.t1);
    else lane_tables<W>(g, C.r1.V, C.r1.T, C.t1);
    if ((C.nr == 2 && !cons) || want_sums) wave_table_sums<W>(g, C.t1, C.s1, want_sums);
    if (C.nr == 2 && cons) {
        // R1 keeps the grid moments, so R2 relaxes towards the same Maxwellian
        C.r2 = C.r1;
        finish_relax(I, tb, &C.r2);
        C.r2.P = C.r1.P;
        C.t2 = C.t1;
        if (want_sums)
            for (int c = 0; c < 3; ++c)
                for (int q = 0; q < 5; ++q) C.s2[c][q] = C.s1[c][q];
    } else if (C.nr == 2) {
        double mp[5], m2[5];
        maxwell_raw(C.r1.P, g.dV, C.s1, mp);
        for (int q = 0; q < 5; ++q) m2[q] = C.r1.a * mp[q] + (1.0 - C.r1.a) * C.raw[q];
        moments_from_raw(m2, &C.r2);
        finish_relax(I, tb, &C.r2);
        lane_tables<W>(g, C.r2.V, C.r2.T, C.t2);
        if (want_sums) wave_table_sums<W>(g, C.t2, C.s2, true);
    }
    if (C.nr == 2) {
        C.c0 = (1.0 - C.r1.a) * (1.0 - C.r2.a);
        C.cA = C.r1.a * (1.0 - C.r2.a) * C.r1.P;
        C.cB = C.r2.a * C.r2.P;
    } else {
        C.c0 = 1.0 - C.r1.a;
        C.cA = C.r1.a * C.r1.P;
    }
}

// Write one entry: c0, TX1 = cA eA_x, TY1 = eA_y, TX2 = cB eB_x, TY2 = eB_y,
// TZ = (eA_z, eB_z) interleaved.
template <typename real, int W = 64>
__device__ __forceinline__ void write_entry(const Geo &g, real *E, double c0, double cA, const Tables &tA, double cB,
                                            const Tables &tB)
{
    const int lane = threadIdx.x & (W - 1);
    if (lane == 0) {
        E[0] = (real)c0;
        // float entries also keep c0 in double (slots 2-3, 8-byte aligned): the
        // centre value's relaxation uses it, since c0 rounded to float would
        // gain or lose that rounding error of mass at every relaxation
        if constexpr (sizeof(real) == 4) *reinterpret_cast<double *>(E + 2) = c0;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int k = lane + W * q;
        if (k < g.nvx) {
            E[g.tx1 + k] = (real)(cA * tA.e[0][q]);
            E[g.tx2 + k] = (real)(cB * tB.e[0][q]);
        }
        if (k < g.nvy) {
            E[g.ty1 + k] = (real)tA.e[1][q];
            E[g.ty2 + k] = (real)tB.e[1][q];
        }
        if (k < g.nvz) {
            E[g.tz + 2 * k] = (real)tA.e[2][q];
            E[g.tz + 2 * k + 1] = (real)tB.e[2][q];
        }
    }
}

// Wall geometry: wall w = 0 left (+x inward), 1 right (-x), 2 bottom (+y),
// 3 top (-y), and for 3D instances 4 back (+z), 5 front (-z): wall w lies
// across axis w / 2, on the low side for even w.  The wall entries of an
// instance come wall by wall; within wall w the face cells are numbered by
// the other two coordinates, the lower axis fastest: (iy, iz) for x walls,
// (ix, iz) for y walls, (ix, iy) for z walls.
__device__ __forceinline__ int wall_size(const Inst &I, int w)
{
    return w < 2 ? I.ny * I.nz : w < 4 ? I.nx * I.nz : I.nx * I.ny;
}

__device__ __forceinline__ int wall_of_entry(const Inst &I, int k, int *pos)
{
    int w = 0;
    while (w < 5 && k >= wall_size(I, w)) k -= wall_size(I, w++);
    *pos = k;
    return w;
}

// First entry of wall w within the instance's wall entries.
__device__ __forceinline__ int wall_offset(const Inst &I, int w)
{
    int o = 0;
    for (int v = 0; v < w; ++v) o += wall_size(I, v);
    return o;
}

// Instance-local cell next to position pos of wall w.
__device__ __forceinline__ int wall_cell(const Inst &I, int w, int pos)
{
    const int axis = w >> 1;
    const bool low = (w & 1) == 0;
    if (axis == 0) {
        const int iy = pos % I.ny, iz = pos / I.ny;
        return (iz * I.ny + iy) * I.nx + (low ? 0 : I.nx - 1);
    }
    if (axis == 1) {
        const int ix = pos % I.nx, iz = pos / I.nx;
        return (iz * I.ny + (low ? 0 : I.ny - 1)) * I.nx + ix;
    }
    const int ix = pos % I.nx, iy = pos / I.nx;
    return ((low ? 0 : I.nz - 1) * I.ny + iy) * I.nx + ix;
}

// Table entry of cell e, computed by the calling W-lane segment from the
// partial moment sums of the streaming input.
template <typename real, int W, bool CONS>
__device__ __forceinline__ void prep_cell(const Args &A, int e, int mode, const double *partial, real *params)
{
    const Geo &g = A.g;
    real *E = params + (long long)e * g.pe;
    Coef C;
    const int ii = find_inst(A.cell_prefix, A.ninst, e);
    cell_coefficients<W, CONS>(A, A.inst[ii], e, mode, partial, C, false);
    write_entry<real, W>(g, E, C.c0, C.cA, C.t1, C.cB, C.t2);
}

// Table entry e >= ncells (a ghost source), likewise.
template <typename real, int W, bool CONS>
__device__ __forceinline__ void prep_ghost(const Args &A, int e, int mode, const double *partial, real *params)
{
    const Geo &g = A.g;
    real *E = params + (long long)e * g.pe;
    Coef C;
    // ghost sources
    const int pe = e - A.ncells;
    const int ii = find_inst(A.pseudo_prefix, A.ninst, pe);
    const Inst &I = A.inst[ii];
    const int k = pe - A.pseudo_prefix[ii];
    Tables z;
    zero_tables(z);
    if (I.kind == KIND_SHOCK) {
        // Far-field Maxwellian of Eq. (bc_shock): k = 0 upstream (x < x0), 1 downstream.
        const double *st = k == 0 ? I.up : I.dn;
        const double V[3] = {st[1], 0.0, 0.0};
        Tables t;
        lane_tables<W>(g, V, st[2], t);
        write_entry<real, W>(g, E, 0.0, st[0] * pi_t_m32(st[2]), t, 0.0, z);
        return;
    }
    // Diffuse wall face, Eq. (bc_cavity): ghost = n_W Phi_W for velocities
    // leaving the wall.  n_W makes the discrete net mass flux zero:
    //   n_W = sum_{v.n<0} |v.n| g0 / sum_{v.n>0} v.n Phi_W,
    // g0 being the wall-adjacent cell of the streaming input, g0 = c0 h + cA e1 + cB e2.
    int pos;
    const int w = wall_of_entry(I, k, &pos);
    const int axis = w >> 1;
    const int adj = wall_cell(I, w, pos);
    cell_coefficients<W, CONS>(A, I, I.cell0 + adj, mode, partial, C, true);
    const double VW[3] = {w == 3 ? I.uw : 0.0, 0.0, 0.0};
    Tables tw;
    lane_tables<W>(g, VW, I.tw, tw);
    double sw[3][5];
    wave_table_sums<W>(g, tw, sw, true);
    const int b1 = axis == 0 ? 1 : 0, b2 = axis == 2 ? 1 : 2;  // the two other components
    // incident: v_axis < 0 for the low walls (sum index 3), v_axis > 0 for the high ones (index 4)
    const bool lowwall = (w & 1) == 0;
    // (run-time axes blend registers with 0/1 weights, exact for the finite
    // sums here: a select of array elements becomes an indexed access, which
    // puts the whole entry's state in scratch memory)
    auto pick = [](const double (&t)[3][5], int a, int q) {
        return t[0][q] * (double)(a == 0) + t[1][q] * (double)(a == 1) + t[2][q] * (double)(a == 2);
    };
    const double hin1 = lowwall ? pick(C.s1, axis, 3) : pick(C.s1, axis, 4);
    const double hin2 = lowwall ? pick(C.s2, axis, 3) : pick(C.s2, axis, 4);
    const double out_w = lowwall ? pick(sw, axis, 4) : pick(sw, axis, 3);
    const double o1 = pick(C.s1, b1, 0), o2 = pick(C.s2, b1, 0), ow = pick(sw, b1, 0);
    double hraw = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) hraw += C.raw[5 + q] * (double)(w == q);
    double flux = C.c0 * hraw;
    if (C.nr >= 1) flux += C.cA * g.dV * hin1 * o1 * pick(C.s1, b2, 0);
    if (C.nr == 2) flux += C.cB * g.dV * hin2 * o2 * pick(C.s2, b2, 0);
    const double pw = pi_t_m32(I.tw);
    const double den = pw * g.dV * out_w * ow * pick(sw, b2, 0);
    write_entry<real, W>(g, E, 0.0, flux / den * pw, tw, 0.0, z);
    if ((threadIdx.x & (W - 1)) == 1) E[1] = (real)(flux / den);  // n_W, read by the reverse sweep
}

// Table preparation between streaming passes: one W-lane segment per entry,
// 64 / W entries per wave (W = the smallest of 16, 32, 64 that holds the
// largest velocity axis, so few lanes idle on small grids; every sum is a
// butterfly inside the segment, and a segment's results equal those of a
// whole wave with the extra lanes holding zeros).
// The table entries of one preparation: cells (GHOST = false, entries
// [0, ncells)) or ghost sources (GHOST = true, entries [ncells, nentries)),
// two launches, so that the cells' kernel keeps its state in registers (the
// ghost faces index per-axis sums with a run-time axis).
template <typename real, int W, bool GHOST, bool CONS>
__global__ void __launch_bounds__(256) k_prep(Args A, const double *__restrict__ partial, real *__restrict__ params,
                                              int mode, int nentries, real *__restrict__ params_shock_copy)
{
    // Tables of these modes follow a streaming pass: advance the rounding
    // counter once (stream order puts this after that pass's reads).
    if (!GHOST && blockIdx.x == 0 && threadIdx.x == 0 && (mode == MODE_MID || mode == MODE_FINAL))
        A.pass[0] = A.pass[0] + 1u;
    const int e = (GHOST ? A.ncells : 0) + (blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 / W) +
                  (int)((threadIdx.x & 63) / W);
    if (e >= (GHOST ? nentries : A.ncells)) return;  // the whole segment leaves; sums never leave a segment
    if constexpr (!GHOST) {
        prep_cell<real, W, CONS>(A, e, mode, partial, params);
    } else {
        prep_ghost<real, W, CONS>(A, e, mode, partial, params);
        // Far-field entries never change: give the other parity buffer a copy.
        if (params_shock_copy) {
            const int ii = find_inst(A.pseudo_prefix, A.ninst, e - A.ncells);
            if (A.inst[ii].kind == KIND_SHOCK) prep_ghost<real, W, CONS>(A, e, mode, partial, params_shock_copy);
        }
    }
}

// ---------------------------------------------------------------- stream
// One workgroup per (cell, jz chunk).  Thread lanes run over the (jx, jy)
// plane, each lane loops over jz.  Per lane and velocity the upwind stencil
// in each direction is {i - 2s, i - s, i, i + s} with s = sign(v_d); a slot
// table resolves every stencil position (interior cell, periodic image,
// far-field Maxwellian, wall-adjacent cell or emitted wall Maxwellian) once
// per workgroup, so the inner loop is branch-free.  In three dimensions the
// sign of v_z, and with it the z stencil, changes along a lane's jz loop:
// the loop runs in two sweeps, the planes with v_z < 0 and then those with
// v_z > 0, each with the z taps of its sign.
//
// Slots: 0 centre; 1 + 6 d + 3 si + m for direction d (x, y, z), si = 0
// for s = +1, 1 for s = -1; m = 0, 1, 2 for k = -2, -1, +1.
constexpr int MAXSLOT = 19;
struct SlotInfo { int cell[MAXSLOT]; int par[MAXSLOT]; uint32_t off[MAXSLOT]; };  // off: byte offset of the slot cell's h

// The stencil position `delta` cells from cell (ix, iy, iz) along `axis`,
// for velocities whose component along it has sign sgn: the cell whose h is
// read and the table entry that relaxes it.  Inside the instance: that cell.
// Periodic kinds: its image.  Shock: the far-field entry (c0 = 0, so the
// cell read is irrelevant; the own cell).  Walls: for velocities leaving the
// wall, the wall's emitted-Maxwellian entry of the face cell; for velocities
// arriving at it, the wall-adjacent cell itself.
__device__ __forceinline__ void resolve_slot(const Inst &I, int axis, int ix, int iy, int iz, int delta, int sgn,
                                             int own, int *cell, int *par)
{
    // An instance of lower dimension in a batch run at a higher one does not
    // stream along this axis (its Courant number there is 0): its own cell.
    if (axis >= inst_dim(I)) { *cell = own; *par = I.cell0 + own; return; }
    const int N = axis == 0 ? I.nx : axis == 1 ? I.ny : I.nz;
    const int pos = (axis == 0 ? ix : axis == 1 ? iy : iz) + delta;
    auto at = [&](int q) {
        const int x = axis == 0 ? q : ix, y = axis == 1 ? q : iy, z = axis == 2 ? q : iz;
        return (z * I.ny + y) * I.nx + x;
    };
    if (pos >= 0 && pos < N) { *cell = at(pos); *par = I.cell0 + *cell; return; }
    if (I.kind == KIND_PER1 || I.kind == KIND_PER2 || I.kind == KIND_PER3) {
        const int q = ((pos % N) + N) % N;
        *cell = at(q); *par = I.cell0 + *cell; return;
    }
    if (I.kind == KIND_SHOCK) { *cell = own; *par = I.pseudo0 + (pos < 0 ? 0 : 1); return; }
    const bool low = pos < 0;
    const bool emitted = low ? (sgn > 0) : (sgn < 0);
    if (emitted) {
        const int w = 2 * axis + (low ? 0 : 1);
        const int face = axis == 0 ? iz * I.ny + iy : axis == 1 ? iz * I.nx + ix : iy * I.nx + ix;
        *cell = own;
        *par = I.pseudo0 + wall_offset(I, w) + face;
    } else {
        *cell = at(low ? 0 : N - 1);
        *par = I.cell0 + *cell;
    }
}


// One stencil input for the current lane: VEC consecutive jx at one jy.
template <typename real, int VEC>
struct Tap {
    using V = vec_t<real, VEC>;
    uint32_t off;      // byte offset of h at (slot cell, jz = 0, first jx of the group)
    const real *tz;    // TZ of the slot entry (LDS)
    real c0;
    V l1, l2;
    __device__ __forceinline__ V load(const real *base, uint32_t zoff) const { return ld<V>(base, off + zoff); }
    __device__ __forceinline__ V relax(V h, int jz) const
    {
        const real a = tz[2 * jz], b = tz[2 * jz + 1];
        return c0 * h + (l1 * a + l2 * b);
    }
    // same arithmetic with the plane's table values given
    __device__ __forceinline__ V relax_ab(V h, real a, real b) const { return c0 * h + (l1 * a + l2 * b); }
};

// Tap reading h of instance-local cell `cell` with the tables of entry E.
template <typename real, int VEC>
__device__ __forceinline__ Tap<real, VEC> make_tap_at(const Geo &g, const real *E, int cell, int p0, int jx0, int jy)
{
    Tap<real, VEC> t;
    t.off = (uint32_t)(((long long)cell * g.nv + p0) * sizeof(real));
    t.tz = E + g.tz;
    t.c0 = E[0];
    const real y1 = E[g.ty1 + jy], y2 = E[g.ty2 + jy];
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
        t.l1[k] = E[g.tx1 + jx0 + k] * y1;
        t.l2[k] = E[g.tx2 + jx0 + k] * y2;
    }
    return t;
}

template <typename real, int VEC>
__device__ __forceinline__ Tap<real, VEC> make_tap(const Geo &g, const real *sp, const SlotInfo &SI, int slot, int p0,
                                                   int jx0, int jy)
{
    return make_tap_at<real, VEC>(g, sp + slot * g.pe, SI.cell[slot], p0, jx0, jy);
}

// The same with the slot cell's byte offset from the workgroup's slot table
// (computed once per work item instead of a 32-bit product per lane and tap).
template <typename real, int VEC>
__device__ __forceinline__ Tap<real, VEC> make_tap_slot(const Geo &g, const real *sp, const SlotInfo &SI, int slot,
                                                        int p0, int jx0, int jy)
{
    const real *E = sp + slot * g.pe;
    Tap<real, VEC> t;
    t.off = SI.off[slot] + (uint32_t)(p0 * (int)sizeof(real));
    t.tz = E + g.tz;
    t.c0 = E[0];
    const real y1 = E[g.ty1 + jy], y2 = E[g.ty2 + jy];
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
        t.l1[k] = E[g.tx1 + jx0 + k] * y1;
        t.l2[k] = E[g.tx2 + jx0 + k] * y2;
    }
    return t;
}

// Upwind flux difference along one direction, values in upwind order
// (u_{-2}, u_{-1}, u_0, u_1), Courant magnitudes C and slope factors k = (1 - C)/2.
// With d0 = u_0 - u_{-1} and the limited slopes m1 = minmod(u_1 - u_0, d0),
// m0 = minmod(d0, u_{-1} - u_{-2}), the two face values differ by
// face(u_0) - face(u_{-1}) = d0 + k (m1 - m0).
template <typename real>
__device__ __forceinline__ real fmadd(real a, real b, real c)
{
    if constexpr (sizeof(real) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

template <typename real, int VEC>
__device__ __forceinline__ vec_t<real, VEC> flux_diff(vec_t<real, VEC> um2, vec_t<real, VEC> um1, vec_t<real, VEC> u0,
                                                      vec_t<real, VEC> u1, vec_t<real, VEC> C, vec_t<real, VEC> k)
{
    vec_t<real, VEC> r;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const real d0 = u0[e] - um1[e];
        const real m1 = minmod3(u1[e] - u0[e], d0), m0 = minmod3(d0, um1[e] - um2[e]);
        r[e] = C[e] * fmadd(k[e], m1 - m0, d0);
    }
    return r;
}

// Lane tasks.  A task is (group of VEC consecutive jx at one jy, residue zr of
// jz modulo ZR); it loops over jz = z0 + zr, z0 + zr + ZR, ... < z1.  The host
// picks VEC so that all v_x of a group share a sign, and ZR so that the task
// count fills whole waves.
// UNR, PD: the jz pipeline -- UNR planes per stage (1 or 2); with one plane
// per stage, PD planes in flight ahead of the one computed (1 to 3).
// NTSTORE: store the output non-temporally (chosen by the host when the working
// set exceeds the last-level cache; a plain store otherwise).
// ZU: one jz residue (ZR = 1), so all lanes of a wave walk the same plane.
// The plane's byte offset is then wave-uniform: the taps are buffer loads
// with it as their scalar offset (no per-tap vector address arithmetic), and
// the z-tables of the taps are re-laid out in LDS as [sign combination][jz]
// [tap role][2] so that one vector address per plane reaches every tap's
// pair through immediate offsets.
// Byte offset of the per-thread moment sums in the streaming kernel's dynamic
// LDS: after `elems` table values, 8-byte aligned.
template <typename real>
__host__ __device__ constexpr size_t stream_acc_offset(size_t elems) { return (elems * sizeof(real) + 7) & ~(size_t)7; }

template <typename real, int DIM, int VEC, int UNR, int PD, bool NTSTORE, bool ZU, bool REC = false>
__global__ void __launch_bounds__(256)
    k_stream(Args A, const real *__restrict__ src, real *__restrict__ dst, const real *__restrict__ params,
             double *__restrict__ partial)
{
    static_assert(!REC || DIM <= 2, "branch records of one- and two-dimensional kinds");
    using V = vec_t<real, VEC>;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NSLOT = 1 + 6 * DIM;
    real *sp = reinterpret_cast<real *>(smem);
    __shared__ SlotInfo SI;
    const Geo &g = A.g;
    constexpr int NROLE = 1 + 3 * DIM;        // centre, x (-2, -1, +1), y (-2, -1, +1), z (-2, -1, +1)
    constexpr int NCOMBO = DIM == 1 ? 2 : 4;  // sign of v_x (and of v_y; the z roles follow the plane)
    // moment sums kept per thread: without z streaming the z half fluxes are
    // zero and stay out of LDS
    constexpr int NACC = DIM == 3 ? NQ : 9;
    // Dynamic LDS: the slot entries (NSLOT table entries), the role-ordered
    // z-tables (one-residue form), then 8-byte aligned: this thread's moment
    // sums (acc[q * blockDim.x]) and the node tables, v_z and v_z^2 of every
    // plane (vzt[2 jz], vzt[2 jz + 1]; wave-uniform per plane: one LDS
    // broadcast instead of recomputing them per lane; in reduced velocity
    // space the planes' mass shares and energy terms -- the column fold takes
    // the mass from the first sum there, reduced contexts run with VEC = 1),
    // v_x and v_y of every node (the lane constants of a task and the column
    // fold read them instead of recomputing the nodes in double).
    double *const acc_base = reinterpret_cast<double *>(
        smem + stream_acc_offset<real>(NSLOT * g.pe + (ZU ? NCOMBO * g.nvz * NROLE * 2 : 0)));
    double *const vzt = acc_base + NACC * blockDim.x;
    double *const vxt = vzt + 2 * g.nvz;
    double *const vyt = vxt + g.nvx;
    for (int k = threadIdx.x; k < g.nvz; k += blockDim.x) {
        const ZW w = zweights(g, k);
        vzt[2 * k] = g.red ? w.m : w.z;
        vzt[2 * k + 1] = w.zz;
    }
    for (int k = threadIdx.x; k < g.nvx; k += blockDim.x) vxt[k] = vnode(g, 0, k);
    for (int k = threadIdx.x; k < g.nvy; k += blockDim.x) vyt[k] = vnode(g, 1, k);
    // (the first barrier of the item loop orders these writes before any read)
    // Work items (cell, jz chunk).  A grid smaller than the item count makes
    // the kernel persistent: each workgroup walks items gridDim.x apart (a
    // multiple of 8 keeps every workgroup on one XCD's contiguous range).
    const int nitems = A.ncells * A.vsplit;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int Lq = xcd_remap(item, nitems);
    int gq, split;
    item_cell_chunk(Lq, A.ncells, A.vsplit, &gq, &split);
    const int ii = find_inst(A.cell_prefix, A.ninst, gq);
    const Inst &I = A.inst[ii];
    const int c = strip_cell(I, gq - I.cell0);
    const int gc = I.cell0 + c;
    const int L = gc * A.vsplit + split;  // (cell, chunk) index of the partial sums
    const int pl = I.nx * I.ny, iz = c / pl, ix = c % I.nx, iy = (c - iz * pl) / I.nx;

    if (threadIdx.x < NSLOT) {
        const int s = threadIdx.x;
        int cell, par;
        if (s == 0) { cell = c; par = gc; }
        else {
            const int d = (s - 1) / 6, r = (s - 1) % 6, si = r / 3, m = r % 3;
            const int sgn = si == 0 ? 1 : -1, k = m == 0 ? -2 : (m == 1 ? -1 : 1);
            resolve_slot(I, d, ix, iy, iz, sgn * k, sgn, c, &cell, &par);
        }
        SI.cell[s] = cell;
        SI.par[s] = par;
        SI.off[s] = (uint32_t)cell * (uint32_t)g.nv * (uint32_t)sizeof(real);  // instance bytes < 2^32 (init)
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NSLOT * g.pe; t += blockDim.x) {
        const int s = t / g.pe, o = t - s * g.pe;
        sp[t] = params[(long long)SI.par[s] * g.pe + o];
    }
    __syncthreads();
    real *tzr = sp + NSLOT * g.pe;           // [combo][jz][role][2]
    if constexpr (ZU) {
        const int n = NCOMBO * g.nvz * NROLE;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            const int role = t % NROLE, jz = (t / NROLE) % g.nvz, combo = t / (NROLE * g.nvz);
            const int sx = combo & 1, sy = combo >> 1, sz = jz < g.zneg ? 1 : 0;
            const int slot = role == 0   ? 0
                             : role <= 3 ? 1 + 3 * sx + (role - 1)
                             : role <= 6 ? 7 + 3 * sy + (role - 4)
                                         : 13 + 3 * sz + (role - 7);
            const real *E = sp + slot * g.pe + g.tz + 2 * jz;
            tzr[2 * t] = E[0];
            tzr[2 * t + 1] = E[1];
        }
        __syncthreads();
    }

    const real *base = src + I.f0;
    real *outb = dst + I.f0;
    // the instance's f as a buffer (its byte size is below 2^32, checked at init)
    const __amdgpu_buffer_rsrc_t frs = make_rsrc(base, (uint32_t)((long long)I.ncell * g.nv * sizeof(real)));
    const uint32_t out0 = (uint32_t)((long long)c * g.nv * sizeof(real));
    int z0, z1;
    chunk_bounds(g.nvz, A.vsplit, split, &z0, &z1);
    const bool lim = I.minmod != 0;
    const int ngx = g.nvx / VEC, ngroups = ngx * g.nvy, ntask = ngroups * A.zr;
    const uint32_t zstep = (uint32_t)(g.npl * sizeof(real));
    const uint32_t ecell = (uint32_t)c * (uint32_t)g.nv;  // element index of (cell, 0) in the instance
    const uint32_t key = sizeof(real) == 4 ? pass_key(A.pass, 0) : 0u;
    // the centre entry's c0 - 1 as a two-float sum (float path)
    const double c0m1 = sizeof(real) == 4 ? *reinterpret_cast<const double *>(sp + 2) - 1.0 : 0.0;
    const float c0m1_hi = (float)c0m1, c0m1_lo = (float)(c0m1 - (double)c0m1_hi);
    double *acc = acc_base + threadIdx.x;  // this thread's moment sums, zeroed per work item
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q * blockDim.x] = 0.0;

    // (jx group, jy) of a one-residue task by a float reciprocal: task <
    // 2^14 and ngx <= 128, so (task + 1/2) / ngx stays at least 1/256 away
    // from an integer, far beyond the product's rounding error
    const float inv_ngx = 1.0f / (float)ngx;
    for (int task = threadIdx.x; task < ntask; task += blockDim.x) {
        int pg, zr, jy;
        if constexpr (ZU) {
            pg = task;
            zr = 0;
            jy = (int)(((float)task + 0.5f) * inv_ngx);
        } else {
            pg = task % ngroups;
            zr = task / ngroups;
            jy = pg / ngx;
        }
        const int jx0 = (pg - jy * ngx) * VEC;
        const int p0 = jy * g.nvx + jx0;
        V Cx, kx;
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            Cx[k] = (real)(fabs(vxt[jx0 + k]) * I.cx);
            kx[k] = lim ? (real)0.5 * ((real)1 - Cx[k]) : (real)0;
        }
        const double vy = vyt[jy];
        const int sx = vxt[jx0] > 0.0 ? 0 : 1;
        const Tap<real, VEC> tc = make_tap_slot<real, VEC>(g, sp, SI, 0, p0, jx0, jy);
        const Tap<real, VEC> xa = make_tap_slot<real, VEC>(g, sp, SI, 1 + 3 * sx + 0, p0, jx0, jy);
        const Tap<real, VEC> xb = make_tap_slot<real, VEC>(g, sp, SI, 1 + 3 * sx + 1, p0, jx0, jy);
        const Tap<real, VEC> xd = make_tap_slot<real, VEC>(g, sp, SI, 1 + 3 * sx + 2, p0, jx0, jy);
        Tap<real, VEC> ya, yb, yd, za, zb, zd;
        V Cy = 0, ky = 0;
        if constexpr (DIM >= 2) {
            const int sy = vy > 0.0 ? 0 : 1;
            const real cy = (real)(fabs(vy) * I.cy);
            Cy = cy;
            ky = lim ? (real)0.5 * ((real)1 - cy) : (real)0;
            ya = make_tap_slot<real, VEC>(g, sp, SI, 7 + 3 * sy + 0, p0, jx0, jy);
            yb = make_tap_slot<real, VEC>(g, sp, SI, 7 + 3 * sy + 1, p0, jx0, jy);
            yd = make_tap_slot<real, VEC>(g, sp, SI, 7 + 3 * sy + 2, p0, jx0, jy);
        }
        double A0[VEC];
#pragma unroll
        for (int k = 0; k < VEC; ++k) A0[k] = 0.0;
        double Az = 0.0, Azz = 0.0;
        constexpr int NT = NROLE;
        const Tap<real, VEC> *taps[10] = {&tc, &xa, &xb, &xd, &ya, &yb, &yd, &za, &zb, &zd};
        // this lane's z-table rows (ZU): combination of the signs of v_x, v_y
        const int combo = DIM == 1 ? sx : sx + 2 * (vy > 0.0 ? 0 : 1);
        const real *tzl = tzr + combo * g.nvz * NROLE * 2;
        // One jz: relax the loaded taps, stream, store, accumulate moments.
        // One jz: relax the loaded taps, stream, store, accumulate moments.
        // zo is the byte offset of plane jz (jz * Nvx * Nvy elements).
        // hp: the hashes of this plane pair when the caller computed them
        // (have), for two consecutive planes of one stage.
        using U = vec_t<uint32_t, VEC>;
        // have_c: std::true_type when the caller passes the plane pair's hash
        // in hp (one-residue float forms, whose chunks start on even planes),
        // std::false_type when each element hashes its own index
        auto finish = [&](const V (&hv)[NT], int jz, uint32_t zo, U hp, auto have_c) {
            constexpr bool HAVE = decltype(have_c)::value;
            real ta[NT], tb[NT];  // the taps' z-table values at plane jz
            if constexpr (ZU) {
                const real *row = tzl + jz * (NROLE * 2);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    ta[t] = row[2 * t];
                    tb[t] = row[2 * t + 1];
                }
            } else {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    ta[t] = taps[t]->tz[2 * jz];
                    tb[t] = taps[t]->tz[2 * jz + 1];
                }
            }
            const V u0 = tc.relax_ab(hv[0], ta[0], tb[0]);
            const V xm2 = xa.relax_ab(hv[1], ta[1], tb[1]), xm1 = xb.relax_ab(hv[2], ta[2], tb[2]);
            const V xp1 = xd.relax_ab(hv[3], ta[3], tb[3]);
            V dx = flux_diff<real, VEC>(xm2, xm1, u0, xp1, Cx, kx);
            V dy = 0;
            V ym2 = 0, ym1 = 0, yp1 = 0;
            if constexpr (DIM >= 2) {
                ym2 = ya.relax_ab(hv[4], ta[4], tb[4]);
                ym1 = yb.relax_ab(hv[5], ta[5], tb[5]);
                yp1 = yd.relax_ab(hv[6], ta[6], tb[6]);
                dy = flux_diff<real, VEC>(ym2, ym1, u0, yp1, Cy, ky);
            }
            if constexpr (REC) {
                // branch record for the reverse sweep, one byte per element:
                // per direction (x in bits 0-3, y in bits 4-7) the branch of
                // the slope at the upwind neighbour (low two bits) and at the
                // element itself (high two), from the limiter arguments above
                unsigned char *rp = A.rec + I.f0 + ecell + (uint32_t)p0 + zo / (uint32_t)sizeof(real);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const real dx0 = u0[e] - xm1[e];
                    uint32_t code = mm_code<real>(dx0, xm1[e] - xm2[e]) | mm_code<real>(xp1[e] - u0[e], dx0) << 2;
                    if constexpr (DIM >= 2) {
                        const real dy0 = u0[e] - ym1[e];
                        code |= (mm_code<real>(dy0, ym1[e] - ym2[e]) | mm_code<real>(yp1[e] - u0[e], dy0) << 2) << 4;
                    }
                    rp[e] = (unsigned char)code;
                }
            }
            if constexpr (DIM == 3) {
                // the plane's Courant number along z (v_z of the plane from LDS)
                const real cz = (real)(fabs(vzt[2 * jz]) * I.cz);
                const V Cz = cz, kz = lim ? (real)0.5 * ((real)1 - cz) : (real)0;
                dy += flux_diff<real, VEC>(za.relax_ab(hv[7], ta[7], tb[7]), zb.relax_ab(hv[8], ta[8], tb[8]), u0,
                                           zd.relax_ab(hv[9], ta[9], tb[9]), Cz, kz);
            }
            V r;
            if constexpr (sizeof(real) == 4) {
                // New value h + d with the increment d = (c0 - 1) h + M - fluxes
                // formed in float (c0 - 1 as a two-float sum, so the relaxation
                // keeps its mass to ~2^-48), then h + d in double and one
                // stochastic rounding.  The increment's own rounding is
                // relative to d, far below an ulp of h wherever d is small.
                const real a = ta[0], b = tb[0];
                // random bits: one hash per element pair (planes 2k and 2k + 1 of
                // one velocity column, keyed by the even member's index), low
                // half for the even plane
                const bool odd = (jz & 1) != 0;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const real M = tc.l1[e] * a + tc.l2[e] * b;
                    const real d = __builtin_fmaf(c0m1_hi, hv[0][e], __builtin_fmaf(c0m1_lo, hv[0][e], M)) - (dx[e] + dy[e]);
                    uint32_t hb;
                    if constexpr (HAVE) {
                        hb = hp[e];
                    } else {
                        const uint32_t ieven =
                            ecell + (uint32_t)p0 + zo / (uint32_t)sizeof(real) - (odd ? (uint32_t)g.npl : 0u);
                        hb = hash32((ieven + (uint32_t)e) ^ key);
                    }
                    // bits 0-15 for the even plane, 16-31 for the odd one
                    r[e] = round_stochastic16((double)hv[0][e] + (double)d,
                                              __builtin_amdgcn_ubfe(hb, odd ? 16u : 0u, 16u));
                }
            } else {
                r = u0 - dx - dy;
            }
            V *op = reinterpret_cast<V *>(reinterpret_cast<char *>(outb) + out0 + zo + (uint32_t)(p0 * sizeof(real)));
            if constexpr (NTSTORE) __builtin_nontemporal_store(r, op);
            else *op = r;
            double s = (double)r[0];
            A0[0] += s;
#pragma unroll
            for (int k = 1; k < VEC; ++k) {
                const double hk = (double)r[k];
                A0[k] += hk;
                s += hk;
            }
            Az += vzt[2 * jz] * s;
            Azz += vzt[2 * jz + 1] * s;
        };
        // Software pipeline: the loads of the next UNR jz planes are issued
        // before the current ones are relaxed and streamed, so every wave keeps
        // one group of loads in flight while it computes.  Plane offsets
        // advance by additions; prefetches past the lane's last plane re-read
        // it.  With two planes per stage the loop body is written twice over
        // alternating register sets, so a prefetched value is consumed one
        // stage later and never copied; with one plane per stage a ring of
        // PD + 1 single-plane buffers keeps PD planes in flight (more loads in
        // flight per register than two-plane stages, where half the buffers
        // are being computed on).
        const int zs = UNR * A.zr;
        // One sweep over the planes [zb0, zb1) of the chunk: the lane's first
        // plane there is the first of its residue class (chunk start + zr).
        auto sweep = [&](int zb0, int zb1) {
        int jz = zb0 + ((z0 + zr - zb0) % A.zr + A.zr) % A.zr;
        if (jz < zb1) {
            const int zlast = ZU ? zb1 - 1 : zb1 - 1 - ((zb1 - 1 - jz) % A.zr);  // last jz of this lane's residue
            const uint32_t zlast_off = (uint32_t)zlast * zstep, zr_off = (uint32_t)A.zr * zstep;
            const uint32_t zs_off = (uint32_t)zs * zstep;
            uint32_t zoff = (uint32_t)jz * zstep;
            auto load_stage = [&](V (&h)[UNR][NT], uint32_t off) {
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const uint32_t o = min(off + (uint32_t)u * zr_off, zlast_off);
                    if constexpr (ZU) {
                        // buffer loads: tap offset per lane, wave-uniform plane offset
                        const uint32_t so = __builtin_amdgcn_readfirstlane(o);
#pragma unroll
                        for (int t = 0; t < NT; ++t) h[u][t] = buf_ld<V>(frs, taps[t]->off, so);
                    } else {
#pragma unroll
                        for (int t = 0; t < NT; ++t) h[u][t] = taps[t]->load(base, o);
                    }
                }
            };
            auto compute_stage = [&](const V (&h)[UNR][NT], int j, uint32_t off) {
                if constexpr (sizeof(real) == 4 && UNR == 2 && ZU) {
                    // one residue, chunks starting on even planes, two planes per
                    // stage: j is even, and one hash serves the pair (j, j + 1)
                    U hp;
                    const uint32_t ieven = ecell + (uint32_t)p0 + off / (uint32_t)sizeof(real);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) hp[e] = hash32((ieven + (uint32_t)e) ^ key);
                    finish(h[0], j, off, hp, std::true_type{});
                    if (j + 1 < zb1) finish(h[1], j + 1, off + zr_off, hp, std::true_type{});
                } else {
#pragma unroll
                    for (int u = 0; u < UNR; ++u)
                        if (j + u * A.zr < zb1)
                            finish(h[u], j + u * A.zr, off + (uint32_t)u * zr_off, U(0), std::false_type{});
                }
            };
            if constexpr (UNR == 2) {
                V ha[UNR][NT], hb[UNR][NT];
                load_stage(ha, zoff);
                for (;;) {
                    load_stage(hb, zoff + zs_off);
                    compute_stage(ha, jz, zoff);
                    jz += zs;
                    zoff += zs_off;
                    if (jz >= zb1) break;
                    load_stage(ha, zoff + zs_off);
                    compute_stage(hb, jz, zoff);
                    jz += zs;
                    zoff += zs_off;
                    if (jz >= zb1) break;
                }
            } else {
                // One plane per stage.  With one residue a lane's planes are
                // consecutive from an even first plane, and the random bits of
                // an even plane are kept for its odd partner.
                U hcar = 0;
                auto stage1 = [&](const V (&h)[1][NT], int j, uint32_t off) {
                    if constexpr (sizeof(real) == 4 && ZU) {
                        if ((j & 1) == 0) {
                            const uint32_t ieven = ecell + (uint32_t)p0 + off / (uint32_t)sizeof(real);
#pragma unroll
                            for (int e = 0; e < VEC; ++e) hcar[e] = hash32((ieven + (uint32_t)e) ^ key);
                        }
                        finish(h[0], j, off, hcar, std::true_type{});
                    } else {
                        finish(h[0], j, off, hcar, std::false_type{});
                    }
                };
                if constexpr (PD == 1) {
                    // one plane in flight: plain rotation (the compiler
                    // renames the copies)
                    V ha[1][NT];
                    load_stage(ha, zoff);
                    for (; jz < zb1; jz += zs, zoff += zs_off) {
                        V hn[1][NT];
                        load_stage(hn, zoff + zs_off);
                        stage1(ha, jz, zoff);
#pragma unroll
                        for (int t = 0; t < NT; ++t) ha[0][t] = hn[0][t];
                    }
                } else {
                    // PD planes in flight: a ring of PD + 1 buffers (buffer
                    // r % (PD + 1) holds the lane's plane jz + r * zr)
                    V hr[PD + 1][1][NT];
#pragma unroll
                    for (int d = 0; d < PD; ++d) load_stage(hr[d], zoff + (uint32_t)d * zs_off);
                    for (;;) {
#pragma unroll
                        for (int r = 0; r <= PD; ++r) {
                            load_stage(hr[(r + PD) % (PD + 1)], zoff + (uint32_t)PD * zs_off);
                            stage1(hr[r], jz, zoff);
                            jz += zs;
                            zoff += zs_off;
                            if (jz >= zb1) goto ring_done;
                        }
                    }
                ring_done:;
                }
            }
        }
        };
        double Azm = 0.0, Azp = 0.0;
        if constexpr (DIM == 3) {
            // planes with v_z < 0 (upwind neighbours on the +z side, s = -1),
            // then those with v_z > 0 (s = +1); Az splits into the two half
            // fluxes on the way
            za = make_tap_slot<real, VEC>(g, sp, SI, 16, p0, jx0, jy);
            zb = make_tap_slot<real, VEC>(g, sp, SI, 17, p0, jx0, jy);
            zd = make_tap_slot<real, VEC>(g, sp, SI, 18, p0, jx0, jy);
            sweep(z0, min(z1, g.zneg));
            const double Aneg = Az;
            Az = 0.0;
            za = make_tap_slot<real, VEC>(g, sp, SI, 13, p0, jx0, jy);
            zb = make_tap_slot<real, VEC>(g, sp, SI, 14, p0, jx0, jy);
            zd = make_tap_slot<real, VEC>(g, sp, SI, 15, p0, jx0, jy);
            sweep(max(z0, g.zneg), z1);
            Azm = -Aneg;
            Azp = Az;
            Az = Aneg + Az;
        } else {
            sweep(z0, z1);
        }
#pragma unroll
        for (int k = 0; k < VEC; ++k)
            if (g.red) fold_column_lds<NACC>(acc, blockDim.x, vxt[jx0 + k], vy, k == 0 ? Az : 0.0, 0.0, k == 0 ? Azz : 0.0);
            else fold_column_lds<NACC>(acc, blockDim.x, vxt[jx0 + k], vy, A0[k], k == 0 ? Az : 0.0,
                                       k == 0 ? Azz : 0.0, k == 0 ? Azm : 0.0, k == 0 ? Azp : 0.0);
    }
    {
        double sums[NACC];
#pragma unroll
        for (int q = 0; q < NACC; ++q) sums[q] = acc[q * blockDim.x];
        block_sum_store<NACC>(sums, partial + (long long)L * NQ);
        if (threadIdx.x >= NACC && threadIdx.x < NQ) partial[(long long)L * NQ + threadIdx.x] = 0.0;
    }
    __syncthreads();  // LDS (slots, tables, reduction) is reused by the next item
    }
}

// ---------------------------------------------------------------- shift
// Streaming pass in the translation form of Sec. 2.1 (the text below Eq.
// (exact)), for one-dimensional instances and any Courant number: with
// C = v_x dt / dx, |C| = m + th, the value of cell i is taken from cells
// a = i - s m and b = i - s (m + 1) (s = sign v_x) and blended over the
// fraction th as in Eq. (upwind):
//     out = u_a - th (u_a - u_b),   u = the relaxed input (table entries of a, b).
// A lane task is one (jx, jy) at one jz residue, as in the per-cell kernel
// with VEC = 1; the two sources and their entries depend on v_x, so each
// lane resolves them itself (entries from global memory instead of the
// workgroup's slot table).  With STAGE the v_z tables of the 2 Nvx source
// entries of the workgroup's cell (one pair per jx and source) are copied
// to LDS once per cell, [jz][source][jx][2], so the jz loop issues two
// global loads per element (the two sources' h) instead of six.  With
// |C| < 1 (m = 0) every operation, the rounding bits and the moment
// epilogue are those of the per-cell kernel with the limiter off, so the
// two agree bit for bit there.

// Source k (0: a = c - s m, 1: b = a - s) of cell c: the cell whose h is
// read and the table entry that relaxes it (ghosts read cell c; their
// entries have c0 = 0).
__device__ __forceinline__ void shift_source(const Inst &I, int c, int sgn, int m, int k, int *cell, int *par)
{
    const int pos = c - sgn * (m + k);
    if (pos >= 0 && pos < I.nx) { *cell = pos; *par = I.cell0 + pos; }
    else if (I.kind == KIND_PER1) { *cell = ((pos % I.nx) + I.nx) % I.nx; *par = I.cell0 + *cell; }
    else { *cell = c; *par = I.pseudo0 + (pos < 0 ? 0 : 1); }
}

__device__ __forceinline__ void shift_of(const Geo &g, const Inst &I, int jx, int *m, int *sgn, double *ac)
{
    const double vx = vnode(g, 0, jx);
    *ac = fabs(vx) * I.cx;
    *m = (int)floor(*ac);
    *sgn = vx > 0.0 ? 1 : -1;
}

template <typename real, bool NTSTORE, bool STAGE>
__global__ void __launch_bounds__(256)
    k_shift(Args A, const real *__restrict__ src, real *__restrict__ dst, const real *__restrict__ params,
            double *__restrict__ partial)
{
    using V = vec_t<real, 1>;
    extern __shared__ __align__(16) unsigned char smem[];
    real *stz = reinterpret_cast<real *>(smem);  // STAGE: [jz - z0][source][jx][2]
    __shared__ double vzt[NVMAX][2];
    const Geo &g = A.g;
    for (int k = threadIdx.x; k < g.nvz; k += blockDim.x) {
        const ZW w = zweights(g, k);  // as in k_stream: mass shares first when reduced
        vzt[k][0] = g.red ? w.m : w.z;
        vzt[k][1] = w.zz;
    }
    __syncthreads();
    const int nitems = A.ncells * A.vsplit;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int Lq = xcd_remap(item, nitems);
        const int gq = Lq / A.vsplit, split = Lq % A.vsplit;
        const int ii = find_inst(A.cell_prefix, A.ninst, gq);
        const Inst &I = A.inst[ii];
        const int c = gq - I.cell0;
        const int L = gq * A.vsplit + split;
        const real *base = src + I.f0;
        real *outb = dst + I.f0;
        const __amdgpu_buffer_rsrc_t frs = make_rsrc(base, (uint32_t)((long long)I.ncell * g.nv * sizeof(real)));
        const uint32_t out0 = (uint32_t)((long long)c * g.nv * sizeof(real));
        int z0, z1;
    chunk_bounds(g.nvz, A.vsplit, split, &z0, &z1);
        const int ntask = g.npl * A.zr;
        const uint32_t zstep = (uint32_t)(g.npl * sizeof(real));
        const uint32_t ecell = (uint32_t)c * (uint32_t)g.nv;
        const uint32_t key = sizeof(real) == 4 ? pass_key(A.pass, 0) : 0u;
        double acc[NQ] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        if constexpr (STAGE) {
            // the previous item's reads of stz ended at its closing barrier
            const int nst = 2 * g.nvx * (z1 - z0);
            for (int q = threadIdx.x; q < nst; q += blockDim.x) {
                const int zl = q % (z1 - z0), r = q / (z1 - z0), jx = r % g.nvx, k = r / g.nvx;
                int m, sgn, cell, par;
                double ac;
                shift_of(g, I, jx, &m, &sgn, &ac);
                shift_source(I, c, sgn, m, k, &cell, &par);
                const real *E = params + (long long)par * g.pe + g.tz + 2 * (z0 + zl);
                real *d = stz + (((size_t)zl * 2 + k) * g.nvx + jx) * 2;
                d[0] = E[0];
                d[1] = E[1];
            }
            __syncthreads();
        }
        for (int task = threadIdx.x; task < ntask; task += blockDim.x) {
            const int p0 = task % g.npl, zr = task / g.npl;
            const int jy = p0 / g.nvx, jx = p0 - jy * g.nvx;
            const double vx = vnode(g, 0, jx), vy = vnode(g, 1, jy);
            int m, sgn;
            double ac;
            shift_of(g, I, jx, &m, &sgn, &ac);
            const real th = (real)(ac - (double)m);
            Tap<real, 1> tp[2];
            const real *Ez[2];
            for (int k = 0; k < 2; ++k) {
                int cell, par;
                shift_source(I, c, sgn, m, k, &cell, &par);
                const real *E = params + (long long)par * g.pe;
                tp[k] = make_tap_at<real, 1>(g, E, cell, p0, jx, jy);
                Ez[k] = E + g.tz;
            }
            // c0 - 1 of source a as a two-float sum (float path)
            float c0m1_hi = 0.0f, c0m1_lo = 0.0f;
            if constexpr (sizeof(real) == 4) {
                const double c0m1 = *reinterpret_cast<const double *>(Ez[0] - g.tz + 2) - 1.0;
                c0m1_hi = (float)c0m1;
                c0m1_lo = (float)(c0m1 - (double)c0m1_hi);
            }
            double A0 = 0.0, Az = 0.0, Azz = 0.0;
            int jz = z0 + zr;
            if (jz < z1) {
                const int zlast = z1 - 1 - ((z1 - 1 - (z0 + zr)) % A.zr);
                V h[2], hn[2];
                auto load = [&](V (&hv)[2], int j) {
                    const uint32_t so = (uint32_t)min(j, zlast) * zstep;
                    hv[0] = buf_ld<V>(frs, tp[0].off, so);
                    hv[1] = buf_ld<V>(frs, tp[1].off, so);
                };
                load(h, jz);
                for (; jz < z1; jz += A.zr) {
                    load(hn, jz + A.zr);
                    real a0, b0, a1, b1;
                    if constexpr (STAGE) {
                        const real *s0 = stz + ((size_t)(jz - z0) * 2 * g.nvx + jx) * 2;
                        const real *s1 = s0 + 2 * g.nvx;
                        a0 = s0[0];
                        b0 = s0[1];
                        a1 = s1[0];
                        b1 = s1[1];
                    } else {
                        a0 = Ez[0][2 * jz];
                        b0 = Ez[0][2 * jz + 1];
                        a1 = Ez[1][2 * jz];
                        b1 = Ez[1][2 * jz + 1];
                    }
                    const V u0 = tp[0].relax_ab(h[0], a0, b0);
                    const V u1 = tp[1].relax_ab(h[1], a1, b1);
                    const real dx = th * (u0[0] - u1[0]), dy = 0;
                    real r;
                    if constexpr (sizeof(real) == 4) {
                        const bool odd = (jz & 1) != 0;
                        const uint32_t ieven = ecell + (uint32_t)p0 + (uint32_t)jz * (uint32_t)g.npl -
                                               (odd ? (uint32_t)g.npl : 0u);
                        const real M = tp[0].l1[0] * a0 + tp[0].l2[0] * b0;
                        const real d = __builtin_fmaf(c0m1_hi, h[0][0], __builtin_fmaf(c0m1_lo, h[0][0], M)) - (dx + dy);
                        const uint32_t hb = hash32(ieven ^ key);
                        r = round_stochastic16((double)h[0][0] + (double)d, __builtin_amdgcn_ubfe(hb, odd ? 16u : 0u, 16u));
                    } else {
                        r = u0[0] - dx - dy;
                    }
                    real *op = reinterpret_cast<real *>(reinterpret_cast<char *>(outb) + out0 +
                                                        (uint32_t)jz * zstep + (uint32_t)(p0 * sizeof(real)));
                    if constexpr (NTSTORE) __builtin_nontemporal_store(r, op);
                    else *op = r;
                    const double hk = (double)r;
                    A0 += hk;
                    Az += vzt[jz][0] * hk;
                    Azz += vzt[jz][1] * hk;
                    h[0] = hn[0];
                    h[1] = hn[1];
                }
            }
            if (g.red) fold_column(acc, vx, vy, Az, 0.0, Azz);
            else fold_column(acc, vx, vy, A0, Az, Azz);
        }
        block_sum_store<NQ>(acc, partial + (long long)L * NQ);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- shift, row tiles
// The translation form again, organised for coalesced access.  At a fixed
// velocity the sources of consecutive cells are consecutive cells, but the
// shift m depends on jx: the per-cell kernel above gathers, per lane, one
// value from a different source cell, so every load touches its own cache
// line, and the source rows that one cell's velocity grid reaches (2 m_max
// cells of them) leave the L2 between their uses.  Here a work item is
// (tile of TT consecutive cells of one instance, plane jz), and for each
// velocity row jy of the plane the workgroup
//   1. loads the row (N_vx contiguous values) of every source cell the tile
//      reaches, relaxes it with that cell's table entry, and keeps per jx
//      the TT + 1 consecutive sources of the tile in LDS ([jx][k]);
//   2. lane (t, jx) blends its two sources from LDS and stores its value, the
//      N_vx lanes of a cell storing one contiguous row.
// Work items run plane-major, so the items in flight on one XCD are
// consecutive tiles of one plane and share their source rows in its L2.
// Moments: per (t, jx) a lane owns, the sums over the plane's rows of h,
// v_y h, v_y^2 h and the v_y < 0 part of v_y h (v_x, v_z are fixed), folded
// into the NQ sums of the cell at the end of the item and written to
// partial[(cell * N_vz + jz) * NQ + q] (the launch runs with vsplit = N_vz).
// Arithmetic: FP64 out = u_a - th (u_a - u_b) as in Eq. (upwind); FP32 keeps
// h and the relaxation increment r = (c0 - 1) h + M of each source
// (u = h + r), forms d = r_a - th (u_a - u_b) in float and rounds h_a + d
// stochastically with the random bits of the element (as every streaming
// kernel does).  Lane groups: G = 2^lg >= N_vx lanes per cell (N_vx <= 64),
// PPL (t, jx) pairs per lane, TT = PPL * ROW_THREADS / G - 1.

struct RowJx { int wb, ka, kb, pad; double th; };  // window index of source k = 0; source offsets of a and b

template <typename real>
struct RowCell { int par, cell; real c0, cmh, cml, z1, z2; real yz[4]; };  // yz: (TY1 TZ1, TY2 TZ2) of two rows

// Byte offsets of the row kernel's dynamic LDS.
struct RowLds { size_t stage, jx, cell, ent, scan, total; };

__host__ __device__ inline size_t row_align(size_t x) { return (x + 15) & ~(size_t)15; }

// Workgroups of ROW_THREADS lanes, two per CU (their barriers interleave);
// the window holds at most ROW_THREADS cells (one per lane in the per-cell
// passes).  ROW_EPL: staged sources per lane and row, (TT + 1) N_vx <=
// 4 ROW_THREADS of them (TT = 4 ROW_THREADS / G - 1).
constexpr int ROW_THREADS = 512;
constexpr int ROW_EPL = 4;

// Source list entry: element offset of the source at jy = 0 (-1: far field)
// and (stage index | w << 13 | jx << 23); with XIN also its v_x table values.
template <typename real, bool XIN>
struct RowEnt { int off; uint32_t packed; real x[XIN ? 2 : 1]; };

// Stage row stride (8-byte elements) of one jx: odd, so the 32 jx of a wave
// at one cell fall on distinct LDS banks.
__host__ __device__ inline int row_stride(int tt) { return (tt + 1) | 1; }

template <typename real, bool XIN>
__host__ __device__ inline RowLds row_lds(int nvx, int tt, int wmax)
{
    RowLds L;
    L.stage = 0;  // nvx rows of stride S holding tt + 1 sources, and one slot written by padding entries
    L.jx = row_align(((size_t)nvx * row_stride(tt) + 1) * 8);
    L.cell = L.jx + row_align((size_t)nvx * sizeof(RowJx));
    L.ent = L.cell + row_align((size_t)wmax * sizeof(RowCell<real>));
    L.scan = L.ent + row_align((size_t)ROW_EPL * ROW_THREADS * sizeof(RowEnt<real, XIN>));
    L.total = L.scan + row_align(32 * sizeof(int));
    return L;
}

// Per work item the window's needed (cell, jx) sources, TT + 1 per jx, are
// listed once in LDS (cell-major, so consecutive entries are consecutive jx
// of one cell row and their loads coalesce; the list is padded to ROW_EPL
// entries per lane with entries that load nothing useful and stage into a
// spare slot); each row then loads and relaxes just those, the loads of row
// jy + 1 (and the y-table values of row jy + 2) being issued before row jy
// is blended, so they are in flight during the blend.  Every global load
// and store is issued unconditionally (padding lanes repeat a valid lane's
// address and value), so the waits on them are static counts and a row's
// staging waits for its own loads only, not for the stores issued after.
template <typename real, int PPL, bool XIN, bool NTSTORE>
__global__ void __launch_bounds__(ROW_THREADS, 4)
    k_shift_rows(Args A, const real *__restrict__ src, real *__restrict__ dst, const real *__restrict__ params,
                 double *__restrict__ partial, int tt, int wmax, int lg)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Geo &g = A.g;
    const RowLds Lo = row_lds<real, XIN>(g.nvx, tt, wmax);
    // stage[jx * S + k], 8 bytes: FP32 (h, r) of the source, FP64 u
    using S2 = vec_t<real, sizeof(real) == 4 ? 2 : 1>;
    static_assert(sizeof(S2) == 8, "stage elements of 8 bytes");
    using Ent = RowEnt<real, XIN>;
    const int S = row_stride(tt);
    S2 *stage = reinterpret_cast<S2 *>(smem + Lo.stage);
    RowJx *JX = reinterpret_cast<RowJx *>(smem + Lo.jx);
    RowCell<real> *CT = reinterpret_cast<RowCell<real> *>(smem + Lo.cell);
    Ent *EN = reinterpret_cast<Ent *>(smem + Lo.ent);
    int *SC = reinterpret_cast<int *>(smem + Lo.scan);
    const int G = 1 << lg, tid = threadIdx.x, nth = blockDim.x;
    const int ntl = A.ntiles, nitems = ntl * g.nvz;
    const uint32_t key = sizeof(real) == 4 ? pass_key(A.pass, 0) : 0u;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int Lq = xcd_remap(item, nitems);
        const int jz = Lq / ntl, tile = Lq - jz * ntl;
        int lo = 0, hi = A.ninst;  // inst[lo].tile0 <= tile < inst[hi].tile0
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (A.inst[mid].tile0 <= tile) lo = mid; else hi = mid;
        }
        const Inst &I = A.inst[lo];
        const int i0 = (tile - I.tile0) * tt;
        const int te = min(tt, I.nx - i0);
        const int wlo = i0 - I.reach_lo;
        const int W = min(te + I.reach_lo + I.reach_hi, wmax);
        const uint32_t zoff = (uint32_t)jz * (uint32_t)g.npl;
        // per jx: shift, fraction and the window index of its first source
        for (int jx = tid; jx < g.nvx; jx += nth) {
            const double vx = vnode(g, 0, jx), ac = fabs(vx) * I.cx;
            const int m = (int)floor(ac);
            const bool pos = vx > 0.0;
            RowJx r;
            const int wb = (pos ? i0 - m - 1 : i0 + m) - wlo;
            r.wb = max(0, min(wb, W - 1 - te));  // (inside the window by the host's reach margins)
            r.ka = pos ? 1 : 0;
            r.kb = pos ? 0 : 1;
            r.pad = 0;
            r.th = ac - (double)m;
            JX[jx] = r;
        }
        // per window cell (one per lane): its table entry and the plane's factors
        const int w = tid;
        int cell = -1;
        if (w < W) {
            const int q = wlo + w;
            RowCell<real> c;
            if (q >= 0 && q < I.nx) { c.cell = q; c.par = I.cell0 + q; }
            else if (I.kind == KIND_PER1) { c.cell = ((q % I.nx) + I.nx) % I.nx; c.par = I.cell0 + c.cell; }
            else { c.cell = -1; c.par = I.pseudo0 + (q < 0 ? 0 : 1); }
            cell = c.cell;
            const real *E = params + (long long)c.par * g.pe;
            double c0;
            if constexpr (sizeof(real) == 4) c0 = *reinterpret_cast<const double *>(E + 2);
            else c0 = E[0];
            c.c0 = (real)c0;
            const double cm = c0 - 1.0;
            c.cmh = (real)cm;
            c.cml = (real)(cm - (double)c.cmh);
            c.z1 = E[g.tz + 2 * jz];
            c.z2 = E[g.tz + 2 * jz + 1];
            c.yz[0] = c.yz[1] = c.yz[2] = c.yz[3] = 0;
            CT[w] = c;
        }
        __syncthreads();
        // list the needed sources: count per cell, block-wide exclusive scan, fill
        int cnt = 0;
        if (w < W)
            for (int jx = 0; jx < g.nvx; ++jx) cnt += (unsigned)(w - JX[jx].wb) <= (unsigned)te ? 1 : 0;
        int inc = cnt;
        const int lane = tid & 63, wave = tid >> 6;
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(inc, o, 64);
            if (lane >= o) inc += v;
        }
        if (lane == 63) SC[wave] = inc;
        __syncthreads();
        int pre = 0, nent = 0;
        for (int k = 0; k < (nth >> 6); ++k) {
            const int v = SC[k];
            pre += k < wave ? v : 0;
            nent += v;
        }
        if (w < W) {
            int e = pre + inc - cnt;
            for (int jx = 0; jx < g.nvx; ++jx) {
                const int k = w - JX[jx].wb;
                if ((unsigned)k > (unsigned)te) continue;
                Ent en;
                en.off = cell >= 0 ? (int)((uint32_t)cell * (uint32_t)g.nv + zoff + (uint32_t)jx) : -1;
                en.packed = (uint32_t)(jx * S + k) | ((uint32_t)w << 13) | ((uint32_t)jx << 23);
                EN[e++] = en;
            }
        }
        // padding entries up to ROW_EPL per lane: no source, the spare stage slot
        for (int e = nent + tid; e < ROW_EPL * nth; e += nth) {
            Ent en;
            en.off = -1;
            en.packed = (uint32_t)(g.nvx * S);
            EN[e] = en;
        }
        __syncthreads();
        if constexpr (XIN) {
            for (int e = tid; e < ROW_EPL * nth; e += nth) {
                const uint32_t pk = EN[e].packed;
                const int ww = (pk >> 13) & 1023, jx = pk >> 23;
                const real *E = params + (long long)CT[ww].par * g.pe;
                EN[e].x[0] = E[g.tx1 + jx];
                EN[e].x[1] = E[g.tx2 + jx];
            }
        }
        // this lane's (t, jx) pairs: stage index of the lower source, which
        // of the two is a, fraction, output offset.  A padding lane (jx or t
        // beyond the grid or the tile) takes the last valid jx and t, so it
        // computes and stores that pair's value again; it adds no moments.
        int i0s[PPL];
        bool valid[PPL], apos[PPL];
        real th[PPL];
        uint32_t ooff[PPL];  // byte offset of the pair's value at jy = 0 in the instance
        double S0[PPL], Sy[PPL], Syy[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int q = tid + p * nth, tq = q >> lg, jq = q & (G - 1);
            valid[p] = jq < g.nvx && tq < te;
            const int t = min(tq, te - 1), jj = min(jq, g.nvx - 1);
            const RowJx r = JX[jj];
            // stage index k = window index - wb: the sources of cell i0 + t sit at
            // k = t, t + 1 (a the upper one for v_x > 0)
            i0s[p] = jj * S + t;
            apos[p] = r.ka != 0;
            th[p] = (real)r.th;
            ooff[p] = (uint32_t)(((long long)(i0 + t) * g.nv + (long long)jz * g.npl + jj) * sizeof(real));
            S0[p] = Sy[p] = Syy[p] = 0.0;
        }
        const real *base = src + I.f0;
        real *outb = dst + I.f0;
        // this lane's list entries tid + u nth: h of the row being fetched (a
        // far field or padding entry loads the instance's first row and keeps 0)
        // (the loaded values are used raw; the staging zeroes those of far
        // fields and padding, so no instruction consumes a load before its row)
        auto fetch = [&](int jy, real (&hreg)[ROW_EPL]) {
            int off[ROW_EPL];
#pragma unroll
            for (int u = 0; u < ROW_EPL; ++u) off[u] = EN[tid + u * nth].off;
#pragma unroll
            for (int u = 0; u < ROW_EPL; ++u) hreg[u] = base[(uint32_t)max(off[u], 0) + (uint32_t)(jy * g.nvx)];
        };
        real ty1 = 0, ty2 = 0;  // window cell tid (lanes past the window read the last one)
        const int wq = min(w, W - 1);
        auto fetch_ty = [&](int jy) {
            const real *E = params + (long long)CT[wq].par * g.pe;
            ty1 = E[g.ty1 + jy];
            ty2 = E[g.ty2 + jy];
        };
        auto put_yz = [&](int b) {
            if (w < W) {
                CT[w].yz[2 * b] = ty1 * CT[w].z1;
                CT[w].yz[2 * b + 1] = ty2 * CT[w].z2;
            }
        };
        // One row: stage from the loads in hreg, then reuse hreg for the loads
        // of row jy + 2 (two rows of latency cover), blend.  Rows come in
        // pairs with alternating buffers; with an odd row count the last pair
        // repeats row N_vy - 1 (same values stored again, no moments added).
        auto row = [&](int jyr, real (&hreg)[ROW_EPL]) {
            const bool live = jyr < g.nvy;
            const int jy = min(jyr, g.nvy - 1), b = jyr & 1;
            // stage the relaxed sources of row jy: all LDS reads first, then
            // the arithmetic, then the stage writes
            Ent en[ROW_EPL];
#pragma unroll
            for (int u = 0; u < ROW_EPL; ++u) en[u] = EN[tid + u * nth];
            real y1[ROW_EPL], y2[ROW_EPL], ch[ROW_EPL], cl[ROW_EPL], x1[ROW_EPL], x2[ROW_EPL];
#pragma unroll
            for (int u = 0; u < ROW_EPL; ++u) {
                const int ww = (en[u].packed >> 13) & 1023, jx = en[u].packed >> 23;
                const RowCell<real> &c = CT[ww];
                y1[u] = c.yz[2 * b];
                y2[u] = c.yz[2 * b + 1];
                if constexpr (sizeof(real) == 4) {
                    ch[u] = c.cmh;
                    cl[u] = c.cml;
                } else {
                    ch[u] = c.c0;
                    cl[u] = 0;
                }
                if constexpr (XIN) {
                    x1[u] = en[u].x[0];
                    x2[u] = en[u].x[1];
                } else {
                    const real *E = params + (long long)c.par * g.pe;
                    x1[u] = E[g.tx1 + jx];
                    x2[u] = E[g.tx2 + jx];
                }
            }
            S2 sv[ROW_EPL];
#pragma unroll
            for (int u = 0; u < ROW_EPL; ++u) {
                const real h = en[u].off >= 0 ? hreg[u] : (real)0;
                const real M = x1[u] * y1[u] + x2[u] * y2[u];
                if constexpr (sizeof(real) == 4) {
                    sv[u][0] = h;
                    sv[u][1] = __builtin_fmaf(ch[u], h, __builtin_fmaf(cl[u], h, M));
                } else {
                    sv[u][0] = ch[u] * h + M;
                }
            }
#pragma unroll
            for (int u = 0; u < ROW_EPL; ++u) stage[en[u].packed & 8191] = sv[u];
            put_yz(b ^ 1);  // (the last row's write is never read)
            __syncthreads();
            // loads of row jy + 2 in flight during this row's and the next row's
            // blend (the last rows load row N_vy - 1 again)
            fetch(min(jyr + 2, g.nvy - 1), hreg);
            fetch_ty(min(jyr + 2, g.nvy - 1));
            // blend, store, accumulate
            const double vy = vnode(g, 1, jy);
            const uint32_t yoff = (uint32_t)(jy * g.nvx) * (uint32_t)sizeof(real);
            S2 slo[PPL], shi[PPL];
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                slo[p] = stage[i0s[p]];
                shi[p] = stage[i0s[p] + 1];
            }
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                const S2 a = apos[p] ? shi[p] : slo[p], bb = apos[p] ? slo[p] : shi[p];
                real r;
                if constexpr (sizeof(real) == 4) {
                    const real ua = a[0] + a[1], ub = bb[0] + bb[1];
                    const real d = a[1] - th[p] * (ua - ub);
                    const uint32_t e = ooff[p] / (uint32_t)sizeof(real) + (uint32_t)(jy * g.nvx);  // element index
                    const bool odd = (jz & 1) != 0;
                    const uint32_t hb = hash32((e - (odd ? (uint32_t)g.npl : 0u)) ^ key);
                    r = round_stochastic16((double)a[0] + (double)d, __builtin_amdgcn_ubfe(hb, odd ? 16u : 0u, 16u));
                } else {
                    r = a[0] - th[p] * (a[0] - bb[0]);
                }
                real *op = reinterpret_cast<real *>(reinterpret_cast<char *>(outb) + ooff[p] + yoff);
                if constexpr (NTSTORE) __builtin_nontemporal_store(r, op);
                else *op = r;
                const double rd = valid[p] && live ? (double)r : 0.0;
                S0[p] += rd;
                Sy[p] = __builtin_fma(vy, rd, Sy[p]);
                Syy[p] = __builtin_fma(vy * vy, rd, Syy[p]);
            }
            __syncthreads();  // the next row's staging overwrites the stage
        };
        real hA[ROW_EPL], hB[ROW_EPL];
        fetch_ty(0);
        put_yz(0);
        fetch_ty(min(1, g.nvy - 1));
        fetch(0, hA);
        fetch(min(1, g.nvy - 1), hB);
        __syncthreads();
        for (int jy = 0; jy < g.nvy; jy += 2) {
            row(jy, hA);
            row(jy + 1, hB);
        }
        // fold into the NQ sums of each cell: a cell's G lanes are consecutive
        // lanes of one wave (G <= 64).  The y and z half fluxes (wall sums of
        // 2D and 3D kinds) are not formed: zero for these 1D instances.
        const ZW zw = zweights(g, jz);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int q = tid + p * nth, t = q >> lg, jx = q & (G - 1);
            double v[7];
            if (valid[p]) {
                const double vx = vnode(g, 0, jx), ms = zw.m * S0[p];
                v[0] = ms;
                v[1] = vx * ms;
                v[2] = zw.m * Sy[p];
                v[3] = zw.z * S0[p];
                v[4] = (vx * vx * ms + zw.m * Syy[p]) + zw.zz * S0[p];
                v[5] = vx < 0.0 ? -vx * ms : 0.0;
                v[6] = vx > 0.0 ? vx * ms : 0.0;
            } else {
#pragma unroll
                for (int k = 0; k < 7; ++k) v[k] = 0.0;
            }
#pragma unroll
            for (int k = 0; k < 7; ++k)
                for (int off = G >> 1; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
            if (jx == 0 && t < te) {
                double *out = partial + ((long long)(I.cell0 + i0 + t) * A.vsplit + jz) * NQ;
#pragma unroll
                for (int k = 0; k < 7; ++k) out[k] = v[k];
#pragma unroll
                for (int k = 7; k < NQ; ++k) out[k] = 0.0;
            }
        }
        __syncthreads();  // LDS tables are rebuilt by the next item
    }
}

// ---------------------------------------------------------------- final
// Pointwise f = R2(h) from the cell's own entry (MODE_FINAL tables); VEC
// consecutive jx per lane.  src may be dst (each lane rewrites what it read).
template <typename real, int VEC>
__global__ void __launch_bounds__(256) k_final(Args A, const real *src, real *dst, const real *__restrict__ params)
{
    using V = vec_t<real, VEC>;
    const Geo &g = A.g;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int gc = L / A.vsplit, split = L % A.vsplit;
    const int ii = find_inst(A.cell_prefix, A.ninst, gc);
    const Inst &I = A.inst[ii];
    const long long off = I.f0 + (long long)(gc - I.cell0) * g.nv;
    const real *sc = src + off;
    real *dc = dst + off;
    const real *E = params + (long long)gc * g.pe;
    int z0, z1;
    chunk_bounds(g.nvz, A.vsplit, split, &z0, &z1);
    const real c0 = E[0];
    const uint32_t key = sizeof(real) == 4 ? pass_key(A.pass, 1) : 0u;
    const double c0d = sizeof(real) == 4 ? *reinterpret_cast<const double *>(E + 2) : 0.0;
    const uint32_t ecell = (uint32_t)(gc - I.cell0) * (uint32_t)g.nv;
    const int ngrp = g.npl / VEC;
    for (int q = threadIdx.x; q < ngrp; q += blockDim.x) {
        const int p0 = q * VEC, jx0 = p0 % g.nvx, jy = p0 / g.nvx;
        V l1, l2;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            l1[e] = E[g.tx1 + jx0 + e] * E[g.ty1 + jy];
            l2[e] = E[g.tx2 + jx0 + e] * E[g.ty2 + jy];
        }
#pragma unroll 4
        for (int jz = z0; jz < z1; ++jz) {
            const uint32_t o = (uint32_t)((jz * g.npl + p0) * (int)sizeof(real));
            const V h = ld<V>(sc, o);
            const real a = E[g.tz + 2 * jz], b = E[g.tz + 2 * jz + 1];
            V r;
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if constexpr (sizeof(real) == 4) {
                    const double v = c0d * (double)h[e] + ((double)l1[e] * (double)a + (double)l2[e] * (double)b);
                    r[e] = round_stochastic(v, hash32((ecell + (uint32_t)(jz * g.npl + p0 + e)) ^ key));
                } else {
                    r[e] = c0 * h[e] + (l1[e] * a + l2[e] * b);
                }
            }
            *reinterpret_cast<V *>(reinterpret_cast<char *>(dc) + o) = r;
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
#pragma clang fp contract(off)
        // Sec. 4.1: upstream state for x < 0, downstream state for x >= 0.  The
        // centre is rounded after the product and after the sum (no fused
        // multiply-add), so a centre on x = 0 falls on the same side as in a
        // plain evaluation.
        const double x = I.x0 + (c + 0.5) * I.dx;
        const double *st = x < 0.0 ? I.up : I.dn;
        n = st[0]; V = st[1]; T = st[2];
    }
    const double P = n * pi_t_m32(T);
    const long long off = I.f0 + (long long)c * g.nv;
    int z0, z1;
    chunk_bounds(g.nvz, A.vsplit, split, &z0, &z1);
    for (int p = threadIdx.x; p < g.npl; p += blockDim.x) {
        const int jx = p % g.nvx, jy = p / g.nvx;
        const double dx = vnode(g, 0, jx) - V, vy = vnode(g, 1, jy);
        for (int jz = z0; jz < z1; ++jz) {
            if (g.red) {
                f[off + (long long)jz * g.npl + p] = (real)(P * exp(-(dx * dx + vy * vy) / T) * zfactor(g, jz, 0.0, T));
                continue;
            }
            const double vz = vnode(g, 2, jz);
            f[off + (long long)jz * g.npl + p] = (real)(P * exp(-(dx * dx + vy * vy + vz * vz) / T));
        }
    }
}

}  // namespace bgk
