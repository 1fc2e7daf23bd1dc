// bgk_adjoint.h -- gfx950 kernels of the reverse sweep (adjoint of one step).
//
// For a scalar loss L of the final state, lambda^n = dL/df^n obeys
// lambda^n = (d f^{n+1}/d f^n)^T lambda^{n+1} (plain sum over all entries as
// inner product).  With a = R_a(f^n) and h = S(a), f^{n+1} = R_b(h):
//     hbar     = R_b^T(lambda^{n+1}) at h,
//     abar     = S^T(hbar) at a,
//     lambda^n = R_a^T(abar) at f^n,
// plus the parameter gradients dL/dKn (every relaxation) and dL/dT_w (every
// wall).  Relaxation, Eq. (relaxation) of Sec. 2.1, is y = (1 - E) Phi + E x
// with E = exp(-nu tau), so its transpose is E mu plus a velocity polynomial
// 1, v, |v|^2 per cell whose coefficients come from six sums of mu against
// Phi and x (k_adj_sums, then k_adj_coef; k_adj_apply applies them; with
// one chunk per cell k_adj_close does all three in one pass per cell).  The
// minmod streaming step is transposed on the branches the forward step takes
// (k_adj_stream, gather form): the step's own streaming pass h = S(a), run in
// its recording form, stores each element's limiter branches, and the gather
// reads them with lambda^{n+1}; hbar is formed on the fly from per-cell
// coefficients and never stored.  The diffuse-wall ghosts of Eq. (bc_cavity)
// return their adjoint to the wall density n_W and from there to the
// wall-adjacent cell (k_adj_wall).
#pragma once

#include "bgk_device.h"

namespace bgk {

constexpr int NINFO = 8;  // per cell: n, Vx, Vy, Vz, T, nu, E, tau
constexpr int NSUM = 6;   // per cell part: A, Bx, By, Bz, C, D
constexpr int NWALL = 8;  // per cell part: (S_gamma, S_gamma') for walls 0..3

// Relaxation data of every cell from its moment sums: which = 0 is the
// opening relaxation R_a of a step (Strang R_{dt/2}, Lie none), 1 the
// closing one R_b (Strang R_{dt/2}, Lie R_dt).  One thread per cell.
__global__ void k_relax_info(Args A, const double *__restrict__ partial, double *__restrict__ info, int which)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= A.ncells) return;
    const Inst &I = A.inst[find_inst(A.cell_prefix, A.ninst, c)];
    double raw[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < A.nparts; ++k)
        for (int q = 0; q < 5; ++q) raw[q] += partial[((long long)c * A.nparts + k) * NQ + q];
    for (int q = 0; q < 5; ++q) raw[q] *= A.g.dV;
    Relax r;
    moments_from_raw(raw, &r);
    const double tau = which == 0 ? (I.strang ? 0.5 * I.dt : 0.0) : (I.strang ? 0.5 * I.dt : I.dt);
    const double nu = r.n * (I.omega == 0.5 ? sqrt(r.T) : pow(r.T, 1.0 - I.omega)) / I.kn;
    double *o = info + (long long)c * NINFO;
    o[0] = r.n;
    o[1] = r.V[0];
    o[2] = r.V[1];
    o[3] = r.V[2];
    o[4] = r.T;
    o[5] = nu;
    o[6] = exp(-nu * tau);
    o[7] = tau;
}

// LDS tables of one cell's Maxwellian: phi(j) = P ex[jx] ey[jy] ez[jz].
struct PhiTab {
    double e[3][NVMAX];
    double P;
};

__device__ __forceinline__ void build_phi(const Geo &g, const double *in, PhiTab &T)
{
    const int n = g.nvx + g.nvy + g.nvz;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        int a, k;
        if (t < g.nvx) { a = 0; k = t; }
        else if (t < g.nvx + g.nvy) { a = 1; k = t - g.nvx; }
        else { a = 2; k = t - g.nvx - g.nvy; }
        const double d = vnode(g, a, k) - in[1 + a];
        T.e[a][k] = exp(-d * d / in[4]);
    }
    if (threadIdx.x == 0) T.P = in[0] * pi_t_m32(in[4]);
    __syncthreads();
}

// Six sums of one cell part: A = sum mu Phi, B = sum mu Phi (v - V),
// C = sum mu Phi |v - V|^2, D = sum mu (x - Phi).
template <typename real>
__global__ void __launch_bounds__(256) k_adj_sums(Args A, const real *__restrict__ x, const real *__restrict__ mu,
                                                  const double *__restrict__ info, double *__restrict__ sums)
{
    __shared__ PhiTab T;
    const Geo &g = A.g;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int gc = L / A.vsplit, split = L % A.vsplit;
    const Inst &I = A.inst[find_inst(A.cell_prefix, A.ninst, gc)];
    const double *in = info + (long long)gc * NINFO;
    build_phi(g, in, T);
    const long long off = I.f0 + (long long)(gc - I.cell0) * g.nv;
    int z0, z1;
    chunk_bounds(g.nvz, A.vsplit, split, &z0, &z1);
    double acc[NSUM] = {0, 0, 0, 0, 0, 0};
    for (int p = threadIdx.x; p < g.npl; p += blockDim.x) {
        const int jx = p % g.nvx, jy = p / g.nvx;
        const double cx = vnode(g, 0, jx) - in[1], cy = vnode(g, 1, jy) - in[2];
        const double pxy = T.P * T.e[0][jx] * T.e[1][jy];
#pragma unroll 4
        for (int jz = z0; jz < z1; ++jz) {
            const long long i = off + (long long)jz * g.npl + p;
            const double m = (double)mu[i], xv = (double)x[i];
            const double cz = vnode(g, 2, jz) - in[3];
            const double phi = pxy * T.e[2][jz];
            const double w = m * phi;
            acc[0] += w;
            acc[1] += w * cx;
            acc[2] += w * cy;
            acc[3] += w * cz;
            acc[4] += w * (cx * cx + cy * cy + cz * cz);
            acc[5] += m * (xv - phi);
        }
    }
    block_sum_store<NSUM>(acc, sums + (long long)L * NSUM);
}

// Per-cell coefficients of the transpose of one relaxation at x,
//     R^T mu = E mu + dV (G0 + G1 vx + G2 vy + G3 vz + G4 |v|^2),
// from the six sums of the cell's parts: coef[cell] = (G0, G1, G2, G3, G4, E).
// The relaxation's dL/dKn goes to gk[cell].  One thread per cell.
constexpr int NCOEF = 8;

// Coefficients of one cell from its six sums s and relaxation data in:
// o = (G0, G1, G2, G3, G4, E, 0, 0); returns the relaxation's dL/dKn.
__device__ __forceinline__ double cell_coef(const Inst &I, const double *in, const double (&s)[NSUM], double *o)
{
    const double n = in[0], T = in[4], nu = in[5], E = in[6], tau = in[7];
    const double V[3] = {in[1], in[2], in[3]};
    // adjoints of n, V, T (dPhi/dn = Phi/n, dPhi/dV = 2 Phi (v - V)/T,
    // dPhi/dT = Phi (|v - V|^2/T^2 - 3/(2T)), dE/dn = -tau E nu/n,
    // dE/dT = -tau E (1 - omega) nu/T, dy/dE = x - Phi)
    const double Gn = (1.0 - E) * s[0] / n - tau * E * nu / n * s[5];
    const double GV[3] = {(1.0 - E) * 2.0 * s[1] / T, (1.0 - E) * 2.0 * s[2] / T, (1.0 - E) * 2.0 * s[3] / T};
    const double GT = (1.0 - E) * (s[4] / (T * T) - 1.5 * s[0] / T) - tau * E * (1.0 - I.omega) * nu / T * s[5];
    // chain to the raw sums M0 = n, M1 = n V, M2 = n (|V|^2 + 3T/2)
    const double V2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
    double G0 = Gn + GT * (2.0 / 3.0) * (V2 - 1.5 * T) / n;
    for (int a = 0; a < 3; ++a) {
        G0 -= GV[a] * V[a] / n;
        o[1 + a] = GV[a] / n - GT * (4.0 / 3.0) * V[a] / n;
    }
    o[0] = G0;
    o[4] = GT * (2.0 / 3.0) / n;
    o[5] = E;
    o[6] = 0.0;
    o[7] = 0.0;
    return tau * E * nu / I.kn * s[5];  // dE/dKn = tau E nu / Kn
}

__global__ void k_adj_coef(Args A, const double *__restrict__ info, const double *__restrict__ sums,
                           double *__restrict__ coef, double *__restrict__ gk)
{
    const int gc = blockIdx.x * blockDim.x + threadIdx.x;
    if (gc >= A.ncells) return;
    const Inst &I = A.inst[find_inst(A.cell_prefix, A.ninst, gc)];
    double s[NSUM] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < A.vsplit; ++k)
        for (int q = 0; q < NSUM; ++q) s[q] += sums[((long long)gc * A.vsplit + k) * NSUM + q];
    gk[gc] += cell_coef(I, info + (long long)gc * NINFO, s, coef + (long long)gc * NCOEF);
}

// out = R^T mu with the cell coefficients of k_adj_coef.
template <typename real>
__global__ void __launch_bounds__(256) k_adj_apply(Args A, const real *__restrict__ mu, const double *__restrict__ coef,
                                                   real *__restrict__ out)
{
    const Geo &g = A.g;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int gc = L / A.vsplit, split = L % A.vsplit;
    const Inst &I = A.inst[find_inst(A.cell_prefix, A.ninst, gc)];
    const double *G = coef + (long long)gc * NCOEF;
    const double G0 = G[0], G1 = G[1], G2 = G[2], G3 = G[3], G4 = G[4], E = G[5];
    const real *mc = mu + I.f0 + (long long)(gc - I.cell0) * g.nv;
    real *oc = out + I.f0 + (long long)(gc - I.cell0) * g.nv;
    int z0, z1;
    chunk_bounds(g.nvz, A.vsplit, split, &z0, &z1);
    const double dV = g.dV;
    for (int p = threadIdx.x; p < g.npl; p += blockDim.x) {
        const int jx = p % g.nvx, jy = p / g.nvx;
        const double vx = vnode(g, 0, jx), vy = vnode(g, 1, jy);
        const double base = G0 + G1 * vx + G2 * vy + G4 * (vx * vx + vy * vy);
#pragma unroll 4
        for (int jz = z0; jz < z1; ++jz) {
            const int i = jz * g.npl + p;
            const double vz = vnode(g, 2, jz);
            oc[i] = (real)(E * (double)mc[i] + dV * (base + G3 * vz + G4 * vz * vz));
        }
    }
}

// The last part of a reverse step in one pass per cell (one workgroup per
// cell, all its velocities): the six sums of mu against the Maxwellian of x
// and x itself, the cell's coefficients (dL/dKn into gk), and
// out = R^T mu with them; the second read of mu hits the cache.  The same
// arithmetic as k_adj_sums, k_adj_coef and k_adj_apply with one chunk per
// cell, so the same bits.
// NEXT (a reverse sweep over step records): out is lambda^n, and the pass also
// forms the six sums of the previous step's closing relaxation, of out
// against the Maxwellian of that step's streamed intermediate hn (relaxation
// data info_n) and hn itself, into sums_n -- k_adj_sums' arithmetic on
// (hn, out), so the same bits, without reading out again.
template <typename real, bool NEXT = false>
__global__ void __launch_bounds__(256) k_adj_close(Args A, const real *__restrict__ x, const real *__restrict__ mu,
                                                   const double *__restrict__ info, double *__restrict__ gk,
                                                   real *__restrict__ out, const real *__restrict__ hn,
                                                   const double *__restrict__ info_n, double *__restrict__ sums_n)
{
    __shared__ PhiTab T;
    __shared__ PhiTab Tn;
    __shared__ double sums[NSUM], G[NCOEF];
    const Geo &g = A.g;
    const int gc = xcd_remap(blockIdx.x, gridDim.x);
    const Inst &I = A.inst[find_inst(A.cell_prefix, A.ninst, gc)];
    const double *in = info + (long long)gc * NINFO;
    const double *inn = NEXT ? info_n + (long long)gc * NINFO : in;
    build_phi(g, in, T);
    if constexpr (NEXT) build_phi(g, inn, Tn);
    const long long off = I.f0 + (long long)(gc - I.cell0) * g.nv;
    double acc[NSUM] = {0, 0, 0, 0, 0, 0};
    for (int p = threadIdx.x; p < g.npl; p += blockDim.x) {
        const int jx = p % g.nvx, jy = p / g.nvx;
        const double cx = vnode(g, 0, jx) - in[1], cy = vnode(g, 1, jy) - in[2];
        const double pxy = T.P * T.e[0][jx] * T.e[1][jy];
#pragma unroll 4
        for (int jz = 0; jz < g.nvz; ++jz) {
            const long long i = off + (long long)jz * g.npl + p;
            const double m = (double)mu[i], xv = (double)x[i];
            const double cz = vnode(g, 2, jz) - in[3];
            const double phi = pxy * T.e[2][jz];
            const double w = m * phi;
            acc[0] += w;
            acc[1] += w * cx;
            acc[2] += w * cy;
            acc[3] += w * cz;
            acc[4] += w * (cx * cx + cy * cy + cz * cz);
            acc[5] += m * (xv - phi);
        }
    }
    block_sum_store<NSUM>(acc, sums);
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[NSUM];
        for (int q = 0; q < NSUM; ++q) s[q] = 0.0 + sums[q];
        gk[gc] += cell_coef(I, in, s, G);
    }
    __syncthreads();
    const double G0 = G[0], G1 = G[1], G2 = G[2], G3 = G[3], G4 = G[4], E = G[5];
    const real *mc = mu + off;
    real *oc = out + off;
    const double dV = g.dV;
    double accn[NSUM] = {0, 0, 0, 0, 0, 0};
    for (int p = threadIdx.x; p < g.npl; p += blockDim.x) {
        const int jx = p % g.nvx, jy = p / g.nvx;
        const double vx = vnode(g, 0, jx), vy = vnode(g, 1, jy);
        const double base = G0 + G1 * vx + G2 * vy + G4 * (vx * vx + vy * vy);
        double cxn = 0.0, cyn = 0.0, pxyn = 0.0;
        if constexpr (NEXT) {
            cxn = vnode(g, 0, jx) - inn[1];
            cyn = vnode(g, 1, jy) - inn[2];
            pxyn = Tn.P * Tn.e[0][jx] * Tn.e[1][jy];
        }
#pragma unroll 4
        for (int jz = 0; jz < g.nvz; ++jz) {
            const int i = jz * g.npl + p;
            const double vz = vnode(g, 2, jz);
            const real r = (real)(E * (double)mc[i] + dV * (base + G3 * vz + G4 * vz * vz));
            oc[i] = r;
            if constexpr (NEXT) {
                const double m = (double)r, xv = (double)hn[off + i];
                const double cz = vnode(g, 2, jz) - inn[3];
                const double phi = pxyn * Tn.e[2][jz];
                const double w = m * phi;
                accn[0] += w;
                accn[1] += w * cxn;
                accn[2] += w * cyn;
                accn[3] += w * cz;
                accn[4] += w * (cxn * cxn + cyn * cyn + cz * cz);
                accn[5] += m * (xv - phi);
            }
        }
    }
    if constexpr (NEXT) block_sum_store<NSUM>(accn, sums_n + (long long)gc * NSUM);
}

// ---------------------------------------------------------------- streaming
//
// The transposed minmod streaming step in gather form, at the branches of
// the forward step.  In the upwind frame of one direction, u_m = G(i + s m)
// (s the sign of the velocity component, G the relaxed streaming input),
// beta(m) the branch of the slope at u_m (0: zero, a: forward difference
// u_{m+1} - u_m, b: backward difference u_m - u_{m-1}), C = |Courant number|
// and k = (1 - C)/2 (0 without limiter), output i receives from this
// direction
//   C (mu(1) - mu(0)) + C k ( mu(0) A0 + mu(1) A1 - mu(2) [b1 = b] - mu(-1) [b-1 = a] ),
//   A0 = [b0 = a] - [b0 = b] + [b-1 = a],   A1 = [b1 = b] - [b0 = a] + [b0 = b],
// plus mu(0) once for all directions; mu(m) is the adjoint at i + s m (zero
// outside a non-periodic domain).  Here mu = R_b^T(lambda^{n+1}) is formed on
// the fly from lambda^{n+1} and each slot cell's relaxation coefficients.
// The branches are not recomputed: the step's own streaming pass, run in its
// recording form, stored per element and direction beta(-1) and beta(0) as
// it took them (one byte, x in bits 0-3, y in bits 4-7), and beta(1) is the
// beta(0) that the pass recorded at i + s.  Where i + s lies outside the
// domain, mu(1) = mu(2) = 0 and beta(1) does not enter.
//
// Slots: 0 centre; 1 + 8*d + 4*si + m for direction d (0 x, 1 y), si = 0 for
// s = +1, 1 for s = -1, m = 0..3 for k = -2, -1, +1, +2.
struct AdjSlots {
    int cell[17], par[17], mucell[17];
};

// Adjoint input at a slot: mu = c0 lambda + l1 + (g3 + g4 vz) vz, all zero at a ghost.
template <typename real, int VEC>
struct MuTap {
    using V = vec_t<real, VEC>;
    uint32_t off;
    real c0, g3, g4;
    V l1;
    __device__ __forceinline__ V load(const real *base, uint32_t zoff) const { return ld<V>(base, off + zoff); }
    __device__ __forceinline__ V value(V lam, real vz) const { return c0 * lam + (l1 + (g3 + g4 * vz) * vz); }
};

template <typename real, int VEC>
__device__ __forceinline__ MuTap<real, VEC> mu_tap(const Geo &g, const double *cf, int mucell, int own, int p0,
                                                   int jx0, double vy)
{
    MuTap<real, VEC> t;
    const bool in = mucell >= 0;
    t.off = (uint32_t)(((long long)(in ? mucell : own) * g.nv + p0) * sizeof(real));
    const double dV = g.dV;
    t.c0 = in ? (real)cf[5] : (real)0;
    t.g3 = in ? (real)(dV * cf[3]) : (real)0;
    t.g4 = in ? (real)(dV * cf[4]) : (real)0;
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
        const double vx = vnode(g, 0, jx0 + k);
        t.l1[k] = in ? (real)(dV * (cf[0] + cf[1] * vx + cf[2] * vy + cf[4] * (vx * vx + vy * vy))) : (real)0;
    }
    return t;
}

// One direction's contribution (see above) from the branch codes bm1, b0, b1
// of the slopes at i - s, i, i + s (mm_code: 0 zero, 1 a, 2 b).  The codes
// enter only through 0/1 indicators, so the adjoint is a short sum of exact
// integer multiples of the mu values.
template <typename real>
__device__ __forceinline__ real direction_adjoint(uint32_t bm1, uint32_t b0, uint32_t b1, real mm1, real m0, real m1,
                                                  real m2, real C, real k)
{
    const real am1 = bm1 == 1u ? (real)1 : (real)0;
    const real a0 = b0 == 1u ? (real)1 : (real)0, c0 = b0 == 2u ? (real)1 : (real)0;
    const real c1 = b1 == 2u ? (real)1 : (real)0;
    const real A0 = a0 - c0 + am1;
    const real A1 = c1 - a0 + c0;
    const real lim = m0 * A0 + m1 * A1 - c1 * m2 - am1 * mm1;
    return C * (m1 - m0) + C * k * lim;
}

// Lane tasks as in the forward kernel: VEC consecutive jx of one v_x sign at
// one jy, residue zr of jz modulo A.zr.  Per element the kernel reads its
// branch byte, the branch bytes of its two downwind neighbours (x, y) and the
// 7 (1D: 4) lambda taps.  The block of a wall-adjacent cavity cell also
// accumulates, per wall it feeds, S_gamma = sum gamma Phi_W and
// S_gamma' = sum gamma dPhi_W/dT_w over the emitted velocities, where
// gamma = C mu(0) + C k [b0 = b] (mu(0) - mu(1)) is the adjoint of that
// velocity's emitted ghost value per unit n_W; the emitted ghosts' table
// entries sit in dynamic LDS (2 per direction: the k = -1 slots of both
// signs).  ZU (one jz residue, all lanes of a wave on one plane): the plane
// offset goes into the scalar base of the lambda loads.
template <typename real, int DIM, int VEC, bool ZU>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, 256),
                               amdgpu_waves_per_eu(sizeof(real) == 4 && VEC == 1 ? 4 : 1)))
    k_adj_stream(Args A, const unsigned char *__restrict__ rec, const real *__restrict__ params,
                 const real *__restrict__ lam, const double *__restrict__ coef, real *__restrict__ out,
                 double *__restrict__ wsum)
{
    using V = vec_t<real, VEC>;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NSL = DIM == 1 ? 9 : 17;
    real *sp = reinterpret_cast<real *>(smem);  // [2 d + si][entry]: the k = -1 slots' entries
    __shared__ AdjSlots S;
    __shared__ double cf[NSL][NCOEF];
    __shared__ double vzs[NVMAX];  // v_z of every plane (wave-uniform reads)
    const Geo &g = A.g;
    const int Lq = xcd_remap(blockIdx.x, gridDim.x);
    const int gq = Lq / A.vsplit, split = Lq % A.vsplit;
    const Inst &I = A.inst[find_inst(A.cell_prefix, A.ninst, gq)];
    const int c = strip_cell(I, gq - I.cell0), ix = c % I.nx, iy = c / I.nx;
    const int gc = I.cell0 + c;
    const int L = gc * A.vsplit + split;  // (cell, chunk) index of the wall sums
    const bool per = I.kind == KIND_PER1 || I.kind == KIND_PER2;
    for (int k = threadIdx.x; k < g.nvz; k += blockDim.x) vzs[k] = vnode(g, 2, k);
    if (threadIdx.x < NSL) {
        const int sl = threadIdx.x;
        int cell = c, par = gc, mc = c;
        if (sl > 0) {
            const int d = (sl - 1) / 8, r = (sl - 1) % 8, si = r / 4, m = r % 4;
            const int sgn = si == 0 ? 1 : -1, k = m == 0 ? -2 : m == 1 ? -1 : m == 2 ? 1 : 2;
            const int N = d == 0 ? I.nx : I.ny;
            const int pos = (d == 0 ? ix : iy) + sgn * k;
            resolve_slot(I, d, ix, iy, 0, sgn * k, sgn, c, &cell, &par);
            mc = ((pos >= 0 && pos < N) || per) ? cell : -1;
        }
        S.cell[sl] = cell;
        S.par[sl] = par;
        S.mucell[sl] = mc;
    }
    __syncthreads();
    const bool cav = I.kind == KIND_CAVITY;
    // walls whose emitted ghosts this cell's stencils read: 0 left, 1 right, 2 bottom, 3 top
    const bool wl = cav && ix == 0, wr = cav && ix == I.nx - 1, wb = cav && iy == 0, wt = cav && iy == I.ny - 1;
    const bool wall = wl || wr || wb || wt;
    if (wall)
        for (int t = threadIdx.x; t < 2 * DIM * g.pe; t += blockDim.x) {
            const int q = t / g.pe, o = t - q * g.pe;  // q = 2 d + si
            sp[t] = params[(long long)S.par[1 + 8 * (q >> 1) + 4 * (q & 1) + 1] * g.pe + o];
        }
    for (int t = threadIdx.x; t < NSL * NCOEF; t += blockDim.x) {
        const int sl = t / NCOEF, q = t - sl * NCOEF;
        cf[sl][q] = S.mucell[sl] >= 0 ? coef[(long long)(I.cell0 + S.mucell[sl]) * NCOEF + q] : 0.0;
    }
    __syncthreads();

    const real *lb = lam + I.f0;
    const unsigned char *rb = rec + I.f0;
    real *ob = out + I.f0;
    const uint32_t ibytes = (uint32_t)((long long)I.ncell * g.nv * sizeof(real));  // below 2^32 (init)
    const __amdgpu_buffer_rsrc_t lrs = make_rsrc(lb, ibytes);
    // the branch record of the instance as a buffer too (one byte per element)
    const __amdgpu_buffer_rsrc_t brs = make_rsrc(rb, (uint32_t)((long long)I.ncell * g.nv));
    const uint32_t out0 = (uint32_t)((long long)c * g.nv * sizeof(real));
    const uint32_t rown = (uint32_t)c * (uint32_t)g.nv;  // element index of (cell, 0) in the instance
    int z0, z1;
    chunk_bounds(g.nvz, A.vsplit, split, &z0, &z1);
    const bool lim = I.minmod != 0;
    const int ngx = g.nvx / VEC, ngroups = ngx * g.nvy, ntask = ngroups * A.zr;
    const uint32_t zstep = (uint32_t)(g.npl * sizeof(real));
    const double itw = 1.0 / I.tw;
    // this thread's wall sums, accumulated in LDS (wall cells only; an LDS
    // address per wall instead of registers indexed by the lane's wall)
    __shared__ double wsl[NWALL][256];
    if (wall)
        for (int q = 0; q < NWALL; ++q) wsl[q][threadIdx.x] = 0.0;

    for (int task = threadIdx.x; task < ntask; task += blockDim.x) {
        const int pg = task % ngroups, zr = ZU ? 0 : task / ngroups;
        const int jy = pg / ngx, jx0 = (pg - jy * ngx) * VEC;
        const int p0 = jy * g.nvx + jx0;
        V Cx, kx;
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            Cx[k] = (real)(fabs(vnode(g, 0, jx0 + k)) * I.cx);
            kx[k] = lim ? (real)0.5 * ((real)1 - Cx[k]) : (real)0;
        }
        const double vy = vnode(g, 1, jy);
        const int sx = vnode(g, 0, jx0) > 0.0 ? 0 : 1;
        const int bx = 1 + 4 * sx;
        const MuTap<real, VEC> mc = mu_tap<real, VEC>(g, cf[0], S.mucell[0], c, p0, jx0, vy);
        const MuTap<real, VEC> mxb = mu_tap<real, VEC>(g, cf[bx + 1], S.mucell[bx + 1], c, p0, jx0, vy);
        const MuTap<real, VEC> mxd = mu_tap<real, VEC>(g, cf[bx + 2], S.mucell[bx + 2], c, p0, jx0, vy);
        const MuTap<real, VEC> mxe = mu_tap<real, VEC>(g, cf[bx + 3], S.mucell[bx + 3], c, p0, jx0, vy);
        // branch records: this element's, and its downwind x (and y) neighbour's
        // (element offsets in the instance's record)
        const uint32_t rc = rown + (uint32_t)p0;
        const uint32_t rx = (uint32_t)S.cell[bx + 2] * (uint32_t)g.nv + (uint32_t)p0;
        uint32_t ry = rc;
        // emitted x ghosts read by this cell: its own wall entry (slot k = -1)
        const bool emx = ((sx == 0 && wl) || (sx == 1 && wr));
        const int wx = sx == 0 ? 0 : 1;
        MuTap<real, VEC> myb, myd, mye;
        V Cy = 0, ky = 0;
        int sy = 0;
        bool emy = false;
        int wy = 2;
        if constexpr (DIM == 2) {
            sy = vy > 0.0 ? 0 : 1;
            const int by = 9 + 4 * sy;
            const real cy = (real)(fabs(vy) * I.cy);
            Cy = cy;
            ky = lim ? (real)0.5 * ((real)1 - cy) : (real)0;
            myb = mu_tap<real, VEC>(g, cf[by + 1], S.mucell[by + 1], c, p0, jx0, vy);
            myd = mu_tap<real, VEC>(g, cf[by + 2], S.mucell[by + 2], c, p0, jx0, vy);
            mye = mu_tap<real, VEC>(g, cf[by + 3], S.mucell[by + 3], c, p0, jx0, vy);
            ry = (uint32_t)S.cell[by + 2] * (uint32_t)g.nv + (uint32_t)p0;
            emy = (sy == 0 && wb) || (sy == 1 && wt);
            wy = sy == 0 ? 2 : 3;
        }
        // The 7 (1D: 4) lambda taps and the branch bytes of one plane, loaded
        // one plane ahead of their use (software pipeline; the prefetch after
        // the lane's last plane re-reads it).
        constexpr int NL = DIM == 1 ? 4 : 7;
        using B = vec_t<uint32_t, VEC>;
        auto load_plane = [&](int j, V (&Lm)[NL], B (&Rc)[3]) {
            const uint32_t zo = (uint32_t)j * zstep;
            // under ZU the plane offset is wave-uniform: buffer loads take it as
            // their scalar offset next to the tap's per-lane offset
            const uint32_t zb = ZU ? __builtin_amdgcn_readfirstlane(zo) : 0u;
            auto ll = [&](const auto &tp) -> V {
                if constexpr (ZU) return buf_ld<V>(lrs, tp.off, zb);
                else return tp.load(lb, zo);
            };
            Lm[0] = ll(mc);
            Lm[1] = ll(mxb);
            Lm[2] = ll(mxd);
            Lm[3] = ll(mxe);
            if constexpr (DIM == 2) {
                Lm[4] = ll(myb);
                Lm[5] = ll(myd);
                Lm[6] = ll(mye);
            }
            const uint32_t zi = (uint32_t)j * (uint32_t)g.npl;
            if constexpr (ZU) {
                const uint32_t zs = __builtin_amdgcn_readfirstlane(zi);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    Rc[0][e] = __builtin_amdgcn_raw_buffer_load_b8(brs, (int)(rc + e), (int)zs, 0);
                    Rc[1][e] = __builtin_amdgcn_raw_buffer_load_b8(brs, (int)(rx + e), (int)zs, 0);
                    Rc[2][e] = DIM == 2 ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(brs, (int)(ry + e), (int)zs, 0)
                                        : 0u;
                }
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    Rc[0][e] = rb[rc + zi + e];
                    Rc[1][e] = rb[rx + zi + e];
                    Rc[2][e] = DIM == 2 ? (uint32_t)rb[ry + zi + e] : 0u;
                }
            }
        };
        int jz = z0 + zr;
        if (jz >= z1) continue;
        const int zlast = z1 - 1 - ((z1 - 1 - jz) % A.zr);  // last plane of this lane's residue
        V Lm[NL];
        B R[3];
        load_plane(jz, Lm, R);
        for (; jz < z1; jz += A.zr) {
            V Ln[NL];
            B Rn[3];
            load_plane(min(jz + A.zr, zlast), Ln, Rn);
            const uint32_t zo = (uint32_t)jz * zstep;
            const double vzd = vzs[jz];
            const real vz = (real)vzd;
            const V m0 = mc.value(Lm[0], vz);
            V r = m0;
            {
                const V mm1 = mxb.value(Lm[1], vz), m1 = mxd.value(Lm[2], vz);
                const V m2 = mxe.value(Lm[3], vz);
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    r[e] += direction_adjoint<real>(R[0][e] & 3u, (R[0][e] >> 2) & 3u, (R[1][e] >> 2) & 3u, mm1[e],
                                                    m0[e], m1[e], m2[e], Cx[e], kx[e]);
                if (emx) {
                    const real *E = sp + sx * g.pe;
                    const double nw = (double)E[1];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const bool b0b = ((R[0][e] >> 2) & 3u) == 2u;
                        const double C = (double)Cx[e];
                        const double gam = C * (double)m0[e] + C * (double)kx[e] * b0b * ((double)m0[e] - (double)m1[e]);
                        const double phiw = (double)E[g.tx1 + jx0 + e] * (double)E[g.ty1 + jy] *
                                            (double)E[g.tz + 2 * jz] / nw;
                        const double vx = vnode(g, 0, jx0 + e);
                        const double c2 = vx * vx + vy * vy + vzd * vzd;
                        wsl[2 * wx][threadIdx.x] += gam * phiw;
                        wsl[2 * wx + 1][threadIdx.x] += gam * phiw * (c2 * itw * itw - 1.5 * itw);
                    }
                }
            }
            if constexpr (DIM == 2) {
                const V mm1 = myb.value(Lm[4], vz), m1 = myd.value(Lm[5], vz);
                const V m2 = mye.value(Lm[6], vz);
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    r[e] += direction_adjoint<real>((R[0][e] >> 4) & 3u, (R[0][e] >> 6) & 3u, (R[2][e] >> 6) & 3u,
                                                    mm1[e], m0[e], m1[e], m2[e], Cy[e], ky[e]);
                if (emy) {
                    const real *E = sp + (2 + sy) * g.pe;
                    const double nw = (double)E[1];
                    const double uw = wy == 3 ? I.uw : 0.0;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const bool b0b = ((R[0][e] >> 6) & 3u) == 2u;
                        const double C = (double)Cy[e];
                        const double gam = C * (double)m0[e] + C * (double)ky[e] * b0b * ((double)m0[e] - (double)m1[e]);
                        const double phiw = (double)E[g.tx1 + jx0 + e] * (double)E[g.ty1 + jy] *
                                            (double)E[g.tz + 2 * jz] / nw;
                        const double ux = vnode(g, 0, jx0 + e) - uw;
                        const double c2 = ux * ux + vy * vy + vzd * vzd;
                        wsl[2 * wy][threadIdx.x] += gam * phiw;
                        wsl[2 * wy + 1][threadIdx.x] += gam * phiw * (c2 * itw * itw - 1.5 * itw);
                    }
                }
            }
            *reinterpret_cast<V *>(reinterpret_cast<char *>(ob) + out0 + zo + (uint32_t)(p0 * sizeof(real))) = r;
#pragma unroll
            for (int t = 0; t < NL; ++t) Lm[t] = Ln[t];
#pragma unroll
            for (int t = 0; t < 3; ++t) R[t] = Rn[t];
        }
    }
    if (wall) {
        double ws[NWALL];
#pragma unroll
        for (int q = 0; q < NWALL; ++q) ws[q] = wsl[q][threadIdx.x];
        block_sum_store<NWALL>(ws, wsum + (long long)L * NWALL);
    }
}

// Per-cell totals of the partial moment sums (the step record keeps them
// independent of the chunk count): tot[c][q] = sum over the nparts slots in
// slot order, as the table preparation adds them.  One thread per (cell, q).
__global__ void k_part_totals(Args A, const double *__restrict__ partial, double *__restrict__ tot)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)A.ncells * NQ) return;
    const long long c = t / NQ;
    const int q = (int)(t - c * NQ);
    double v = 0.0;
    for (int k = 0; k < A.nparts; ++k) v += partial[(c * A.nparts + k) * NQ + q];
    tot[t] = v;
}

// The inverse for the current chunk count: slot 0 holds the total, the
// others zero (so every consumer's slot sum is the total again, exactly).
__global__ void k_part_restore(Args A, const double *__restrict__ tot, double *__restrict__ partial)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)A.ncells * A.nparts * NQ) return;
    const long long slot = t / NQ;
    const int q = (int)(t - slot * NQ);
    const long long c = slot / A.nparts;
    partial[t] = slot - c * A.nparts == 0 ? tot[c * NQ + q] : 0.0;
}

// Per (instance, wall): D = sum_em (v.n) Phi_W and D' = dD/dT_w over the
// emitted velocities, Phi_W the unit-density wall Maxwellian of the wall's
// first table entry.  One workgroup per (instance, wall); 0 for non-cavities.
template <typename real>
__global__ void __launch_bounds__(256) k_adj_wall_flux(Args A, const real *__restrict__ params, double *__restrict__ dw)
{
    __shared__ double red[4][2];
    const Geo &g = A.g;
    const int ii = blockIdx.x / 4, w = blockIdx.x % 4;
    const Inst &I = A.inst[ii];
    double D = 0.0, Dp = 0.0;
    if (I.kind == KIND_CAVITY) {
        const int axis = w < 2 ? 0 : 1;
        const double sgn = (w == 0 || w == 2) ? 1.0 : -1.0;
        const int off = w == 0 ? 0 : w == 1 ? I.ny : w == 2 ? 2 * I.ny : 2 * I.ny + I.nx;
        const real *E = params + (long long)(I.pseudo0 + off) * g.pe;
        const double nW = (double)E[1];
        const double uw = w == 3 ? I.uw : 0.0;
        for (int p = threadIdx.x; p < g.npl; p += blockDim.x) {
            const int jx = p % g.nvx, jy = p / g.nvx;
            const double vx = vnode(g, 0, jx), vy = vnode(g, 1, jy);
            const double vn = sgn * (axis == 0 ? vx : vy);
            if (!(vn > 0.0)) continue;
            const double exy = (double)E[g.tx1 + jx] * (double)E[g.ty1 + jy] / nW;
            for (int jz = 0; jz < g.nvz; ++jz) {
                const double vz = vnode(g, 2, jz);
                const double phiw = exy * (double)E[g.tz + 2 * jz];
                const double c2 = (vx - uw) * (vx - uw) + vy * vy + vz * vz;
                D += vn * phiw;
                Dp += vn * phiw * (c2 / (I.tw * I.tw) - 1.5 / I.tw);
            }
        }
    }
    D = wave_sum(D);
    Dp = wave_sum(Dp);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { red[wv][0] = D; red[wv][1] = Dp; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double d = 0.0, dp = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { d += red[k][0]; dp += red[k][1]; }
        dw[2 * blockIdx.x] = d;
        dw[2 * blockIdx.x + 1] = dp;
    }
}

// Transpose of the wall ghost construction for one wall-adjacent cell:
// n_W-bar = S_gamma, dL/dT_w += n_W (S_gamma' - S_gamma D'/D), and
// abar(j) += n_W-bar |v.n| / D for every velocity arriving at the wall
// (n_W = incident flux / D).  One workgroup per cell of the cavity perimeters
// (global cell ids in `cells`).
template <typename real>
__global__ void __launch_bounds__(256) k_adj_wall(Args A, const int *__restrict__ cells, const real *__restrict__ params,
                                                  const double *__restrict__ dw, const double *__restrict__ wsum,
                                                  real *__restrict__ out, double *__restrict__ gt)
{
    __shared__ double coef[4], tgrad[4];  // n_W-bar / D and the T_w term per wall (0 off the wall)
    const Geo &g = A.g;
    const int gc = cells[blockIdx.x];
    const int ii = find_inst(A.cell_prefix, A.ninst, gc);
    const Inst &I = A.inst[ii];
    const int c = gc - I.cell0, ix = c % I.nx, iy = c / I.nx;
    const bool on[4] = {ix == 0, ix == I.nx - 1, iy == 0, iy == I.ny - 1};
    if (threadIdx.x < 4) {
        const int w = threadIdx.x;
        double cw = 0.0, tg = 0.0;
        if (on[w]) {
            const int pos = w < 2 ? iy : ix;
            const int off = w == 0 ? 0 : w == 1 ? I.ny : w == 2 ? 2 * I.ny : 2 * I.ny + I.nx;
            const double nW = (double)params[(long long)(I.pseudo0 + off + pos) * g.pe + 1];
            const double d = dw[2 * (4 * ii + w)], dp = dw[2 * (4 * ii + w) + 1];
            double s = 0.0, sp = 0.0;
            for (int k = 0; k < A.vsplit; ++k) {
                s += wsum[((long long)gc * A.vsplit + k) * NWALL + 2 * w];
                sp += wsum[((long long)gc * A.vsplit + k) * NWALL + 2 * w + 1];
            }
            cw = s / d;
            tg = nW * (sp - s * dp / d);
        }
        coef[w] = cw;
        tgrad[w] = tg;
    }
    __syncthreads();
    if (threadIdx.x == 0) gt[gc] += ((tgrad[0] + tgrad[1]) + tgrad[2]) + tgrad[3];
    real *ob = out + I.f0 + (long long)c * g.nv;
    for (int p = threadIdx.x; p < g.npl; p += blockDim.x) {
        const int jx = p % g.nvx, jy = p / g.nvx;
        const double vx = vnode(g, 0, jx), vy = vnode(g, 1, jy);
        double add = 0.0;
        if (on[0] && vx < 0.0) add += coef[0] * (-vx);
        if (on[1] && vx > 0.0) add += coef[1] * vx;
        if (on[2] && vy < 0.0) add += coef[2] * (-vy);
        if (on[3] && vy > 0.0) add += coef[3] * vy;
        if (add != 0.0)
            for (int jz = 0; jz < g.nvz; ++jz) {
                const int i = jz * g.npl + p;
                ob[i] = (real)((double)ob[i] + add);
            }
    }
}

__global__ void k_fill(double *__restrict__ x, long long n, double v)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// Per-instance parameter gradients from the per-cell contributions, one
// workgroup per instance (fixed-order strided sums and tree, so the result
// does not depend on timing): grad[inst][0] += dL/dKn, [1] += dL/dT_w.
__global__ void __launch_bounds__(256) k_grad_reduce(Args A, const double *__restrict__ gk,
                                                     const double *__restrict__ gt, double *__restrict__ grad)
{
    __shared__ double red[2][256];
    const int i = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int c = A.cell_prefix[i] + threadIdx.x; c < A.cell_prefix[i + 1]; c += blockDim.x) {
        a += gk[c];
        b += gt[c];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        grad[2 * i] += red[0][0];
        grad[2 * i + 1] += red[1][0];
    }
}

// ---------------------------------------------------------------- lid shear

// Per top-row cell of a cavity: Sin = sum_{vy>0} vx vy f, N = sum_{vy>0} vy f.
template <typename real>
__global__ void __launch_bounds__(256) k_lid_sums(Args A, const real *__restrict__ f, double *__restrict__ out)
{
    const Geo &g = A.g;
    const int gc = blockIdx.x;
    const Inst &I = A.inst[find_inst(A.cell_prefix, A.ninst, gc)];
    const int c = gc - I.cell0;
    double acc[2] = {0.0, 0.0};
    if (I.kind == KIND_CAVITY && c / I.nx == I.ny - 1) {
        const real *fc = f + I.f0 + (long long)c * g.nv;
        for (long long j = threadIdx.x; j < g.nv; j += blockDim.x) {
            const int jx = (int)(j % g.nvx), jy = (int)((j / g.nvx) % g.nvy);
            const double vx = vnode(g, 0, jx), vy = vnode(g, 1, jy);
            if (vy > 0.0 && (!g.red || j < g.npl)) {  // reduced: the g plane carries mass
                acc[0] += vx * vy * (double)fc[j];
                acc[1] += vy * (double)fc[j];
            }
        }
    }
    block_sum_store<2>(acc, out + 2 * (long long)gc);
}

// Lid Maxwellian sums of one instance (one 64-thread wave):
// K = sum_{vy<0} vx vy Phi_W, D = sum_{vy<0} |vy| Phi_W, and their T_w derivatives.
__device__ __forceinline__ void lid_constants(const Geo &g, const Inst &I, double *K, double *D, double *Kp,
                                              double *Dp)
{
    double k = 0, d = 0, kp = 0, dp = 0;
    const double pw = pi_t_m32(I.tw);
    for (long long j = threadIdx.x & 63; j < g.nv; j += 64) {
        const int jx = (int)(j % g.nvx), jy = (int)((j / g.nvx) % g.nvy), jz = (int)(j / g.npl);
        const double vx = vnode(g, 0, jx), vy = vnode(g, 1, jy), vz = vnode(g, 2, jz);
        if (g.red && jz > 0) continue;  // reduced: the g plane carries mass and momentum
        if (vy < 0.0) {
            const double c2 = g.red ? (vx - I.uw) * (vx - I.uw) + vy * vy
                                    : (vx - I.uw) * (vx - I.uw) + vy * vy + vz * vz;
            const double phi = pw * exp(-c2 / I.tw) * (g.red ? zfactor(g, 0, 0.0, I.tw) : 1.0);
            const double dphi = phi * (c2 / (I.tw * I.tw) - 1.5 / I.tw);
            k += vx * vy * phi;
            d += -vy * phi;
            kp += vx * vy * dphi;
            dp += -vy * dphi;
        }
    }
    *K = wave_sum(k);
    *D = wave_sum(d);
    *Kp = wave_sum(kp);
    *Dp = wave_sum(dp);
}

// Loss per instance: L = sum_i dx dV (Sin_i + N_i K / D); one wave per instance.
__global__ void __launch_bounds__(64) k_lid_finish(Args A, const double *__restrict__ sums, double *__restrict__ L,
                                                   double *__restrict__ grad)
{
    const int i = blockIdx.x;
    const Inst &I = A.inst[i];
    if (I.kind != KIND_CAVITY) {
        if (threadIdx.x == 0 && L) L[i] = 0.0;
        return;
    }
    double K, D, Kp, Dp;
    lid_constants(A.g, I, &K, &D, &Kp, &Dp);
    if (threadIdx.x == 0) {
        double l = 0.0, nsum = 0.0;
        for (int x = 0; x < I.nx; ++x) {
            const long long gc = I.cell0 + (long long)(I.ny - 1) * I.nx + x;
            l += sums[2 * gc] + sums[2 * gc + 1] * K / D;
            nsum += sums[2 * gc + 1];
        }
        const double w = I.dx * A.g.dV;
        if (L) L[i] = w * l;
        if (grad) grad[2 * i + 1] += w * nsum * (Kp / D - K * Dp / (D * D));
    }
}

// Seed of the reverse sweep: lam = dL/df (zero outside the top rows).
template <typename real>
__global__ void __launch_bounds__(256) k_lid_seed(Args A, real *__restrict__ lam)
{
    __shared__ double KD;
    const Geo &g = A.g;
    const int gc = blockIdx.x;
    const Inst &I = A.inst[find_inst(A.cell_prefix, A.ninst, gc)];
    const int c = gc - I.cell0;
    real *lc = lam + I.f0 + (long long)c * g.nv;
    const bool top = I.kind == KIND_CAVITY && c / I.nx == I.ny - 1;
    if (top && threadIdx.x < 64) {
        double K, D, Kp, Dp;
        lid_constants(g, I, &K, &D, &Kp, &Dp);
        if (threadIdx.x == 0) KD = K / D;
    }
    __syncthreads();
    const double w = I.dx * g.dV;
    for (long long j = threadIdx.x; j < g.nv; j += blockDim.x) {
        double v = 0.0;
        if (top) {
            const int jx = (int)(j % g.nvx), jy = (int)((j / g.nvx) % g.nvy);
            const double vx = vnode(g, 0, jx), vy = vnode(g, 1, jy);
            if (vy > 0.0) v = w * (vx * vy + vy * KD);
        }
        lc[j] = (real)v;
    }
}

}  // namespace bgk
