// Device kernels of liblbe (gfx950, FP64 state).
//
// One RK stage of every instance is two launches:
//   k_node  - per-node coefficients from the moment sums of the stage input (eqs. (macro_def),
//             (fm), (chi), (viscosity)-(tau), (prandtl)), 4th-order radial gradients (Sec. III),
//             the discrete equilibrium factors (Sec. III.C) and, in two extra blocks, the wall
//             densities of diffuse reflection (zero net mass flux through each wall);
//   k_stage - one workgroup per (node, instance): the node's velocity plane is staged in LDS
//             for the momentum-derivative contractions (eqs. (force1)/(force2)); each lane
//             takes velocities v = lane, lane + 256, ... (coalesced), evaluates WENO-5 fluxes
//             at both faces of the cell (flux form of Sec. II.B/II.C), the inertial terms,
//             Shakhov + J1 collision (eqs. (j0), (j1)), combines the TVD-RK3 stage and stores,
//             and the workgroup reduces the moment sums of the stored plane (no atomics, fixed
//             order, so runs are bitwise reproducible).
#include <hip/hip_runtime.h>

#include <cmath>

#include "lbe_equilibrium.h"
#include "lbe_internal.h"

namespace lbe {

constexpr int kBlock = 256;
constexpr int kNodeChunk = 32;  // nodes per node-kernel workgroup
constexpr int kHalo = 4;        // gradient stencils reach 4 nodes (one-sided at the walls)
constexpr int kMaxNr = 1024;    // largest radial grid (node-kernel LDS)

// ------------------------------------------------------------------ helpers

__device__ inline double weno5(double a, double b, double c, double d, double e)
{
    // Jiang-Shu WENO-5 reconstruction at the downwind face of c from (a, b, c, d, e) ordered
    // along the upwind direction; smoothness indicators with epsilon = 1e-6, power 2.
    const double eps = 1e-6;
    const double q0 = (2 * a - 7 * b + 11 * c) * (1.0 / 6);
    const double q1 = (-b + 5 * c + 2 * d) * (1.0 / 6);
    const double q2 = (2 * c + 5 * d - e) * (1.0 / 6);
    const double t0 = a - 2 * b + c, s0 = a - 4 * b + 3 * c;
    const double t1 = b - 2 * c + d, s1 = b - d;
    const double t2 = c - 2 * d + e, s2 = 3 * c - 4 * d + e;
    const double b0 = (13.0 / 12) * t0 * t0 + 0.25 * s0 * s0;
    const double b1 = (13.0 / 12) * t1 * t1 + 0.25 * s1 * s1;
    const double b2 = (13.0 / 12) * t2 * t2 + 0.25 * s2 * s2;
    const double e0 = eps + b0, e1 = eps + b1, e2 = eps + b2;
    // alpha_k = d_k / (eps + beta_k)^2, written over the common denominator (e0 e1 e2)^2
    const double p01 = e0 * e1, p02 = e0 * e2, p12 = e1 * e2;
    const double a0 = 0.1 * p12 * p12, a1 = 0.6 * p02 * p02, a2 = 0.3 * p01 * p01;
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// Loads and stores through explicit global (address space 1) pointers: generic pointers
// would compile to flat accesses, whose completion is tracked together with LDS traffic, so a
// prefetch would stall the next LDS wait.
typedef __attribute__((address_space(1))) const double gcdouble;
typedef __attribute__((address_space(1))) double gdouble;
__device__ inline double gload(const double* p) { return *(gcdouble*)p; }
__device__ inline void gstore(double* p, double v) { *(gdouble*)p = v; }

template <typename T>
__device__ inline T wave_sum(T v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum NV values per lane over the workgroup; result valid in red[0..NV) after the call.
template <int NV>
__device__ inline void block_sum(double* vals, double* red /* LDS, >= NV * 4 */)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        double s = wave_sum(vals[k]);
        if (lane == 0) red[k * 4 + wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int k = threadIdx.x;
        red[k * 4 + 0] = ((red[k * 4 + 0] + red[k * 4 + 1]) + red[k * 4 + 2]) + red[k * 4 + 3];
    }
    __syncthreads();
}

// Conversion of the shifted moment sums of one node to n, u, T, q, P (eqs. (macro_def)).
struct Macro {
    double n, u[3], T, q[3], P01;
};

__device__ inline Macro macro_from_sums(const double* m)
{
    Macro o;
    const double S0 = m[MF_S0];
    const double S1[3] = {m[MF_S1X], m[MF_S1Y], m[MF_S1Z]};
    const double S2[3][3] = {{m[MF_SXX], m[MF_SXY], m[MF_SXZ]}, {m[MF_SXY], m[MF_SYY], m[MF_SYZ]},
                             {m[MF_SXZ], m[MF_SYZ], m[MF_SZZ]}};
    const double S3[3] = {m[MF_S3X], m[MF_S3Y], m[MF_S3Z]};
    const double c[3] = {m[MF_CX], m[MF_CY], m[MF_CZ]};
    o.n = S0;
    double d[3];
    for (int a = 0; a < 3; a++) {
        d[a] = S1[a] / S0;
        o.u[a] = c[a] + d[a];
    }
    const double tr = S2[0][0] + S2[1][1] + S2[2][2];
    const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    o.T = (tr - (S1[0] * d[0] + S1[1] * d[1] + S1[2] * d[2])) / (3 * S0);
    for (int a = 0; a < 3; a++) {
        const double S2d = S2[a][0] * d[0] + S2[a][1] * d[1] + S2[a][2] * d[2];
        o.q[a] = 0.5 * (S3[a] - d[a] * tr - 2 * S2d + 2 * dd * d[a] * S0);
    }
    o.P01 = S2[0][1] - S1[0] * d[1];
    return o;
}

// Moment sums of node i summed over the velocity slices (fixed order); the shift is common.
__device__ inline void node_sums(const DevInstance& I, int i, double* m)
{
    const double* b = I.mom + (size_t)i * I.nslices * kMomStride;
    for (int k = 0; k < kMomStride; k++) m[k] = b[k];
    for (int s = 1; s < I.nslices; s++)
        for (int k = 0; k < 13; k++) m[k] += b[s * kMomStride + k];
}

__device__ inline Macro macro_of_node(const DevInstance& I, int i)
{
    double m[kMomStride];
    node_sums(I, i, m);
    return macro_from_sums(m);
}

__device__ inline double chi_of(double eta) { return (2 - eta) / (2 * (1 - eta) * (1 - eta) * (1 - eta)); }

// Value of f at cell c (c may be a ghost: -2, -1, nr, nr+1) for velocity v with radial
// momentum pr.  Entering velocities see n_w times the unit wall Maxwellian; leaving ones
// the quadratic extrapolation of the three nearest cells.
__device__ inline double fcell(const double* __restrict__ f, int c, int v, int nr, int nv, double pr, double nwl,
                               double nwr, const double* __restrict__ gwl, const double* __restrict__ gwr)
{
    if (c >= 0 && c < nr) return gload(f + (size_t)c * nv + v);
    if (c < 0) {
        if (pr > 0) return nwl * gload(gwl + v);
        const double f0 = gload(f + v), f1 = gload(f + nv + v), f2 = gload(f + 2 * (size_t)nv + v);
        return c == -1 ? 3 * f0 - 3 * f1 + f2 : 6 * f0 - 8 * f1 + 3 * f2;
    }
    if (pr < 0) return nwr * gload(gwr + v);
    const double* fl = f + (size_t)(nr - 1) * nv;
    const double a = gload(fl + v), b = gload(fl + v - nv), c3 = gload(fl + v - 2 * (size_t)nv);
    return c == nr ? 3 * a - 3 * b + c3 : 6 * a - 8 * b + 3 * c3;
}

// A wave-uniform double moved to scalar registers (frees vector registers).
__device__ inline double uniform(double x)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

// Reduce-scatter of 16 per-lane doubles over a wave64: after the call, every lane holds the
// wave total of value (lane >> 2) & 15.  Lane halves are combined with v_permlane32_swap, row
// pairs with v_permlane16_swap, then lanes xor 8, xor 4 (DPP row rotations / shifts) and the
// quad (DPP quad_perm).  Fixed order, so reproducible.
__device__ inline double swap32_sum(double a, double b)
{
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

__device__ inline double swap16_sum(double a, double b)
{
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

template <int CTRL, int BANK>
__device__ inline double dpp_or_old(double old, double x)
{
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(x), CTRL, 0xf, BANK, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(x), CTRL, 0xf, BANK, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double reduce_scatter16(const double* v, int lane)
{
    double r[8], t[4], u[2];
#pragma unroll
    for (int k = 0; k < 8; k++) r[k] = swap32_sum(v[k], v[k + 8]);
#pragma unroll
    for (int k = 0; k < 4; k++) t[k] = swap16_sum(r[k], r[k + 4]);
    const bool b3 = lane & 8, b2 = lane & 4;
#pragma unroll
    for (int k = 0; k < 2; k++) {
        const double keep = b3 ? t[k + 2] : t[k], give = b3 ? t[k] : t[k + 2];
        u[k] = keep + dpp_or_old<0x128, 0xf>(0.0, give);  // row_ror:8
    }
    const double keep = b2 ? u[1] : u[0], give = b2 ? u[0] : u[1];
    double part = dpp_or_old<0x104, 0x5>(0.0, give);  // row_shl:4 on banks 0, 2
    part = dpp_or_old<0x114, 0xa>(part, give);         // row_shr:4 on banks 1, 3
    double w = keep + part;
    w += dpp_or_old<0x4e, 0xf>(0.0, w);  // quad_perm [2,3,0,1]
    w += dpp_or_old<0xb1, 0xf>(0.0, w);  // quad_perm [1,0,3,2]
    return w;
}

// ------------------------------------------------------------------ moments of a state

// Moment sums of buffer `buf` with shift 0 (used at start-up and after lbe_set_state).
__global__ void __launch_bounds__(kBlock) k_moments(const DevInstance* __restrict__ insts, int buf)
{
    const DevInstance& I = insts[blockIdx.y];
    const int i = blockIdx.x;
    if (i >= I.nr) return;
    __shared__ double red[16 * 4];
    const double* fi = I.f[buf] + (size_t)i * I.nv;
    double acc[13];
#pragma unroll
    for (int k = 0; k < 13; k++) acc[k] = 0;
    for (int v = threadIdx.x; v < I.nv; v += kBlock) {
        const int i0 = v % I.n0, rest = v / I.n0, i1 = rest % I.n1, i2 = rest / I.n1;
        const double x = I.p0[i0], y = I.p1[i1], z = I.p2[i2], fv = fi[v];
        const double x2 = x * x + y * y + z * z;
        acc[MF_S0] += fv;
        acc[MF_S1X] += fv * x;
        acc[MF_S1Y] += fv * y;
        acc[MF_S1Z] += fv * z;
        acc[MF_SXX] += fv * x * x;
        acc[MF_SYY] += fv * y * y;
        acc[MF_SZZ] += fv * z * z;
        acc[MF_SXY] += fv * x * y;
        acc[MF_SXZ] += fv * x * z;
        acc[MF_SYZ] += fv * y * z;
        acc[MF_S3X] += fv * x2 * x;
        acc[MF_S3Y] += fv * x2 * y;
        acc[MF_S3Z] += fv * x2 * z;
    }
    block_sum<13>(acc, red);
    for (int k = threadIdx.x; k < I.nslices * kMomStride; k += kBlock)
        I.mom[(size_t)i * I.nslices * kMomStride + k] = (k < 13) ? red[k * 4] : 0.0;
}

// ------------------------------------------------------------------ node kernel

__global__ void __launch_bounds__(kBlock) k_node(const DevInstance* __restrict__ insts, int src)
{
    const DevInstance& I = insts[blockIdx.y];
    if (!I.flags[1]) return;
    const int nr = I.nr;
    const int nchunks = (nr + kNodeChunk - 1) / kNodeChunk;
    const int bx = blockIdx.x;
    __shared__ double red[16 * 4];
    if (bx >= nchunks + 2) return;
    const double* f = I.f[src];

    if (bx >= nchunks) {
        // Wall density of diffuse reflection: n_w = - sum_{leaving} p_r f_hat / sum_{entering} p_r g_w.
        const int left = bx == nchunks;
        double acc[1] = {0};
        for (int v = threadIdx.x; v < I.nv; v += kBlock) {
            const double pr = I.p0[v % I.n0];
            if (left && pr < 0) {
                const double f0 = f[v], f1 = f[I.nv + v], f2 = f[2 * (size_t)I.nv + v];
                const double gm1 = 3 * f0 - 3 * f1 + f2, gm2 = 6 * f0 - 8 * f1 + 3 * f2;
                acc[0] += pr * weno5(f2, f1, f0, gm1, gm2);
            } else if (!left && pr > 0) {
                const double* fl = f + (size_t)(nr - 1) * I.nv;
                const double a = fl[v], b = fl[v - I.nv], c = fl[v - 2 * (size_t)I.nv];
                const double gp1 = 3 * a - 3 * b + c, gp2 = 6 * a - 8 * b + 3 * c;
                acc[0] += pr * weno5(c, b, a, gp1, gp2);
            }
        }
        block_sum<1>(acc, red);
        if (threadIdx.x == 0) I.nw[left ? 0 : 1] = -red[0] / (left ? I.gin_l : I.gin_r);
        return;
    }

    // Node chunk [c0, c1) with a halo of kHalo nodes for the gradient stencils.
    const int c0 = bx * kNodeChunk, c1 = min(nr, c0 + kNodeChunk);
    const int h0 = max(0, c0 - kHalo), h1 = min(nr, c1 + kHalo);
    const int nh = h1 - h0;
    __shared__ double sT[kNodeChunk + 2 * kHalo], su[3][kNodeChunk + 2 * kHalo];
    __shared__ double sG1[kNodeChunk + 2 * kHalo], sG2[kNodeChunk + 2 * kHalo], schi[kNodeChunk + 2 * kHalo];
    __shared__ Macro smac[kNodeChunk];
    __shared__ double sdens[kMaxNr];
    __shared__ double snb[kNodeChunk + 2 * kHalo];
    // densities of every node (slice sums), then the averaged density of the chunk + halo,
    // eq. (fm): nbar_j = sum_k W_jk n_k over the band, 8 lanes per row, loads batched by 8
    for (int j = threadIdx.x; j < nr; j += kBlock) {
        const double* b = I.mom + (size_t)j * I.nslices * kMomStride;
        double n = b[MF_S0];
        for (int sl = 1; sl < I.nslices; sl++) n += b[sl * kMomStride + MF_S0];
        sdens[j] = n;
    }
    __syncthreads();
    {
        const int grp = threadIdx.x >> 3, sub = threadIdx.x & 7;
        const int wband = I.wband;
        for (int k = grp; k < nh; k += kBlock / 8) {
            const int j = h0 + k;
            const int lo = I.wlo[j];
            const double* wrow = I.wb + (size_t)j * wband;
            double part = 0;
            for (int base = sub; base < wband; base += 64) {
                double wv[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int k2 = base + 8 * u;
                    wv[u] = (k2 < wband) ? wrow[k2] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int col = lo + base + 8 * u;
                    if (base + 8 * u < wband && col < nr) part += wv[u] * sdens[col];
                }
            }
            // combine the 8 partial sums of the group in a fixed order
            part += __shfl_down(part, 4, 8);
            part += __shfl_down(part, 2, 8);
            part += __shfl_down(part, 1, 8);
            if (sub == 0) snb[k] = part;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nh; k += kBlock) {
        const int j = h0 + k;
        const Macro m = macro_of_node(I, j);
        const double nb = snb[k];
        const double chi = chi_of(I.eta0 * nb);
        sT[k] = m.T;
        for (int a = 0; a < 3; a++) su[a][k] = m.u[a];
        schi[k] = chi;
        sG1[k] = log(m.n * m.n * chi * m.T);
        sG2[k] = log(m.T);
        if (j >= c0 && j < c1) smac[j - c0] = m;
    }
    __syncthreads();
    const double inv12dr = 1.0 / (12 * I.dr);
    const double kSqrt2Pi5_16 = 5 * sqrt(2 * M_PI) / 16;
    const double kC1 = 4.0 / 25 * (1 + 12 / M_PI);
    const double kD1 = 9.0 / 25 * (1 + 32 / (9 * M_PI));
    for (int k = threadIdx.x; k < c1 - c0; k += kBlock) {
        const int i = c0 + k;
        const int li = i - h0;
        const Macro& m = smac[k];
        // gradient stencils read local arrays shifted so that index = global node - h0
        auto g = [&](const double* arr) {
            if (i == 0 || i == 1 || i == nr - 1 || i == nr - 2) {
                double tmp[5];
                const int base = (i <= 1) ? 0 : nr - 5;
                for (int t = 0; t < 5; t++) tmp[t] = arr[base + t - h0];
                if (i == 0) return (-25 * tmp[0] + 48 * tmp[1] - 36 * tmp[2] + 16 * tmp[3] - 3 * tmp[4]) * inv12dr;
                if (i == 1) return (-3 * tmp[0] - 10 * tmp[1] + 18 * tmp[2] - 6 * tmp[3] + tmp[4]) * inv12dr;
                if (i == nr - 1) return (25 * tmp[4] - 48 * tmp[3] + 36 * tmp[2] - 16 * tmp[1] + 3 * tmp[0]) * inv12dr;
                return (3 * tmp[4] + 10 * tmp[3] - 18 * tmp[2] + 6 * tmp[1] - tmp[0]) * inv12dr;
            }
            return (arr[li - 2] - 8 * arr[li - 1] + 8 * arr[li + 1] - arr[li + 2]) * inv12dr;
        };
        const double D1 = g(sG1), D2 = g(sG2), du0 = g(su[0]), du1 = g(su[1]), du2 = g(su[2]);
        const double n = m.n, T = m.T, chi = schi[li];
        const double brho = 4 * I.eta0 * n;
        const double brhochi = brho * chi;
        const double bracket = 1 / chi + 0.8 * brho + kC1 * brho * brho * chi;
        const double tau = kSqrt2Pi5_16 * I.chi0 * I.kn * I.L * bracket / (n * sqrt(T));
        const double x = brhochi;
        const double Pr = (2.0 / 3) * (1 + 0.8 * x + kC1 * x * x) / (1 + 1.2 * x + kD1 * x * x);
        const double invr = I.geo[4 * i + 3];
        double* nd = I.node + (size_t)i * kNodeStride;
        nd[NF_N] = n;
        nd[NF_U0] = m.u[0];
        nd[NF_U1] = m.u[1];
        nd[NF_U2] = m.u[2];
        nd[NF_T] = T;
        nd[NF_Q0] = m.q[0];
        nd[NF_Q1] = m.q[1];
        nd[NF_Q2] = m.q[2];
        nd[NF_TAU] = tau;
        nd[NF_PR] = Pr;
        nd[NF_BRHOCHI] = brhochi;
        nd[NF_D1] = D1;
        nd[NF_D2] = D2;
        nd[NF_DU0] = du0;
        nd[NF_DU1] = du1;
        nd[NF_DU2] = du2;
        nd[NF_NBAR] = snb[li];
        nd[NF_CHI] = chi;
        nd[NF_P01] = m.P01;
        nd[NF_SHAK] = (1 - Pr) / (n * T * T);
        nd[NF_INVTAU] = 1 / tau;
        // divergence and the covariant shear pieces of zeta zeta : grad u (reading of eq. (j1))
        if (I.geometry == LBE_CYL) {
            nd[NF_DIVU] = du0 + m.u[0] * invr;
            nd[NF_SHEAR01] = du1 - m.u[1] * invr;
        } else {
            nd[NF_DIVU] = du0 + 2 * m.u[0] * invr;
            nd[NF_SHEAR01] = 0;
        }
        nd[NF_UR_R] = m.u[0] * invr;
        nd[NF_INV2T] = 1 / (2 * T);
        nd[NF_INV5T] = 1 / (5 * T);
        if (!(n > 0) || !(T > 0) || !isfinite(n) || !isfinite(T)) I.flags[0] = 1;
        // equilibrium coefficients of the full-range axes (eq. (eq_gak_H))
        full_coeffs<kMaxN>(m.u[1], T, I.N1, nd + NF_C1);
        full_coeffs<kMaxN>(m.u[2], T, I.N2, nd + NF_C2);
    }
}

// Half-range projection coefficients I_l^+- (Sec. III.C) of every node: one wave per node,
// the 64 lanes share the quadrature nodes of the panels within 9.6 sqrt(T) of +-u (farther
// panels contribute below 1e-20 of the peak), and the 2 (N0+1) <= 32 sums are reduced with
// the register reduce-scatter.  Runs after k_node (needs u_r and T of the node).
__global__ void __launch_bounds__(kBlock) k_proj(const DevInstance* __restrict__ insts)
{
    const DevInstance& I = insts[blockIdx.y];
    if (!I.flags[1]) return;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (i >= I.nr) return;
    double* nd = I.node + (size_t)i * kNodeStride;
    const double u = nd[NF_U0], T = nd[NF_T];
    const int N0 = I.N0, M = I.M0, npan = M / 16;
    const double reach = 9.6 * sqrt(T), c = kInvSqrt2Pi / sqrt(T), inv2T = 1 / (2 * T);
    double acc[32];
#pragma unroll
    for (int k = 0; k < 32; k++) acc[k] = 0;
    for (int side = 0; side < 2; side++) {
        const double uu = side ? -u : u;
        int p0 = (int)floor((uu - reach) / 0.75), p1 = (int)ceil((uu + reach) / 0.75);
        p0 = max(0, min(p0, npan));
        p1 = max(p0, min(p1, npan));
        for (int m = 16 * p0 + lane; m < 16 * p1; m += 64) {
            const double d = I.qy0[m] - uu;
            const double gw = I.qlam0[m] * c * exp(-d * d * inv2T);
            const double* h = I.qh0 + (size_t)m * (N0 + 1);
#pragma unroll
            for (int l = 0; l < 16; l++)
                if (l <= N0) acc[side * 16 + l] += gw * h[l];
        }
    }
    // two reduce-scatters of 16 values: lanes (l >> 2) & 15 = l-index hold the totals
    const double totp = reduce_scatter16(acc, lane);
    const double totm = reduce_scatter16(acc + 16, lane);
    const int which = (lane >> 2) & 15;
    if ((lane & 3) == 0 && which <= N0) {
        nd[NF_IPLUS + which] = totp;
        nd[NF_IMINUS + which] = totm;
    }
}

// Equilibrium factors g_R, g_1, g_2 of every node into I.geq (for the reference stage kernel).
__global__ void __launch_bounds__(kBlock) k_geq(const DevInstance* __restrict__ insts)
{
    const DevInstance& I = insts[blockIdx.y];
    if (!I.flags[1]) return;
    const int ng = I.n0 + I.n1 + I.n2;
    for (int t = blockIdx.x * kBlock + threadIdx.x; t < I.nr * ng; t += gridDim.x * kBlock) {
        const int i = t / ng, e = t % ng;
        const double* nd = I.node + (size_t)i * kNodeStride;
        double val;
        if (e < I.n0) {
            const double* Ic = nd + (I.p0[e] > 0 ? NF_IPLUS : NF_IMINUS);
            double acc = 0;
            for (int l = 0; l <= I.N0; l++) acc += Ic[l] * I.poly0[e * (I.N0 + 1) + l];
            val = I.w0[e] * acc;
        } else if (e < I.n0 + I.n1) {
            const int kk = e - I.n0;
            double acc = 0;
            for (int l = 0; l <= I.N1; l++) acc += nd[NF_C1 + l] * I.poly1[kk * (I.N1 + 1) + l];
            val = I.w1[kk] * acc;
        } else {
            const int kk = e - I.n0 - I.n1;
            double acc = 0;
            for (int l = 0; l <= I.N2; l++) acc += nd[NF_C2 + l] * I.poly2[kk * (I.N2 + 1) + l];
            val = I.w2[kk] * acc;
        }
        I.geq[(size_t)i * ng + e] = val;
    }
}

// ------------------------------------------------------------------ stage kernel

// mode 0: out = an * f[fn] + bs * (f[src] + dt L(f[src])) stored in f[dst], with moment sums;
// mode 1: L(f[src]) stored in scratch (no state change).
__global__ void __launch_bounds__(kBlock) k_stage(const DevInstance* __restrict__ insts, int src, int fn, int dst,
                                                  double an, double bs, int mode)
{
    const DevInstance& I = insts[blockIdx.y];
    if (!I.flags[1]) return;
    const int i = blockIdx.x;
    const int nr = I.nr, nv = I.nv, n0 = I.n0, n1 = I.n1, n2 = I.n2;
    if (i >= nr) return;
    extern __shared__ double plane[];  // nv doubles
    __shared__ double red[16 * 4];
    __shared__ double snd[kNodeStride];
    const double* __restrict__ f = I.f[src];
    const double* fi = f + (size_t)i * nv;
    for (int v = threadIdx.x; v < nv; v += kBlock) plane[v] = fi[v];
    if (threadIdx.x < kNodeStride) snd[threadIdx.x] = I.node[(size_t)i * kNodeStride + threadIdx.x];
    __syncthreads();

    const int ng = n0 + n1 + n2;
    const double* gR = I.geq + (size_t)i * ng;
    const double* g1 = gR + n0;
    const double* g2 = g1 + n1;
    const double n = snd[NF_N], u0 = snd[NF_U0], u1 = snd[NF_U1], u2 = snd[NF_U2], T = snd[NF_T];
    const double q0 = snd[NF_Q0], q1 = snd[NF_Q1], q2 = snd[NF_Q2];
    const double invtau = snd[NF_INVTAU], shak = snd[NF_SHAK], brhochi = snd[NF_BRHOCHI];
    const double D1 = snd[NF_D1], D2 = snd[NF_D2], du0 = snd[NF_DU0], du2 = snd[NF_DU2];
    const double divu = snd[NF_DIVU], sh01 = snd[NF_SHEAR01], urr = snd[NF_UR_R];
    const double inv2T = 1 / (2 * T), inv5T = 1 / (5 * T);
    const double adv_l = I.geo[4 * i + 0], adv_r = I.geo[4 * i + 1], ffac = I.geo[4 * i + 2];
    const double nwl = I.nw[0], nwr = I.nw[1];
    const double dt = I.dt;
    const bool cyl = I.geometry == LBE_CYL;
    const double* fnp = I.f[fn] + (size_t)i * nv;
    double* out = (mode == 0) ? I.f[dst] + (size_t)i * nv : I.scratch + (size_t)i * nv;

    double acc[13];
#pragma unroll
    for (int k = 0; k < 13; k++) acc[k] = 0;

    for (int v = threadIdx.x; v < nv; v += kBlock) {
        const int i0 = v % n0, rest = v / n0, i1 = rest % n1, i2 = rest / n1;
        const double pr = I.p0[i0], py = I.p1[i1], pz = I.p2[i2];
        // ---- advection: flux form with WENO-5 face values, upwind by the sign of p_r
        double Fl, Fr;
        if (pr > 0) {
            double c[6];  // cells i-3 .. i+2
            for (int t = (i == 0 ? 1 : 0); t < 6; t++)
                c[t] = fcell(f, i - 3 + t, v, nr, nv, pr, nwl, nwr, I.gwl, I.gwr);
            Fl = (i == 0) ? pr * nwl * I.gwl[v] : pr * weno5(c[0], c[1], c[2], c[3], c[4]);
            Fr = pr * weno5(c[1], c[2], c[3], c[4], c[5]);
        } else {
            double c[6];  // cells i-2 .. i+3
            const int tmax = (i == nr - 1) ? 5 : 6;
            for (int t = 0; t < tmax; t++) c[t] = fcell(f, i - 2 + t, v, nr, nv, pr, nwl, nwr, I.gwl, I.gwr);
            Fl = pr * weno5(c[4], c[3], c[2], c[1], c[0]);
            Fr = (i == nr - 1) ? pr * nwr * I.gwr[v] : pr * weno5(c[5], c[4], c[3], c[2], c[1]);
        }
        const double A = adv_r * Fr - adv_l * Fl;
        // ---- inertial terms (momentum-derivative contractions on the LDS plane)
        double d0 = 0, d1 = 0, d2 = 0;
        {
            const double* K = I.K1 + i0 * n0;
            const double* col = plane + n0 * (i1 + n1 * i2);
            for (int k = 0; k < n0; k++) d0 += K[k] * col[k];
            const double* Ka = I.K2a + i1 * n1;
            const double* rowa = plane + i0 + n0 * n1 * i2;
            for (int k = 0; k < n1; k++) d1 += Ka[k] * rowa[n0 * k];
            if (!cyl) {
                const double* Kb = I.K2b + i2 * n2;
                const double* rowb = plane + i0 + n0 * i1;
                for (int k = 0; k < n2; k++) d2 += Kb[k] * rowb[n0 * n1 * k];
            }
        }
        const double Iv = cyl ? ffac * (py * py * d0 - pr * d1) : ffac * ((py * py + pz * pz) * d0 - pr * (d1 + d2));
        // ---- collision: Shakhov J0 and J1[f^MB] on the discrete equilibrium
        const double fmb = n * gR[i0] * g1[i1] * g2[i2];
        const double x0 = pr - u0, x1 = py - u1, x2 = pz - u2;
        const double xi2 = x0 * x0 + x1 * x1 + x2 * x2;
        const double xq = x0 * q0 + x1 * q1 + x2 * q2;
        const double fS = fmb * (1 + shak * (xi2 * inv5T - 1) * xq);
        const double z2 = xi2 * inv2T;
        const double zzgu = cyl ? (x0 * x0 * du0 + x0 * x1 * sh01 + x1 * x1 * urr + x0 * x2 * du2) * inv2T
                                : (x0 * x0 * du0 + (x1 * x1 + x2 * x2) * urr) * inv2T;
        const double S = x0 * (D1 + 0.6 * (z2 - 2.5) * D2) + 0.4 * (2 * zzgu + (z2 - 2.5) * divu);
        const double fv = plane[v];
        const double L = -A - Iv - (fv - fS) * invtau - brhochi * fmb * S;
        if (mode == 1) {
            out[v] = L;
            continue;
        }
        const double o = an * fnp[v] + bs * (fv + dt * L);
        out[v] = o;
        // moment sums of the stored value, shifted by the current velocity
        const double y0 = pr - u0, y1 = py - u1, y2 = pz - u2;
        const double y2s = y0 * y0 + y1 * y1 + y2 * y2;
        acc[MF_S0] += o;
        acc[MF_S1X] += o * y0;
        acc[MF_S1Y] += o * y1;
        acc[MF_S1Z] += o * y2;
        acc[MF_SXX] += o * y0 * y0;
        acc[MF_SYY] += o * y1 * y1;
        acc[MF_SZZ] += o * y2 * y2;
        acc[MF_SXY] += o * y0 * y1;
        acc[MF_SXZ] += o * y0 * y2;
        acc[MF_SYZ] += o * y1 * y2;
        acc[MF_S3X] += o * y2s * y0;
        acc[MF_S3Y] += o * y2s * y1;
        acc[MF_S3Z] += o * y2s * y2;
    }
    if (mode == 1) return;
    block_sum<13>(acc, red);
    if (threadIdx.x < 16) {
        const int k = threadIdx.x;
        double val;
        if (k < 13)
            val = red[k * 4];
        else
            val = (k == MF_CX) ? u0 : (k == MF_CY) ? u1 : u2;
        I.mom[(size_t)i * I.nslices * kMomStride + k] = val;
    }
}

// ------------------------------------------------------------------ tiled stage kernel

typedef double v4d __attribute__((ext_vector_type(4)));

// 64-lane sum of a double with DPP row shifts (within 16-lane rows) and lane reads across the
// four rows; the result is valid in every lane.  Fixed order, so reproducible.
template <int CTRL, int BANK_MASK>
__device__ inline double dpp_shift(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, BANK_MASK, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, BANK_MASK, true);
    return __hiloint2double(hi, lo);
}

__device__ inline double wave_total(double v)
{
    double s = v + dpp_shift<0x111, 0xf>(v);  // row_shr:1
    s += dpp_shift<0x112, 0xf>(v);            // row_shr:2
    s += dpp_shift<0x113, 0xf>(v);            // row_shr:3 -> 4 consecutive lanes
    s += dpp_shift<0x114, 0xe>(s);            // row_shr:4 on banks 1..3
    s += dpp_shift<0x118, 0xc>(s);            // row_shr:8 on banks 2..3 -> lane 15 of each row
    const int lo = __double2loint(s), hi = __double2hiint(s);
    double r0 = __hiloint2double(__builtin_amdgcn_readlane(hi, 15), __builtin_amdgcn_readlane(lo, 15));
    double r1 = __hiloint2double(__builtin_amdgcn_readlane(hi, 31), __builtin_amdgcn_readlane(lo, 31));
    double r2 = __hiloint2double(__builtin_amdgcn_readlane(hi, 47), __builtin_amdgcn_readlane(lo, 47));
    double r3 = __hiloint2double(__builtin_amdgcn_readlane(hi, 63), __builtin_amdgcn_readlane(lo, 63));
    return ((r0 + r1) + r2) + r3;
}

// One RK stage for a tile of NT consecutive nodes x one velocity slice of one instance.
// Lanes own velocities v = vs0 + tid + block * j (j < VPT) for the whole tile and keep, per
// velocity, a register window of the 7 cells i-3 .. i+3 around the current node i, so every
// face flux is computed once and every value of f_src is read once (plus a 6-cell halo per
// tile).  The node's plane is staged in LDS (column stride n0 + 1) and the three
// momentum-derivative contractions run as FP64 MFMA 16x16x4 tiles over it:
//   d0 = K1 P        (n0 x n0) x (n0 x columns)         rows = radial momentum
//   d1 = K2a P_i2    (n1 x n1) x (n1 x n0) per i2
//   d2 = K2b P'      (n2 x n2) x (n2 x n0 n1)           sphere only
// each into its own LDS plane, already multiplied by its momentum and geometry factor.
// Two barriers per node: phase A (MFMA of node t, WENO face flux of node t) and phase B
// (collision + RK combine + store of node t with its moment sums, reduced across the wave by
// a register reduce-scatter; staging of node t+1's plane, prefetch of node t+2's window cell
// and node t+1's f^n).
template <int VPT>
__global__ void __launch_bounds__(1024) k_stage2(const DevInstance* __restrict__ insts,
                                                  const WorkItem* __restrict__ items, const StageGroup G, int src,
                                                  int fn, int dst, double an, double bs)
{
    extern __shared__ double lds[];
    const WorkItem it = items[blockIdx.x];
    const DevInstance& I = insts[it.inst];
    if (!I.flags[1]) return;
    const int nr = I.nr, nv = G.nv, n0 = G.n0, n1 = G.n1, n2 = G.n2;
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63, W = B >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: tile math on scalars
    const int cs = n0 + 1;  // LDS column stride
    const bool sph = G.geometry == LBE_SPH;
    const bool need_fn = an != 0.0;  // stage 1 combines with f_src itself
    const int k1s = G.n0k + 1, k2as = G.n1k + 1, k2bs = G.n2k + 1;  // odd LDS row strides of K
    const int vs0 = it.slice * G.nvs, vs1 = vs0 + G.nvs;
    const int c_s0 = it.slice * G.ncols_s;      // first global column (i1 + n1 i2) of the slice
    const int cp0 = sph ? 0 : c_s0;            // first global column held in the LDS plane
    const int i2s0 = it.slice * G.ns2;          // first i2 of the slice
    const int pslice = cs * G.ncols_s;          // size of one slice plane
    double* plane = lds + G.off_plane;
    double* ib0 = lds + G.off_ibuf;             // d0 terms, then d1, d2 terms, then 2 output planes
    double* ib1 = ib0 + pslice;
    double* ib2 = ib1 + pslice;
    double* K1s = lds + G.off_K1;
    double* K2as = lds + G.off_K2a;
    double* K2bs = lds + G.off_K2b;
    double* snode = lds + G.off_node;
    double* sgeq = lds + G.off_geq;
    double* spart = lds + G.off_part;
    double* sp = lds + G.off_p;
    const double* __restrict__ f = I.f[src];
    const double* __restrict__ fN = I.f[fn];
    double* __restrict__ fout = I.f[dst];
    const int ng = n0 + n1 + n2;

    // ---- per-workgroup set-up: force matrices (zero-padded), momentum nodes, node data
    for (int e = tid; e < G.n0p * k1s; e += B) {
        const int r = e / k1s, k = e % k1s;
        K1s[e] = (r < n0 && k < n0) ? I.K1[r * n0 + k] : 0.0;
    }
    for (int e = tid; e < G.n1p * k2as; e += B) {
        const int r = e / k2as, k = e % k2as;
        K2as[e] = (r < n1 && k < n1) ? I.K2a[r * n1 + k] : 0.0;
    }
    if (sph)
        for (int e = tid; e < G.ns2p * k2bs; e += B) {
            const int r = e / k2bs, k = e % k2bs;
            K2bs[e] = (r < G.ns2 && k < n2) ? I.K2b[(i2s0 + r) * n2 + k] : 0.0;
        }
    // per-column factor of d0 (p_1^2 [+ p_2^2]) and, for the sphere, the (i0, i1) split of the
    // d2 columns with their factor -p_r: avoids per-node integer division
    double* colfac = lds + G.off_colfac;
    int* cpinfo = (int*)(lds + G.off_cpinfo);
    for (int e = tid; e < G.ncols_s; e += B) {
        const int cg = c_s0 + e;
        const double pyy = I.p1[cg % n1];
        double fac = pyy * pyy;
        if (sph) {
            const double pzz = I.p2[cg / n1];
            fac += pzz * pzz;
        }
        colfac[e] = fac;
    }
    if (sph)
        for (int e = tid; e < n0 * n1; e += B) cpinfo[e] = (e % n0) | ((e / n0) << 8);
    for (int e = tid; e < ng; e += B) sp[e] = e < n0 ? I.p0[e] : e < n0 + n1 ? I.p1[e - n0] : I.p2[e - n0 - n1];
    for (int e = tid; e < it.nt * SN_COUNT; e += B) {
        const int t = e / SN_COUNT, fld = e % SN_COUNT, i = it.i0 + t;
        const double* nd = I.node + (size_t)i * kNodeStride;
        double val;
        switch (fld) {
            case SN_N: val = nd[NF_N]; break;
            case SN_U0: val = nd[NF_U0]; break;
            case SN_U1: val = nd[NF_U1]; break;
            case SN_U2: val = nd[NF_U2]; break;
            case SN_T: val = nd[NF_T]; break;
            case SN_Q0: val = nd[NF_Q0]; break;
            case SN_Q1: val = nd[NF_Q1]; break;
            case SN_Q2: val = nd[NF_Q2]; break;
            case SN_INVTAU: val = nd[NF_INVTAU]; break;
            case SN_SHAK: val = nd[NF_SHAK]; break;
            case SN_BRHOCHI: val = nd[NF_BRHOCHI]; break;
            case SN_D1: val = nd[NF_D1]; break;
            case SN_D2: val = nd[NF_D2]; break;
            case SN_DU0: val = nd[NF_DU0]; break;
            case SN_DU2: val = nd[NF_DU2]; break;
            case SN_DIVU: val = nd[NF_DIVU]; break;
            case SN_SH01: val = nd[NF_SHEAR01]; break;
            case SN_URR: val = nd[NF_UR_R]; break;
            case SN_ADVL: val = I.geo[4 * i + 0]; break;
            case SN_ADVR: val = I.geo[4 * i + 1]; break;
            case SN_INV2T: val = nd[NF_INV2T]; break;
            case SN_INV5T: val = nd[NF_INV5T]; break;
            default: val = I.geo[4 * i + 2]; break;
        }
        snode[t * kStageNodeStride + fld] = val;
    }
    // equilibrium factors of the tile's nodes from their projection coefficients (the l sums
    // are unrolled to the largest order so their loads issue together)
    for (int e = tid; e < it.nt * ng; e += B) {
        const int t = e / ng, k = e % ng;
        const double* nd = I.node + (size_t)(it.i0 + t) * kNodeStride;
        const double *cf, *poly, *wt;
        int N, kk;
        if (k < n0) {
            cf = nd + (I.p0[k] > 0 ? NF_IPLUS : NF_IMINUS);
            N = I.N0;
            kk = k;
            poly = I.poly0;
            wt = I.w0;
        } else if (k < n0 + n1) {
            cf = nd + NF_C1;
            N = I.N1;
            kk = k - n0;
            poly = I.poly1;
            wt = I.w1;
        } else {
            cf = nd + NF_C2;
            N = I.N2;
            kk = k - n0 - n1;
            poly = I.poly2;
            wt = I.w2;
        }
        double cv[kMaxN + 1], pv[kMaxN + 1];
#pragma unroll
        for (int l = 0; l <= kMaxN; l++) {
            cv[l] = l <= N ? cf[l] : 0.0;
            pv[l] = l <= N ? poly[kk * (N + 1) + l] : 0.0;
        }
        double acc = 0;
#pragma unroll
        for (int l = 0; l <= kMaxN; l++) acc += cv[l] * pv[l];
        sgeq[t * ng + k] = wt[kk] * acc;
    }

    // ---- per-lane velocities: v = vs0 + tid + B j; code = i0 | i1 << 8 | i2 << 16
    const double nwl = I.nw[0], nwr = I.nw[1];
    int code[VPT];
    double prv[VPT];
#pragma unroll
    for (int j = 0; j < VPT; j++) {
        const int v = min(vs0 + tid + B * j, vs1 - 1);
        const int i0 = v % n0, c = v / n0, i1 = c % n1, i2 = c / n1;
        code[j] = i0 | (i1 << 8) | (i2 << 16);
        prv[j] = I.p0[i0];
    }
    // ---- window of cells i0-3 .. i0+3, f^n of the first node, the first node's plane
    double w[VPT][7], Fl[VPT], wnext[VPT], fnv[VPT];
#pragma unroll
    for (int j = 0; j < VPT; j++) {
        const int v = min(vs0 + tid + B * j, vs1 - 1);
        const double pr = prv[j];
#pragma unroll
        for (int k = 0; k < 7; k++) w[j][k] = fcell(f, it.i0 - 3 + k, v, nr, nv, pr, nwl, nwr, I.gwl, I.gwr);
        wnext[j] = fcell(f, it.i0 + 4, v, nr, nv, pr, nwl, nwr, I.gwl, I.gwr);
        fnv[j] = need_fn ? gload(fN + (size_t)it.i0 * nv + v) : 0.0;
        if (pr > 0)
            Fl[j] = (it.i0 == 0) ? pr * nwl * gload(I.gwl + v)
                                 : pr * weno5(w[j][0], w[j][1], w[j][2], w[j][3], w[j][4]);
        else
            Fl[j] = pr * weno5(w[j][5], w[j][4], w[j][3], w[j][2], w[j][1]);
        if (vs0 + tid + B * j < vs1) {
            const int i0 = code[j] & 0xff, c = (code[j] >> 8 & 0xff) + n1 * (code[j] >> 16);
            plane[i0 + cs * (c - cp0)] = w[j][3];
        }
    }
    if (sph && G.S > 1)
        for (int v = tid; v < nv; v += B)
            if (v < vs0 || v >= vs1) plane[(v % n0) + cs * (v / n0)] = gload(f + (size_t)it.i0 * nv + v);

    const int nM1 = G.n0p / 16, nN1 = (G.ncols_s + 15) / 16;
    const int nM2 = G.n1p / 16, nN2 = G.n0p / 16;
    const int nM3 = G.ns2p / 16, nN3 = (n0 * n1 + 15) / 16;
    const int nT1 = nM1 * nN1, nT2 = G.ns2 * nM2 * nN2, nT3 = sph ? nM3 * nN3 : 0;
    const int q16 = lane & 15, q4 = lane >> 4;

    __syncthreads();
    for (int t = 0; t < it.nt; t++) {
        const int i = it.i0 + t;
        const double* nd = snode + t * kStageNodeStride;
        const double ffac = uniform(nd[SN_FFAC]);
        // ================= phase A: contractions of node t, face flux i+1, moments of node t-1
        for (int tile = wave; tile < nT1 + nT2 + nT3; tile += W) {
            v4d acc = {0, 0, 0, 0};
            if (tile < nT1) {  // d0 = K1 P into ib0, times ffac (p_1^2 [+ p_2^2])
                const int mt = tile / nN1, ntl = tile % nN1;
                const int col = ntl * 16 + q16;
                const bool cok = col < G.ncols_s;
                const double* bp = plane + cs * (c_s0 + (cok ? col : 0) - cp0);
                const double* ap = K1s + (mt * 16 + q16) * k1s;
                const int kval = cok ? n0 : 0;
                for (int ks = 0; ks < G.n0k; ks += 4) {
                    const int k = ks + q4;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[k], (k < kval) ? bp[k] : 0.0, acc, 0, 0, 0);
                }
                if (cok) {
                    const double fac = colfac[col] * ffac;
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int row = mt * 16 + q4 + 4 * r;
                        if (row < n0) ib0[row + cs * col] = fac * acc[r];
                    }
                }
            } else if (tile < nT1 + nT2) {  // d1 = K2a P_i2 into ib1, times -ffac p_r
                const int tl = tile - nT1;
                const int i2l = tl / (nM2 * nN2), rem = tl % (nM2 * nN2), mt = rem / nN2, ntl = rem % nN2;
                const int i0c = ntl * 16 + q16;
                const bool iok = i0c < n0;
                const double* ap = K2as + (mt * 16 + q16) * k2as;
                const double* bp = plane + (iok ? i0c : 0) + cs * (n1 * (i2s0 + i2l) - cp0);
                const int kval = iok ? n1 : 0;
                for (int ks = 0; ks < G.n1k; ks += 4) {
                    const int k = ks + q4;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[k], (k < kval) ? bp[cs * k] : 0.0, acc, 0, 0, 0);
                }
                if (iok) {
                    const double fac = -ffac * sp[i0c];
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int jrow = mt * 16 + q4 + 4 * r;
                        if (jrow < n1) ib1[i0c + cs * (jrow + n1 * i2l)] = fac * acc[r];
                    }
                }
            } else {  // d2 = K2b P' into ib2, times -ffac p_r (sphere)
                const int tl = tile - nT1 - nT2;
                const int mt = tl / nN3, ntl = tl % nN3;
                const int cp = ntl * 16 + q16;
                const bool pok = cp < n0 * n1;
                const int info = pok ? cpinfo[cp] : 0;
                const int bi0 = info & 0xff, bi1 = info >> 8;
                const double* ap = K2bs + (mt * 16 + q16) * k2bs;
                const double* bp = plane + bi0 + cs * bi1;
                const int kval = pok ? n2 : 0;
                for (int ks = 0; ks < G.n2k; ks += 4) {
                    const int k = ks + q4;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[k], (k < kval) ? bp[cs * n1 * k] : 0.0, acc, 0, 0, 0);
                }
                if (pok) {
                    const double fac = -ffac * sp[bi0];
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int krow = mt * 16 + q4 + 4 * r;
                        if (krow < G.ns2) ib2[bi0 + cs * (bi1 + n1 * krow)] = fac * acc[r];
                    }
                }
            }
        }
        double Fr[VPT];
#pragma unroll
        for (int j = 0; j < VPT; j++) {
            const double pr = prv[j];
            if (pr > 0)
                Fr[j] = pr * weno5(w[j][1], w[j][2], w[j][3], w[j][4], w[j][5]);
            else
                Fr[j] = (i == nr - 1) ? pr * nwr * gload(I.gwr + min(vs0 + tid + B * j, vs1 - 1))
                                      : pr * weno5(w[j][6], w[j][5], w[j][4], w[j][3], w[j][2]);
        }
        __syncthreads();
        // ================= phase B: combine and store node t; stage node t+1
        {
            const double n = uniform(nd[SN_N]), u0 = uniform(nd[SN_U0]), u1 = uniform(nd[SN_U1]);
            const double u2 = uniform(nd[SN_U2]), T = uniform(nd[SN_T]);
            const double q0 = uniform(nd[SN_Q0]), q1 = uniform(nd[SN_Q1]), q2 = uniform(nd[SN_Q2]);
            const double invtau = uniform(nd[SN_INVTAU]), shak = uniform(nd[SN_SHAK]);
            const double brhochi = uniform(nd[SN_BRHOCHI]);
            const double D1 = uniform(nd[SN_D1]), D2 = uniform(nd[SN_D2]), du0 = uniform(nd[SN_DU0]);
            const double du2 = uniform(nd[SN_DU2]);
            const double divu = uniform(nd[SN_DIVU]), sh01 = uniform(nd[SN_SH01]), urr = uniform(nd[SN_URR]);
            const double adv_l = uniform(nd[SN_ADVL]), adv_r = uniform(nd[SN_ADVR]);
            const double inv2T = uniform(nd[SN_INV2T]), inv5T = uniform(nd[SN_INV5T]);
            const double* gR = sgeq + t * ng;
            const double* g1 = gR + n0;
            const double* g2 = g1 + n1;
            double acc[16];
#pragma unroll
            for (int k = 0; k < 16; k++) acc[k] = 0;
#pragma unroll
            for (int j = 0; j < VPT; j++) {
                const int v = vs0 + tid + B * j;
                const int i0 = code[j] & 0xff, i1 = code[j] >> 8 & 0xff, i2 = code[j] >> 16;
                const int ib = i0 + cs * (i1 + n1 * i2 - c_s0);
                const double pr = prv[j], py = sp[n0 + i1], pz = sp[n0 + n1 + i2];
                const double A = adv_r * Fr[j] - adv_l * Fl[j];
                double Iv = ib0[ib] + ib1[ib];
                if (sph) Iv += ib2[ib];
                const double fmb = n * gR[i0] * g1[i1] * g2[i2];
                const double x0 = pr - u0, x1 = py - u1, x2 = pz - u2;
                const double xi2 = x0 * x0 + x1 * x1 + x2 * x2;
                const double xq = x0 * q0 + x1 * q1 + x2 * q2;
                const double fS = fmb * (1 + shak * (xi2 * inv5T - 1) * xq);
                const double z2 = xi2 * inv2T;
                const double zzgu = sph ? (x0 * x0 * du0 + (x1 * x1 + x2 * x2) * urr) * inv2T
                                        : (x0 * x0 * du0 + x0 * x1 * sh01 + x1 * x1 * urr + x0 * x2 * du2) * inv2T;
                const double S = x0 * (D1 + 0.6 * (z2 - 2.5) * D2) + 0.4 * (2 * zzgu + (z2 - 2.5) * divu);
                const double fv = w[j][3];
                const double L = -A - Iv - (fv - fS) * invtau - brhochi * fmb * S;
                const double o = (need_fn ? an * fnv[j] : 0.0) + bs * (fv + I.dt * L);
                if (v < vs1) {
                    gstore(fout + (size_t)i * nv + v, o);
                    // moment sums of the stored value, shifted by the node's velocity
                    acc[MF_S0] += o;
                    acc[MF_S1X] += o * x0;
                    acc[MF_S1Y] += o * x1;
                    acc[MF_S1Z] += o * x2;
                    acc[MF_SXX] += o * x0 * x0;
                    acc[MF_SYY] += o * x1 * x1;
                    acc[MF_SZZ] += o * x2 * x2;
                    acc[MF_SXY] += o * x0 * x1;
                    acc[MF_SXZ] += o * x0 * x2;
                    acc[MF_SYZ] += o * x1 * x2;
                    acc[MF_S3X] += o * xi2 * x0;
                    acc[MF_S3Y] += o * xi2 * x1;
                    acc[MF_S3Z] += o * xi2 * x2;
                }
            }
            {
                const double tot = reduce_scatter16(acc, lane);
                const int which = (lane >> 2) & 15;
                if ((lane & 3) == 0 && which < 13) spart[(t * W + wave) * 13 + which] = tot;
            }
            // advance the window to node t+1, stage its plane, prefetch ahead
            if (t + 1 < it.nt) {
#pragma unroll
                for (int j = 0; j < VPT; j++) {
                    const int v = min(vs0 + tid + B * j, vs1 - 1);
#pragma unroll
                    for (int k = 0; k < 6; k++) w[j][k] = w[j][k + 1];
                    w[j][6] = wnext[j];
                    Fl[j] = Fr[j];
                    wnext[j] = fcell(f, i + 5, v, nr, nv, prv[j], nwl, nwr, I.gwl, I.gwr);
                    fnv[j] = need_fn ? gload(fN + (size_t)(i + 1) * nv + v) : 0.0;
                    if (vs0 + tid + B * j < vs1) {
                        const int i0 = code[j] & 0xff, c = (code[j] >> 8 & 0xff) + n1 * (code[j] >> 16);
                        plane[i0 + cs * (c - cp0)] = w[j][3];
                    }
                }
                if (sph && G.S > 1)
                    for (int v = tid; v < nv; v += B)
                        if (v < vs0 || v >= vs1) plane[(v % n0) + cs * (v / n0)] = gload(f + (size_t)(i + 1) * nv + v);
            }
        }
        __syncthreads();
    }
    // ---- moment sums of the tile's nodes (waves summed in order) for this slice
    for (int e = tid; e < it.nt * 16; e += B) {
        const int t = e / 16, k = e % 16, i = it.i0 + t;
        double val;
        if (k < 13) {
            val = 0;
            for (int wv = 0; wv < W; wv++) val += spart[(t * W + wv) * 13 + k];
        } else {
            val = snode[t * kStageNodeStride + (k == MF_CX ? SN_U0 : k == MF_CY ? SN_U1 : SN_U2)];
        }
        I.mom[((size_t)i * I.nslices + it.slice) * kMomStride + k] = val;
    }
}

// ------------------------------------------------------------------ residual

// Snapshot n, u, T (from the current moment sums) before a checked step.
__global__ void __launch_bounds__(kBlock) k_snapshot(const DevInstance* __restrict__ insts)
{
    const DevInstance& I = insts[blockIdx.y];
    if (!I.flags[1]) return;
    for (int i = threadIdx.x; i < I.nr; i += kBlock) {
        const Macro m = macro_of_node(I, i);
        double* s = I.snap + (size_t)i * 5;
        s[0] = m.n;
        s[1] = m.u[0];
        s[2] = m.u[1];
        s[3] = m.u[2];
        s[4] = m.T;
    }
}

// rho = max_i max(|dn|, |du_r|, |du_1|, |du_2|, |dT|) / dt over the last step.
__global__ void __launch_bounds__(kBlock) k_residual(const DevInstance* __restrict__ insts)
{
    const DevInstance& I = insts[blockIdx.y];
    if (!I.flags[1]) return;
    __shared__ double smax[kBlock];
    double r = 0;
    for (int i = threadIdx.x; i < I.nr; i += kBlock) {
        const Macro m = macro_of_node(I, i);
        const double* s = I.snap + (size_t)i * 5;
        const double d[5] = {m.n - s[0], m.u[0] - s[1], m.u[1] - s[2], m.u[2] - s[3], m.T - s[4]};
        for (int k = 0; k < 5; k++) {
            const double a = fabs(d[k]);
            if (a > r || a != a) r = a;
        }
    }
    smax[threadIdx.x] = r;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double o = smax[threadIdx.x + w];
            if (o > smax[threadIdx.x] || o != o) smax[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) I.resid[0] = smax[0] / I.dt;
}

// ------------------------------------------------------------------ launchers

hipError_t launch_moments(const DevInstance* d, int ninst, int maxnr, int buf, hipStream_t s)
{
    hipLaunchKernelGGL(k_moments, dim3(maxnr, ninst), dim3(kBlock), 0, s, d, buf);
    return hipGetLastError();
}

hipError_t launch_node(const DevInstance* d, int ninst, int maxnr, int src, bool with_geq, hipStream_t s)
{
    const int nchunks = (maxnr + kNodeChunk - 1) / kNodeChunk;
    hipLaunchKernelGGL(k_node, dim3(nchunks + 2, ninst), dim3(kBlock), 0, s, d, src);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_proj, dim3((maxnr + 3) / 4, ninst), dim3(kBlock), 0, s, d);
    e = hipGetLastError();
    if (e != hipSuccess || !with_geq) return e;
    hipLaunchKernelGGL(k_geq, dim3(64, ninst), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_stage_kernel(const DevInstance* d, int ninst, int maxnr, int maxnv, int src, int fn, int dst,
                               double an, double bs, int mode, hipStream_t s)
{
    hipLaunchKernelGGL(k_stage, dim3(maxnr, ninst), dim3(kBlock), (size_t)maxnv * sizeof(double), s, d, src, fn, dst,
                       an, bs, mode);
    return hipGetLastError();
}

template <int VPT>
static hipError_t launch_stage2_t(const DevInstance* d, const WorkItem* items, int nitems, const StageGroup& G, int src,
                                  int fn, int dst, double an, double bs, hipStream_t s)
{
    hipLaunchKernelGGL(k_stage2<VPT>, dim3(nitems), dim3(G.block), (size_t)G.lds_doubles * sizeof(double), s, d,
                       items, G, src, fn, dst, an, bs);
    return hipGetLastError();
}

hipError_t launch_stage2(const DevInstance* d, const WorkItem* items, int nitems, const StageGroup& G, int src, int fn,
                         int dst, double an, double bs, hipStream_t s)
{
    switch (G.vpt) {
        case 1: return launch_stage2_t<1>(d, items, nitems, G, src, fn, dst, an, bs, s);
        case 2: return launch_stage2_t<2>(d, items, nitems, G, src, fn, dst, an, bs, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t set_stage2_smem_limit()
{
    const int bytes = 160 * 1024;
    hipError_t e = hipSuccess;
    e = hipFuncSetAttribute((const void*)k_stage2<1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_stage2<2>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}

hipError_t launch_snapshot(const DevInstance* d, int ninst, hipStream_t s)
{
    hipLaunchKernelGGL(k_snapshot, dim3(1, ninst), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_residual(const DevInstance* d, int ninst, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual, dim3(1, ninst), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

hipError_t set_stage_smem_limit(int maxnv)
{
    return hipFuncSetAttribute((const void*)k_stage, hipFuncAttributeMaxDynamicSharedMemorySize,
                               maxnv * (int)sizeof(double));
}

}  // namespace lbe
