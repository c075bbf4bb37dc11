// Internal declarations of liblbe: host-side tables and the per-instance device descriptor.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/lbe.h"

namespace lbe {

constexpr int kMaxQ = 100;   // largest quadrature order per axis (host tables; the stage kernel takes less, see plan_groups)
constexpr int kMaxN = 15;    // largest equilibrium expansion order
constexpr int kNodeStride = 96;  // doubles per node in the node-coefficient block
constexpr int kMomStride = 16;   // doubles per node in the moment-sum block
constexpr int kProjGauss = 32;   // nodes per side of the projection kernel's half-range Gauss rule

// Node-coefficient block layout (doubles, per node), written by the node kernel.  NF_PHI, NF_FR:
// mean-field potential and radial force of the attractive tail (zero without attraction).
enum NodeField {
    NF_N = 0, NF_U0, NF_U1, NF_U2, NF_T, NF_Q0, NF_Q1, NF_Q2,
    NF_TAU, NF_PR, NF_BRHOCHI, NF_D1, NF_D2, NF_DU0, NF_DU1, NF_DU2,
    NF_NBAR, NF_CHI, NF_P01, NF_SHAK, NF_INVTAU, NF_DIVU, NF_SHEAR01, NF_UPHI_R,
    NF_UR_R, NF_INV2T, NF_INV5T, NF_PHI, NF_FR, NF_COUNT,
    // equilibrium projection coefficients (Sec. III.C): half-range I_l^+ and I_l^- of the
    // radial axis, full-range c_l of the two transverse axes (16 slots each)
    NF_IPLUS = 32, NF_IMINUS = 48, NF_C1 = 64, NF_C2 = 80
};
static_assert(NF_COUNT <= NF_IPLUS, "node scalars overlap the projection coefficients");

// Moment-sum block layout (doubles, per node), written by the stage kernel: sums of f times
// powers of xi' = p - c, where c is the shift stored with the block.
enum MomField {
    MF_S0 = 0, MF_S1X, MF_S1Y, MF_S1Z,
    MF_SXX, MF_SYY, MF_SZZ, MF_SXY, MF_SXZ, MF_SYZ,
    MF_S3X, MF_S3Y, MF_S3Z, MF_CX, MF_CY, MF_CZ
};

// Per-axis quadrature and the equilibrium tables of that axis.
struct AxisTables {
    bool half = false;
    int Q = 0;      // order
    int nq = 0;     // nodes (2Q for half-range)
    int N = 0;      // expansion order
    std::vector<double> p, w;    // nodes, weights
    std::vector<double> poly;    // nq x (N+1): h_l(|p_k|) (half) or He_l(p_k) (full)
    std::vector<double> qy, qlam;  // half-range: projection rule on [0, Y] (nodes, weights)
    double qpanel = 0.75;          // half-range: panel width of that rule (16 nodes per panel)
    std::vector<double> qh;        // half-range: h_l(qy_m), M x (N+1)
    std::vector<double> qrec;      // half-range, from x h_l = b_{l+1} h_{l+1} + a_l h_l + b_l h_{l-1}:
                                   // (a_l, b_l^2) for l < N, then h_0 / (b_1 ... b_l) for l <= N
    std::vector<double> gx, gw;    // half-range: the kProjGauss-point Gauss rule for exp(-x^2/2)/sqrt(2 pi)
                                   // on [0, inf) (projection at moderate u / sqrt(T))
};

// Everything the host precomputes for one instance.
struct InstanceTables {
    lbe_params prm{};
    int nr = 0, nv = 0, n0 = 0, n1 = 0, n2 = 0;
    double chi0 = 0, C = 0, L = 0, sigma = 0, rcl = 0, rcr = 0, dr = 0, dt = 0;
    AxisTables ax[3];
    std::vector<double> K1, K2a, K2b;     // force matrices used by the model
    std::vector<double> K2r;              // d(f p)/dp along the radial axis (tables only)
    std::vector<double> r, ri;            // node and interface radii
    std::vector<double> geo;              // per node: adv_l, adv_r, force_fac, 1/r
    int wband = 0;                        // band width of W
    std::vector<int32_t> wlo;             // first column of each band row
    std::vector<double> wb;               // nr x wband band of W
    std::vector<double> gwl, gwr;         // unit wall Maxwellians [nv]
    double gin_l = 0, gin_r = 0;          // sum over entering velocities of p_r * g_w
    std::vector<double> amf;              // nr x nr mean-field weights (empty without attraction)
};

// Device descriptor of one instance (lives in device memory; pointers into the workspace).
struct DevInstance {
    int32_t nr, nv, n0, n1, n2, geometry;
    int32_t f32, reduced;  // f32 1: state buffers hold FP32 deviations from base[] (LBE_FP32_STORE);
                           // reduced 1: the planes i2 = 0, 1 are phi, chi (p_z integrated out)
    int32_t N0, N1, N2, wband;
    double dt, dr, eta0, kn, chi0, L, gin_l, gin_r;
    double rcl, rcr, uw, tratio;  // computational walls, inner wall speed, T_outer / T_inner
    double* f[3];           // state buffers [nr][nv] (FP64, or FP32 when f32; two ghost rows on each
                            // side); f[0] holds the state between steps
    double* base[4];        // f32: per node (n g_0[n0], g_1[n1], g_2[n2]), the discrete equilibrium a
                            // buffer's deviations are taken from: f = dev + B0[i0] (B1[i1] B2[i2]).
                            // Tables 0, 1, 2 belong to buffers 0, 1, 2; the third stage writes
                            // buffer 0's new table into 3, copied to 0 after the step
    double* mom;            // [nr][nslices][kMomStride] moment sums of the last written buffer (per slice)
    double* node;           // [nr][kNodeStride] node coefficients of the current stage
    const double* p0; const double* p1; const double* p2;
    const double* K1; const double* K2a; const double* K2b;
    const double* w0; const double* w1; const double* w2;
    const double* poly0; const double* poly1; const double* poly2;
    const double* qy0; const double* qlam0;  // projection rule, M0 nodes
    const double* qrec0;    // recurrence of the half-range polynomials (AxisTables::qrec)
    const double* pgx0; const double* pgw0;  // half-range Gauss rule of the projection (kProjGauss nodes)
    int32_t M0, nslices;    // equilibrium projection nodes; velocity slices of the stage kernel
    double qpw;             // panel width of the projection rule
    const double* geo;      // [nr][4]
    const double* r;        // [nr]
    const int32_t* wlo;     // [nr]
    const double* wb;       // [nr][wband]
    const double* gwl; const double* gwr;  // [nv]
    double* snap;           // [nr][5] moments at the start of the last step (residual)
    double* resid;          // [1] last residual
    int32_t* flags;         // [4] 0: nan flag, 1: active (1) / frozen (0)
    double* nw;             // [2] wall densities of the current stage
    double* scratch;        // [nr][nv] rhs output (lbe_rhs); staging of lbe_set_init_moments
    const double* rest;     // [n0 + n1 + n2] equilibrium factors at rest (n = 1, u = 0, T = 1)
    const double* amf;      // [nr][nr] mean-field weights, null without attraction
    double* simg;           // [nslices][img_sz] constant part of the stage kernel's LDS per slice
};

// One unit of stage-kernel work: a tile of consecutive nodes of one instance, one velocity slice.
struct WorkItem {
    int32_t inst, i0, nt, slice;
};

constexpr int kMaxTilePerm = 128;  // largest tile count with a balanced slot order
constexpr int kTileDescStride = 16;  // ints per MFMA tile descriptor of the stage kernel

// Launch group of the stage kernel: instances sharing one velocity set (n0, n1, n2, geometry).
// All sizes are uniform over the group; LDS offsets are in doubles.
struct StageGroup {
    int32_t n0, n1, n2, nv, geometry, f32, reduced;
    int32_t S, ns2, nvs, ncols_s, ncols16, plane_cols;  // slices, i2 / velocities / columns per slice
    int32_t ncp16;                                       // d2 columns (n0 n1, sphere) padded to 16
    int32_t plane_sz, op_sz, ib_sz;                      // doubles per plane / output / term buffer
    int32_t n0k, n1k, n2k, n0p, n1p, ns2p;              // K padded to 4, M/N padded to 16
    int32_t NT, block, vpt, wh;                          // nodes per tile, lanes, velocities per lane,
                                                         // waves per sign of the radial momentum
    int32_t nperm;                                       // MFMA tiles when perm is used, else 0
    int16_t perm[kMaxTilePerm];                          // logical tile of each launch slot
    int32_t off_plane, off_op, off_ibuf, off_K1, off_K2a, off_K2b, off_colfac, off_cpinfo, off_tdesc, off_pv,
        off_y0p, off_psi, off_coef, off_geq, off_part, lds_doubles;
    int32_t img_sz;    // doubles of the stage image per slice: img_lds, then poly_sz
    int32_t img_lds;   // its constant LDS part, copied to [off_K1, off_y0p) (even)
    int32_t poly_sz;   // its set-up part, copied to off_poly: expansion polynomials (stride pstride)
    int32_t pstride;   // and weights of every factor (even); off_poly is the term buffers when they
    int32_t off_poly;  // have room (they are written before they are read), else a region of its own
    int32_t ntiles;    // MFMA tiles per node (moment, d0, d1, d2 tiles)
    int32_t xcdmap;    // 1: workgroup b runs work item xcd_item(b), so each XCD takes a contiguous
                       // run of the item list (LBE_XCD_MAP=0 in the environment: item b)
    int32_t off_sb, off_fb, bstride;  // f32: base factors of the window rows / own rows (stride bstride)
};

constexpr int kCoefStride = 20;  // doubles per node of the stage kernel's coefficient block

// Network of the learned warm start (lbe_mlp.hip): buffers and the forward pass used by
// lbe_warm_start.  Outputs are standardised: physical = mean + scale * output.
int mlp_max_rows(const lbe_mlp* m);
float* mlp_input(lbe_mlp* m);
const float* mlp_output(const lbe_mlp* m);
void mlp_scaling(const lbe_mlp* m, double* mean, double* scale);
hipError_t mlp_forward_rows(lbe_mlp* m, const float* X, int rows, hipStream_t s);

// Host table construction (lbe_tables.cpp).
lbe_status validate_params(const lbe_params& in, lbe_params* out, std::string* err);
lbe_status build_instance(const lbe_params& p, InstanceTables* t, std::string* err);
void equilibrium_axis(const AxisTables& ax, double u, double T, double* g);
double ball_in_cylinder(double s, double R, double b);
double ball_in_sphere(double s, double R, double b);
double ball_below_plane(double s, double X, double b);
double chi_cs(double eta);
double mf_potential(int geometry, double sigma, double phi_a, double r, double s);

}  // namespace lbe
