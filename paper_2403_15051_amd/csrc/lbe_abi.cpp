// C ABI of liblbe (declared in include/lbe.h): context set-up, workspace carving, the RK3
// driver, the steady-state driver and state access.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lbe_internal.h"

namespace lbe {
hipError_t launch_moments(const DevInstance* d, int ninst, int maxnr, int buf, int tab, int from_scratch, int only,
                          hipStream_t s);
hipError_t launch_node(const DevInstance* d, const int32_t* ilist, int ninst, int maxnr, int maxn0, int src, int bsrc,
                       hipStream_t s);
hipError_t launch_base_copy(const DevInstance* d, const int32_t* ilist, int ninst, int maxnr, int maxng, hipStream_t s);
hipError_t launch_expand(const DevInstance* d, int inst, int nr, hipStream_t s);
hipError_t launch_mass(const DevInstance* d, int ninst, int only, double* mass, hipStream_t s,
                       const int32_t* mask = nullptr);
hipError_t launch_mass_fix(const DevInstance* d, int ninst, int maxnr, const double* target, hipStream_t s);
hipError_t launch_rebase(const DevInstance* d, int inst, int nr, hipStream_t s);
hipError_t launch_rebase_masked(const DevInstance* d, int ninst, int maxnr, const int32_t* mask, hipStream_t s);
hipError_t launch_snapshot(const DevInstance* d, int ninst, hipStream_t s);
hipError_t launch_residual(const DevInstance* d, int ninst, hipStream_t s);
hipError_t launch_converge(const DevInstance* d, int ninst, double tol, int chunk, int judge, double* st,
                           hipStream_t s);
hipError_t launch_stage(const DevInstance* d, const WorkItem* items, int nitems, const StageGroup& G, int src, int fn,
                        int dst, double an, double bs, int rhs, int bsrc, int bfn, int bdst, hipStream_t s);
hipError_t set_stage_smem_limit();
hipError_t launch_stage_image(const DevInstance* d, const int32_t* ilist, int ninst, const StageGroup& G, hipStream_t s);
hipError_t launch_proj(const DevInstance* d, int ninst, int maxnr, hipStream_t s);
hipError_t launch_warm_profile_net(const DevInstance* d, const int32_t* rowoff, int ninst, int r0, int rows,
                                   float* X, const float* Y, const double* mean, const double* scale,
                                   const int32_t* mask, int features_only, hipStream_t s);
hipError_t launch_profile_from_host(const DevInstance* d, int inst, hipStream_t s);
hipError_t launch_grad13(const DevInstance* d, int ninst, int maxnr, const int32_t* mask, hipStream_t s);
hipError_t launch_rest(const DevInstance* d, int ninst, int maxnr, const int32_t* mask, hipStream_t s);
hipError_t launch_renorm(const DevInstance* d, int ninst, const int32_t* mask, hipStream_t s);
hipError_t launch_collect_resid(const DevInstance* d, int ninst, double* out, hipStream_t s);
}  // namespace lbe

using namespace lbe;

// Largest velocity plane the stage kernel stages in LDS (FP64): 160 KB per CU.
static constexpr int kMaxPlane = 20000;
// Tile heights (nodes per stage work item) lbe_autotune tries.
static constexpr int kTileCandidates[] = {4, 8, 16, 32, 64};
static constexpr int kMinTileNodes = 4;
// FP32 storage: steps between mass fixes in lbe_step (lbe_run_to_steady fixes once per interval)
static constexpr int kMassFixEvery = 10;

struct lbe_ctx {
    std::vector<InstanceTables> tabs;
    std::vector<DevInstance> host_desc;
    DevInstance* dev_desc = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    int ninst = 0, maxnr = 0, maxnv = 0, maxng = 0;
    int maxn0 = 0;  // largest radial expansion order (the node kernel projects orders below 8 itself)
    bool any_f32 = false;
    std::vector<int64_t> steps;
    std::vector<int32_t> active;
    std::string err;
    bool nan_latched = false;
    // optional per-launch timing of the stage and node kernels (lbe_timing)
    bool timing = false;
    std::vector<hipEvent_t> ev;       // pool, reused
    size_t ev_used = 0;
    std::vector<std::pair<int, int>> stage_ev, node_ev;  // (start, stop) indices into ev
    // stage-kernel launch groups and their work items (device copy in the workspace)
    std::vector<StageGroup> groups;
    std::vector<int> group_of;         // instance -> group
    std::vector<int> item_off, item_cnt;
    std::vector<WorkItem> items;
    WorkItem* dev_items = nullptr;
    size_t items_cap = 0;              // work items the device list has room for
    // steady-state bookkeeping [ninst][4] (residual, steps, nan flag, active), device side
    double* dev_status = nullptr;
    // warm start: first row (node) of every instance [ninst + 1], instance mask [ninst], residuals
    int32_t* dev_rowoff = nullptr;
    int32_t* dev_mask = nullptr;
    double* dev_vec = nullptr;
    // FP32 storage: target mass of every instance; steps since the last mass fix (lbe_step)
    double* dev_mass = nullptr;
    int64_t since_fix = 0;
    std::vector<int32_t> rowoff;
    // instances ordered by launch group (device), and per group: offset, count, largest nr and
    // velocity-factor count, FP32 storage; streams and events that fork a step into one chain of
    // launches per group and join them again (independent groups overlap on the device)
    int32_t* dev_glist = nullptr;
    std::vector<int> gl_off, gl_cnt, gl_maxnr, gl_maxng;
    std::vector<char> gl_f32;
    std::vector<hipStream_t> gstreams;
    std::vector<hipEvent_t> gevents;
    // captured launch sequences: one RK3 step, and one steady-state chunk (chunk steps, the
    // residual and the freeze test), replayed on `stream`; captured on a private stream
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t g_step = nullptr, g_chunk = nullptr;
    int g_chunk_n = 0;
    double g_chunk_tol = 0;
    // device whose static workspace this context occupies (lbe_init_static), -1 otherwise
    int static_dev = -1;
    // FP32 storage: start of each state buffer's allocation (laid out at FP64 size, so that an
    // instance can switch to FP64 storage in place), and the step at which each instance did
    // (-1: never); the steady driver switches a launch group whose solves have stopped improving
    std::vector<std::array<char*, 3>> fraw;
    std::vector<int64_t> promoted_at;
    bool promote = true;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte layout of one instance inside the workspace.
struct Layout {
    size_t fraw[3], f[3], mom, node, snap, resid, flags, nw, scratch;
    size_t base[4], rest, p0, p1, p2, K1, K2a, K2b, w0, w1, w2, poly0, poly1, poly2, qy0, qlam0, qrec0, pgx0, pgw0, geo, r, wlo, wb, gwl, gwr;
    size_t amf;  // mean-field weights (0 without attraction)
    size_t simg;
    size_t total;
};

Layout make_layout(const InstanceTables& t, int nslices, size_t img_doubles, size_t base)
{
    Layout L;
    size_t o = base;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t D = sizeof(double);
    const size_t plane = (size_t)t.nr * t.nv * D;
    // state buffers: nr rows plus two ghost rows on each side (filled by the node kernel);
    // L.f points at row 0; FP64 or FP32 values.  Each buffer is sized for FP64 values, so that an
    // FP32-storage instance can be switched to FP64 storage in place (the FP32 values use the
    // first half; the bytes streamed per step are those of the stored precision)
    const size_t E = t.prm.precision == LBE_FP32_STORE ? sizeof(float) : D;
    for (int k = 0; k < 3; k++) {
        L.fraw[k] = take((size_t)(t.nr + 4) * t.nv * D);
        L.f[k] = L.fraw[k] + 2 * t.nv * E;
    }
    const size_t ng = (size_t)(t.n0 + t.n1 + t.n2);
    for (int k = 0; k < 4; k++) L.base[k] = t.prm.precision == LBE_FP32_STORE ? take((size_t)t.nr * ng * D) : 0;
    L.mom = take((size_t)t.nr * nslices * kMomStride * D);
    L.node = take((size_t)t.nr * kNodeStride * D);
    L.snap = take((size_t)t.nr * 5 * D);
    L.resid = take(D);
    L.flags = take(4 * sizeof(int32_t));
    L.nw = take(2 * D);
    L.scratch = take(plane);
    L.rest = take((size_t)(t.n0 + t.n1 + t.n2) * D);
    L.p0 = take(t.n0 * D);
    L.p1 = take(t.n1 * D);
    L.p2 = take(t.n2 * D);
    L.K1 = take(t.K1.size() * D);
    L.K2a = take(t.K2a.size() * D);
    L.K2b = take(t.K2b.size() * D);
    L.w0 = take(t.n0 * D);
    L.w1 = take(t.n1 * D);
    L.w2 = take(t.n2 * D);
    L.poly0 = take(t.ax[0].poly.size() * D);
    L.poly1 = take(t.ax[1].poly.size() * D);
    L.poly2 = take(t.ax[2].poly.size() * D);
    L.qy0 = take(t.ax[0].qy.size() * D);
    L.qlam0 = take(t.ax[0].qlam.size() * D);
    L.qrec0 = take(t.ax[0].qrec.size() * D);
    L.pgx0 = take(kProjGauss * D);
    L.pgw0 = take(kProjGauss * D);
    L.geo = take(t.geo.size() * D);
    L.r = take(t.r.size() * D);
    L.wlo = take(t.wlo.size() * sizeof(int32_t));
    L.wb = take(t.wb.size() * D);
    L.gwl = take(t.nv * D);
    L.gwr = take(t.nv * D);
    L.amf = t.amf.empty() ? 0 : take(t.amf.size() * D);
    L.simg = take(img_doubles * D);
    L.total = o;
    return L;
}

// Doubles of the stage kernel's image of one slice when the velocity set is not sliced
// (layout_group's regions K1 .. p values, then the polynomials and weights at the largest
// order); every region shrinks or stays as the slices grow, so nslices times the sliced size
// never exceeds n2 times this.
size_t stage_image_bound(int n0, int n1, int n2, bool sph)
{
    auto r4 = [](int x) { return (size_t)(x + 3) / 4 * 4; };
    auto r16 = [](int x) { return (size_t)(x + 15) / 16 * 16; };
    const size_t n0p = r16(n0), n1p = r16(n1), n2p = r16(n2), nc16 = r16(n1 * n2), ncp16 = sph ? r16(n0 * n1) : 0;
    const size_t nTall = nc16 / 16 + (n0p / 16) * (nc16 / 16) + (size_t)n2 * (n1p / 16) * (n0p / 16) +
                         (sph ? (n2p / 16) * (ncp16 / 16) : 0);
    return n0p * (r4(n0) + 1) + n1p * (r4(n1) + 1) + (sph ? n2p * (r4(n2) + 1) : 0) + nc16 + n0p + ncp16 +
           (ncp16 + 1) / 2 + (nTall * kTileDescStride + 1) / 2 + n0p + 2 * nc16 + 1 +
           (size_t)(n0 + n1 + n2) * (kMaxN + 3) + 1;
}

// Sizes of a layout without building the tables (for lbe_query).
size_t instance_bytes_estimate(const lbe_params& p)
{
    const int n0 = 2 * p.q_radial, n1 = p.q_t1, n2 = p.q_t2;
    const size_t nv = (size_t)n0 * n1 * n2, nr = p.nr, D = sizeof(double);
    const int N = kMaxN + 2;
    // state buffers at FP64 size whatever the storage (an FP32 instance can switch in place)
    size_t b = align256((size_t)(n0 + n1 + n2) * D) + 3 * align256((nr + 4) * nv * D) + align256(nr * nv * D) +
               align256(nr * n2 * kMomStride * D) + align256(nr * kNodeStride * D) + align256(nr * 5 * D) + 3 * 256;
    b += 3 * align256(n0 * D) + align256((size_t)n0 * n0 * D) + align256((size_t)n1 * n1 * D) +
         align256((size_t)n2 * n2 * D) + 3 * align256(std::max(n0, std::max(n1, n2)) * D);
    b += 3 * align256((size_t)std::max(n0, std::max(n1, n2)) * N * D);
    // projection rule: as build_instance sizes it (panels of 16 nodes, width from the colder wall)
    const double Tmax = std::max(1.0, std::max(p.t_wall_inner, p.t_wall_outer));
    const double Tlow = 0.5 * std::min(p.t_wall_inner, p.t_wall_outer);
    const double hwidth = std::min(1.5, std::max(0.1875, 3.35 * std::sqrt(std::max(Tlow, 0.0))));
    const size_t M = (size_t)(16 * (std::ceil((3 + 13 * std::sqrt(1.5 * Tmax) + std::fabs(p.u_wall_inner)) / hwidth) + 1));
    b += 2 * align256(M * D) + align256((size_t)(3 * N + 1) * D) + 2 * align256(kProjGauss * D);
    b += 3 * align256(nr * 4 * D) + align256(nr * sizeof(int32_t)) + align256(nr * nr * D) + 2 * align256(nv * D);
    b += align256(nr * n2 * sizeof(WorkItem));
    b += 4 * align256(nr * (size_t)(n0 + n1 + n2) * D);
    b += align256((size_t)n2 * stage_image_bound(n0, n1, n2, p.geometry == LBE_SPH) * D);
    if (p.phi_a != 0) b += align256(nr * nr * D);  // mean-field weights
    return b + 4096;
}

// Launch groups of the stage kernel: instances with the same velocity set share one launch.
// Per group: velocity slices S (a divisor of n2; raised while the whole batch has fewer than
// two work items per compute unit), lanes per workgroup and velocities per lane (about 4),
// nodes per tile, and the LDS layout.
constexpr int kLdsDoubles = 160 * 1024 / 8;

bool layout_group(StageGroup* G, int nt0)
{
    const int n0 = G->n0, n1 = G->n1, n2 = G->n2;
    const bool sph = G->geometry == LBE_SPH;
    G->ns2 = n2 / G->S;
    G->nvs = G->nv / G->S;
    G->ncols_s = n1 * G->ns2;
    G->ncols16 = (G->ncols_s + 15) / 16 * 16;
    G->ncp16 = sph ? (n0 * n1 + 15) / 16 * 16 : 0;
    G->plane_cols = sph ? n1 * n2 : G->ncols_s;
    G->n0k = (n0 + 3) / 4 * 4;
    G->n1k = (n1 + 3) / 4 * 4;
    G->n2k = (n2 + 3) / 4 * 4;
    G->n0p = (n0 + 15) / 16 * 16;
    G->n1p = (n1 + 15) / 16 * 16;
    G->ns2p = (G->ns2 + 15) / 16 * 16;
    // lanes: wh waves for the velocities with p_r > 0, wh for p_r < 0, one or two per lane
    const int nh = (n0 / 2) * G->ncols_s;
    if (nh <= 512) {
        G->vpt = 1;
        G->wh = (nh + 63) / 64;
    } else if (nh <= 1024) {
        G->vpt = 2;
        G->wh = (nh + 127) / 128;
    } else {
        return false;
    }
    G->block = 128 * G->wh;
    const int ng = n0 + n1 + n2, cs = n0 + 1;
    // extent of the plane read by the MFMA operands, padding included (d0, d1, d2)
    const int c_last = sph ? (G->S - 1) * G->ncols_s : 0;
    int pmax = (G->n0k - 1) + cs * (c_last + G->ncols16 - 1);
    pmax = std::max(pmax, (G->n0p - 1) + cs * ((sph ? n1 * (n2 - 1) : n1 * (G->ns2 - 1)) + G->n1k - 1));
    if (sph) pmax = std::max(pmax, (n0 - 1) + cs * ((n1 - 1) + n1 * (G->n2k - 1)));
    pmax = std::max(pmax, cs * G->plane_cols - 1);
    const int op_sz = std::max((G->n0k - 1) + cs * (G->ncols16 - 1) + 1, cs * G->ncols_s);
    const int nTm = G->ncols16 / 16;
    const int nTall = nTm + (G->n0p / 16) * (G->ncols16 / 16) + G->ns2 * (G->n1p / 16) * (G->n0p / 16) +
                      (sph ? (G->ns2p / 16) * (G->ncp16 / 16) : 0);
    G->ntiles = nTall;
    // a few more MFMA tiles than waves (the 12^3 set's slices: 15 tiles over 14 waves): add the
    // waves that give each tile a wave of its own (their lanes hold no velocity) when that adds at
    // most a quarter to the workgroup; the tile waves set the node interval, so two tiles on one
    // wave cost more than a few idle lanes (not more than tripling a small workgroup's lanes)
    if (G->vpt == 1 && nTall > 2 * G->wh && 4 * ((nTall + 1) / 2 - G->wh) <= G->wh &&
        (nTall + 1) / 2 * 128 <= 1024) {
        G->wh = (nTall + 1) / 2;
        G->block = 128 * G->wh;
    }
    // slot order of the MFMA tiles: heaviest first, each into the free slot whose SIMD (slot is
    // run by wave slot % W, on SIMD wave % 4) has the least MFMA work so far
    {
        const int W = G->block / 64;
        const int nT1 = (G->n0p / 16) * (G->ncols16 / 16), nT2 = G->ns2 * (G->n1p / 16) * (G->n0p / 16);
        std::vector<std::pair<int, int>> tiles;  // (weight, logical tile)
        for (int k = 0; k < nTall; k++) {
            int wgt;
            // in cycles of the matrix core / 16: a 16x16x4 FP64 MFMA is 4, a 4x4x4 one is 1
            if (k < nTm) wgt = G->n0k / 4 + 3;
            else if (k < nTm + nT1) wgt = G->n0k;
            else if (k < nTm + nT1 + nT2) wgt = G->n1k;
            else wgt = G->n2k;
            tiles.push_back({wgt, k});
        }
        std::stable_sort(tiles.begin(), tiles.end(), [](auto& a, auto& b) { return a.first > b.first; });
        if (nTall <= kMaxTilePerm) {
            std::vector<int> used(nTall, 0);
            long load[4] = {0, 0, 0, 0};
            for (auto& tw : tiles) {
                int best = -1;
                for (int sl = 0; sl < nTall; sl++) {
                    if (used[sl]) continue;
                    if (best < 0 || load[(sl % W) % 4] < load[(best % W) % 4]) best = sl;
                }
                used[best] = 1;
                G->perm[best] = (int16_t)tw.second;
                load[(best % W) % 4] += tw.first;
            }
            G->nperm = nTall;
        } else {
            G->nperm = 0;
        }
    }
    for (int NT = nt0; NT >= 1; NT /= 2) {
        G->NT = NT;
        int o = 0;
        // two of each: plane of the node being contracted, output plane of the node whose
        // moments are taken, inertial-term planes (d0, d1 (, d2)) of the node being updated
        G->plane_sz = pmax + 1;
        G->op_sz = op_sz;
        G->ib_sz = (sph ? 3 : 2) * cs * G->ncols_s;
        G->off_plane = o;
        o += 2 * G->plane_sz;
        G->off_op = o;
        o += 2 * G->op_sz;
        G->off_ibuf = o;
        o += 2 * G->ib_sz;
        G->off_K1 = o;
        o += G->n0p * (G->n0k + 1);
        G->off_K2a = o;
        o += G->n1p * (G->n1k + 1);
        G->off_K2b = o;
        o += sph ? G->ns2p * (G->n2k + 1) : 0;
        G->off_colfac = o;  // d0 column factors, -p_r per radial node, -p_r per d2 column
        o += G->ncols16 + G->n0p + G->ncp16;
        G->off_cpinfo = o;  // ints, two per double
        o += (G->ncp16 + 1) / 2;
        G->off_tdesc = o;   // ints
        o += (nTall * kTileDescStride + 1) / 2;
        G->off_pv = o;      // p_r per radial node, p_1 and p_2 per column of the slice
        o += G->n0p + 2 * G->ncols16;
        o += (o - G->off_K1) & 1;  // the image is copied two doubles at a time
        G->img_lds = o - G->off_K1;
        G->poly_sz = ng * G->pstride + ng;
        G->poly_sz += G->poly_sz & 1;
        G->img_sz = G->img_lds + G->poly_sz;
        G->off_y0p = o;  // powers 0..3 of y_r per radial node
        o += G->n0k * 4;
        G->off_psi = o;
        o += G->ncols16 * 16;
        G->off_coef = o;
        o += NT * kCoefStride;
        G->off_geq = o;
        o += NT * ng;
        G->off_part = o;
        o += NT * nTm * 36;
        // FP32 storage: base factors of the window rows and of the own rows of f^n
        G->bstride = n0 + G->plane_cols;
        G->off_sb = o;
        o += G->f32 ? (NT + 6) * G->bstride : 0;
        G->off_fb = o;
        o += G->f32 ? NT * G->bstride : 0;
        if (G->poly_sz <= 2 * G->ib_sz) {
            G->off_poly = G->off_ibuf;
        } else {
            o += o & 1;
            G->off_poly = o;
            o += G->poly_sz;
        }
        G->lds_doubles = o;
        if (o <= kLdsDoubles) return true;
    }
    return false;
}

// Default nodes per stage work item (LBE_TILE_NODES overrides it; lbe_autotune picks per group).
int default_tile_nodes()
{
    int nt0 = 16;
    if (const char* e = std::getenv("LBE_TILE_NODES")) nt0 = std::max(1, std::min(64, std::atoi(e)));
    return nt0;
}

// Work items of every group: tiles of G.NT consecutive nodes x velocity slices, grouped by launch.
// (only: the instances to include, all when null)
void build_items(lbe_ctx* c, const std::vector<int32_t>* only = nullptr)
{
    c->items.clear();
    c->item_off.assign(c->groups.size(), 0);
    c->item_cnt.assign(c->groups.size(), 0);
    for (size_t q = 0; q < c->groups.size(); q++) {
        const StageGroup& G = c->groups[q];
        c->item_off[q] = (int)c->items.size();
        for (int k = 0; k < c->ninst; k++) {
            if (c->group_of[k] != (int)q || (only && !(*only)[k])) continue;
            const int nr = c->tabs[k].nr;
            for (int i0 = 0; i0 < nr; i0 += G.NT)
                for (int sl = 0; sl < G.S; sl++) c->items.push_back({k, i0, std::min(G.NT, nr - i0), sl});
        }
        c->item_cnt[q] = (int)c->items.size() - c->item_off[q];
    }
}

// Velocity slices of a launch group: one velocity per lane and workgroups of at most `cap`
// lanes (slice while a slice holds more velocities than that; LBE_SLICE_CAP overrides the default
// for tuning), then further while the velocity set needs more than two per lane or the LDS does
// not fit.  False when no slicing of the transverse-2 axis makes it fit.
bool slice_group(StageGroup* G)
{
    int cap = 1024;
    if (const char* e = std::getenv("LBE_SLICE_CAP")) cap = std::max(64, std::atoi(e));
    auto next_slices = [&]() {
        int nextS = G->S + 1;
        while (nextS <= G->n2 && G->n2 % nextS) nextS++;
        return nextS;
    };
    for (;;) {
        const int nextS = next_slices();
        if (G->nv / G->S <= cap || nextS > G->n2) break;
        G->S = nextS;
    }
    while (!layout_group(G, default_tile_nodes())) {
        const int nextS = next_slices();
        if (nextS > G->n2) return false;
        G->S = nextS;
    }
    return true;
}

// Launch group of one validated problem statement on its own (the slicing plan_groups starts from).
StageGroup single_group(const lbe_params& q)
{
    StageGroup G;
    std::memset(&G, 0, sizeof(G));
    G.n0 = 2 * q.q_radial;
    G.n1 = q.q_t1;
    G.n2 = q.q_t2;
    G.nv = G.n0 * G.n1 * G.n2;
    G.geometry = q.geometry;
    G.f32 = q.precision == LBE_FP32_STORE;
    G.reduced = q.reduced;
    G.S = 1;
    G.pstride = (std::max(q.n_expand[0], std::max(q.n_expand[1], q.n_expand[2])) + 1) | 1;
    return G;
}

lbe_status plan_groups(lbe_ctx* c)
{
    c->groups.clear();
    c->group_of.assign(c->ninst, -1);
    for (int k = 0; k < c->ninst; k++) {
        const InstanceTables& t = c->tabs[k];
        int g = -1;
        for (size_t q = 0; q < c->groups.size(); q++) {
            const StageGroup& G = c->groups[q];
            if (G.n0 == t.n0 && G.n1 == t.n1 && G.n2 == t.n2 && G.geometry == t.prm.geometry &&
                G.f32 == (t.prm.precision == LBE_FP32_STORE) && G.reduced == t.prm.reduced)
                g = (int)q;
        }
        if (g < 0) {
            StageGroup G;
            std::memset(&G, 0, sizeof(G));
            G.n0 = t.n0;
            G.n1 = t.n1;
            G.n2 = t.n2;
            G.nv = t.nv;
            G.geometry = t.prm.geometry;
            G.f32 = t.prm.precision == LBE_FP32_STORE;
            G.reduced = t.prm.reduced;
            G.S = 1;
            G.pstride = 1;
            c->groups.push_back(G);
            g = (int)c->groups.size() - 1;
        }
        c->group_of[k] = g;
        // row stride of the expansion polynomials in the stage kernel's LDS: the largest order
        // of the group plus one, odd
        const int nmax = std::max(t.ax[0].N, std::max(t.ax[1].N, t.ax[2].N)) + 1;
        c->groups[g].pstride = std::max(c->groups[g].pstride, nmax | 1);
    }
    // a velocity set holding more than a third of the batch's site-velocities is split into two
    // launch groups (alternate instances), so that the node and projection kernels of one half
    // overlap the stage kernel of the other
    {
        std::vector<double> work(c->groups.size(), 0.0);
        double total = 0;
        for (int k = 0; k < c->ninst; k++) {
            const double w = (double)c->tabs[k].nr * c->tabs[k].nv;
            work[c->group_of[k]] += w;
            total += w;
        }
        const size_t ng0 = c->groups.size();
        for (size_t q = 0; q < ng0; q++) {
            int members = 0;
            for (int k = 0; k < c->ninst; k++) members += c->group_of[k] == (int)q;
            if (work[q] <= total / 3 || members < 2) continue;
            c->groups.push_back(c->groups[q]);
            const int g2 = (int)c->groups.size() - 1;
            int idx = 0;
            for (int k = 0; k < c->ninst; k++)
                if (c->group_of[k] == (int)q && (idx++ & 1)) c->group_of[k] = g2;
        }
    }
    auto total_items = [&]() {
        long tot = 0;
        for (int k = 0; k < c->ninst; k++) {
            const StageGroup& G = c->groups[c->group_of[k]];
            tot += (long)((c->tabs[k].nr + 15) / 16) * G.S;
        }
        return tot;
    };
    // more slices while the batch is too small to fill the chip (two items per compute unit)
    for (int guard = 0; guard < 64 && total_items() < 512; guard++) {
        int best = -1;
        for (size_t q = 0; q < c->groups.size(); q++) {
            const StageGroup& G = c->groups[q];
            int nextS = G.S + 1;
            while (nextS <= G.n2 && G.n2 % nextS) nextS++;
            if (nextS > G.n2 || G.nv / nextS < 256) continue;
            if (best < 0 || G.nv / G.S > c->groups[best].nv / c->groups[best].S) best = (int)q;
        }
        if (best < 0) break;
        StageGroup& G = c->groups[best];
        int nextS = G.S + 1;
        while (G.n2 % nextS) nextS++;
        G.S = nextS;
    }
    int xcdmap = 1;
    if (const char* e = std::getenv("LBE_XCD_MAP")) xcdmap = std::atoi(e) != 0;
    for (StageGroup& G : c->groups) {
        G.xcdmap = xcdmap;
        if (!slice_group(&G)) {
            c->err = "velocity set too large for the stage kernel (its LDS holds the radial force matrix)";
            return LBE_EINVAL;
        }
    }
    build_items(c);
    // room for the work items of the smallest tile height lbe_autotune tries
    c->items_cap = 0;
    for (int k = 0; k < c->ninst; k++)
        c->items_cap += (size_t)((c->tabs[k].nr + kMinTileNodes - 1) / kMinTileNodes) * c->groups[c->group_of[k]].S;
    c->items_cap = std::max(c->items_cap, c->items.size());
    return LBE_OK;
}

lbe_status dev_err(lbe_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return LBE_OK;
    if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
    return LBE_EDEVICE;
}

template <typename T>
hipError_t put(char* ws, size_t off, const std::vector<T>& v, hipStream_t s)
{
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(ws + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

lbe_status upload_flags(lbe_ctx* c)
{
    for (int k = 0; k < c->ninst; k++) {
        int32_t fl[4] = {0, c->active[k], 0, 0};
        hipError_t e = hipMemcpyAsync(c->host_desc[k].flags, fl, sizeof(fl), hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return dev_err(c, e, "flag upload");
    }
    return dev_err(c, hipStreamSynchronize(c->stream), "flag upload sync");
}

hipEvent_t next_event(lbe_ctx* c, int* idx)
{
    if (c->ev_used == c->ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev.push_back(e);
    }
    *idx = (int)c->ev_used;
    return c->ev[c->ev_used++];
}

// Node kernel then stage kernel of one RK stage, with events around each when timing.
void drop_graphs(lbe_ctx* c);

// Launch plan of the given instances (all when null): stage work items and per-group instance
// lists, uploaded to the device; the captured graphs are dropped (they hold the old plan).
hipError_t upload_plan(lbe_ctx* c, const std::vector<int32_t>* only)
{
    build_items(c, only);
    std::vector<int32_t> glist;
    c->gl_off.clear();
    c->gl_cnt.clear();
    c->gl_maxnr.clear();
    c->gl_maxng.clear();
    c->gl_f32.clear();
    for (size_t q = 0; q < c->groups.size(); q++) {
        c->gl_off.push_back((int)glist.size());
        int mnr = 0, mng = 0;
        for (int k = 0; k < c->ninst; k++)
            if (c->group_of[k] == (int)q && (!only || (*only)[k])) {
                glist.push_back(k);
                mnr = std::max(mnr, c->tabs[k].nr);
                mng = std::max(mng, c->tabs[k].n0 + c->tabs[k].n1 + c->tabs[k].n2);
            }
        c->gl_cnt.push_back((int)glist.size() - c->gl_off[q]);
        c->gl_maxnr.push_back(mnr);
        c->gl_maxng.push_back(mng);
        c->gl_f32.push_back(c->groups[q].f32 ? 1 : 0);
    }
    drop_graphs(c);
    hipError_t e = hipSuccess;
    if (!c->items.empty())
        e = hipMemcpyAsync(c->dev_items, c->items.data(), c->items.size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess && !glist.empty())
        e = hipMemcpyAsync(c->dev_glist, glist.data(), glist.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
}

// FP32-storage instances read src and f^n through base tables bsrc, bfn and write the output's
// base table bdst (ignored by FP64 instances).
hipError_t run_stage(lbe_ctx* c, int src, int fn, int dst, double an, double bs, int rhs, int bsrc, int bfn, int bdst)
{
    int a = -1, b = -1, x = -1, y = -1;
    hipError_t e;
    if (c->timing) (void)hipEventRecord(next_event(c, &a), c->stream);
    e = launch_node(c->dev_desc, nullptr, c->ninst, c->maxnr, c->maxn0, src, bsrc, c->stream);
    if (e != hipSuccess) return e;
    if (c->timing) {
        (void)hipEventRecord(next_event(c, &b), c->stream);
        c->node_ev.push_back({a, b});
        (void)hipEventRecord(next_event(c, &x), c->stream);
    }
    for (size_t q = 0; q < c->groups.size() && e == hipSuccess; q++)
        if (c->item_cnt[q] > 0)
            e = launch_stage(c->dev_desc, c->dev_items + c->item_off[q], c->item_cnt[q], c->groups[q], src, fn, dst, an,
                             bs, rhs, bsrc, bfn, bdst, c->stream);
    if (e != hipSuccess) return e;
    if (c->timing) {
        (void)hipEventRecord(next_event(c, &y), c->stream);
        c->stage_ev.push_back({x, y});
    }
    return hipSuccess;
}

// One TVD-RK3 step (Shu-Osher) of every active instance:
//   f1 = f + dt L(f);  f2 = 3/4 f + 1/4 (f1 + dt L(f1));  f <- 1/3 f + 2/3 (f2 + dt L(f2)).
// Whole batch, one launch per kernel (and per group for the stage kernel): the per-launch timing
// path and single-group contexts.
hipError_t launch_step_serial(lbe_ctx* c)
{
    hipError_t e = run_stage(c, 0, 0, 1, 0.0, 1.0, 0, 0, 0, 1);
    if (e == hipSuccess) e = run_stage(c, 1, 0, 2, 0.75, 0.25, 0, 1, 0, 2);
    if (e == hipSuccess) e = run_stage(c, 2, 0, 0, 1.0 / 3, 2.0 / 3, 0, 2, 0, 3);
    if (e == hipSuccess && c->any_f32)
        e = launch_base_copy(c->dev_desc, nullptr, c->ninst, c->maxnr, c->maxng, c->stream);
    return e;
}

// nsteps RK3 steps of launch group q only, on stream s.
hipError_t launch_steps_group(lbe_ctx* c, int q, int nsteps, hipStream_t s)
{
    const int32_t* il = c->dev_glist + c->gl_off[q];
    const int cnt = c->gl_cnt[q], mnr = c->gl_maxnr[q];
    if (cnt == 0 || c->item_cnt[q] == 0) return hipSuccess;
    // (src, fn, dst, an, bs, src table, f^n table, output table) of the three stages
    struct St {
        int src, fn, dst;
        double an, bs;
        int bsrc, bfn, bdst;
    };
    const St st[3] = {{0, 0, 1, 0.0, 1.0, 0, 0, 1}, {1, 0, 2, 0.75, 0.25, 1, 0, 2}, {2, 0, 0, 1.0 / 3, 2.0 / 3, 2, 0, 3}};
    hipError_t e = hipSuccess;
    for (int k = 0; k < nsteps && e == hipSuccess; k++) {
        for (int j = 0; j < 3 && e == hipSuccess; j++) {
            e = launch_node(c->dev_desc, il, cnt, mnr, c->maxn0, st[j].src, st[j].bsrc, s);
            if (e == hipSuccess)
                e = launch_stage(c->dev_desc, c->dev_items + c->item_off[q], c->item_cnt[q], c->groups[q], st[j].src,
                                 st[j].fn, st[j].dst, st[j].an, st[j].bs, 0, st[j].bsrc, st[j].bfn, st[j].bdst, s);
        }
        if (e == hipSuccess && c->gl_f32[q]) e = launch_base_copy(c->dev_desc, il, cnt, mnr, c->gl_maxng[q], s);
    }
    return e;
}

// nsteps steps of every group, each group a chain of launches on its own stream (forked from and
// joined back into the context's stream, default priorities); instances of different groups share
// no data within a step, so the chains overlap on the device.
hipError_t launch_steps_forked(lbe_ctx* c, int nsteps)
{
    const int ng = (int)c->groups.size();
    if (c->timing || ng == 1) {
        hipError_t e = hipSuccess;
        for (int k = 0; k < nsteps && e == hipSuccess; k++) e = launch_step_serial(c);
        return e;
    }
    hipError_t e = hipSuccess;
    while ((int)c->gstreams.size() < ng && e == hipSuccess) {
        hipStream_t t = nullptr;
        e = hipStreamCreateWithFlags(&t, hipStreamNonBlocking);
        if (e == hipSuccess) c->gstreams.push_back(t);
    }
    while ((int)c->gevents.size() < ng + 1 && e == hipSuccess) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) c->gevents.push_back(ev);
    }
    if (e == hipSuccess) e = hipEventRecord(c->gevents[ng], c->stream);
    for (int q = 1; q < ng && e == hipSuccess; q++) e = hipStreamWaitEvent(c->gstreams[q], c->gevents[ng], 0);
    // chains in order of increasing work (site-velocities of the group's work items), whatever the
    // order of the instances: on the sweep, the heaviest first made the step 2.5 % slower
    std::vector<int> ord(ng);
    for (int q = 0; q < ng; q++) ord[q] = q;
    auto work = [&](int q) { return (double)c->item_cnt[q] * c->groups[q].nvs * c->groups[q].NT; };
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return work(a) < work(b); });
    for (int k = 0; k < ng && e == hipSuccess; k++)
        e = launch_steps_group(c, ord[k], nsteps, k == 0 ? c->stream : c->gstreams[k]);
    // join (also after an error, so that no stream is left forked)
    for (int q = 1; q < ng; q++) {
        hipError_t ej = hipEventRecord(c->gevents[q], c->gstreams[q]);
        if (ej == hipSuccess) ej = hipStreamWaitEvent(c->stream, c->gevents[q], 0);
        if (e == hipSuccess) e = ej;
    }
    return e;
}

hipError_t launch_step(lbe_ctx* c) { return launch_steps_forked(c, 1); }

// `chunk` steps with the moment snapshot taken before the last one, then the residual of that
// step and the freeze test of every instance (lbe_run_to_steady).
hipError_t launch_chunk(lbe_ctx* c, int chunk, double tol, int judge)
{
    hipError_t e = hipSuccess;
    if (c->any_f32) e = launch_mass_fix(c->dev_desc, c->ninst, c->maxnr, c->dev_mass, c->stream);
    if (e == hipSuccess && chunk > 1) e = launch_steps_forked(c, chunk - 1);
    if (e == hipSuccess) e = launch_snapshot(c->dev_desc, c->ninst, c->stream);
    if (e == hipSuccess) e = launch_steps_forked(c, 1);
    if (e == hipSuccess) e = launch_residual(c->dev_desc, c->ninst, c->stream);
    if (e == hipSuccess) e = launch_converge(c->dev_desc, c->ninst, tol, chunk, judge, c->dev_status, c->stream);
    return e;
}

void drop_graphs(lbe_ctx* c)
{
    if (c->g_step) (void)hipGraphExecDestroy(c->g_step);
    if (c->g_chunk) (void)hipGraphExecDestroy(c->g_chunk);
    c->g_step = c->g_chunk = nullptr;
    c->g_chunk_n = 0;
}

// Record the launches `body` makes on the context's stream into an executable graph: the body
// runs with the context's stream swapped for a private capturing stream (nothing executes).
template <typename F>
hipError_t capture(lbe_ctx* c, F&& body, hipGraphExec_t* out)
{
    hipError_t e = hipSuccess;
    if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipError_t eb = body();
    c->stream = user;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->cap_stream, &g);
    if (eb != hipSuccess) e = eb;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

// Enqueue one RK3 step: replay of the captured step, or the launches themselves while the
// per-launch timing is on or graphs are disabled (LBE_GRAPH=0).
lbe_status enqueue_step(lbe_ctx* c)
{
    if (!c->use_graph || c->timing) return dev_err(c, launch_step(c), "step");
    if (!c->g_step) {
        lbe_status st = dev_err(c, capture(c, [&]() { return launch_step(c); }, &c->g_step), "step capture");
        if (st != LBE_OK) return st;
    }
    return dev_err(c, hipGraphLaunch(c->g_step, c->stream), "step launch");
}

lbe_status enqueue_chunk(lbe_ctx* c, int chunk, double tol, int judge)
{
    if (!c->use_graph || c->timing || !judge) return dev_err(c, launch_chunk(c, chunk, tol, judge), "chunk");
    if (!c->g_chunk || c->g_chunk_n != chunk || c->g_chunk_tol != tol) {
        if (c->g_chunk) (void)hipGraphExecDestroy(c->g_chunk);
        c->g_chunk = nullptr;
        lbe_status st = dev_err(
            c, capture(c, [&]() { return launch_chunk(c, chunk, tol, judge); }, &c->g_chunk), "chunk capture");
        if (st != LBE_OK) return st;
        c->g_chunk_n = chunk;
        c->g_chunk_tol = tol;
    }
    return dev_err(c, hipGraphLaunch(c->g_chunk, c->stream), "chunk launch");
}

// Switch every instance of launch group q from FP32 to FP64 storage, in place: buffer 0 becomes
// the FP64 state (the stored deviations plus their base, as lbe_get_state returns it), the
// instances' descriptors point at FP64 buffers (their allocations are FP64-sized) and the group's
// stage kernel takes its FP64 form.  The stage image does not depend on the storage, so it is
// kept.  `also`: another copy of the groups to keep in step (the steady driver's saved plan).
// The caller re-uploads the launch plan.
lbe_status promote_group(lbe_ctx* c, int q, int64_t at_step, std::vector<StageGroup>* also)
{
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    for (int k = 0; k < c->ninst && st == LBE_OK; k++) {
        if (c->group_of[k] != q || !c->host_desc[k].f32) continue;
        DevInstance& d = c->host_desc[k];
        const size_t plane = (size_t)d.nr * d.nv * sizeof(double);
        char* row0 = c->fraw[k][0] + 2 * (size_t)d.nv * sizeof(double);
        st = dev_err(c, launch_expand(c->dev_desc, k, d.nr, c->stream), "expand");
        if (st == LBE_OK)
            st = dev_err(c, hipMemcpyAsync(row0, d.scratch, plane, hipMemcpyDeviceToDevice, c->stream), "promote");
        if (st != LBE_OK) break;
        d.f32 = 0;
        for (int b = 0; b < 3; b++) d.f[b] = (double*)(c->fraw[k][b] + 2 * (size_t)d.nv * sizeof(double));
        c->tabs[k].prm.precision = LBE_FP64;
        c->promoted_at[k] = c->steps[k] + at_step;
    }
    if (st == LBE_OK)
        st = dev_err(c, hipMemcpyAsync(c->dev_desc, c->host_desc.data(), sizeof(DevInstance) * c->ninst,
                                       hipMemcpyHostToDevice, c->stream),
                     "descriptor upload");
    // moment sums of the FP64 states (the next stage's node kernel reads them)
    for (int k = 0; k < c->ninst && st == LBE_OK; k++)
        if (c->group_of[k] == q)
            st = dev_err(c, launch_moments(c->dev_desc, c->ninst, c->maxnr, 0, 0, 0, k, c->stream), "moments");
    if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    auto relayout = [&](StageGroup& G) {
        G.f32 = 0;
        return layout_group(&G, G.NT);
    };
    if (!relayout(c->groups[q]) || (also && !relayout((*also)[q]))) {
        c->err = "stage kernel layout of the promoted group";
        return LBE_EINVAL;
    }
    c->any_f32 = false;
    for (int k = 0; k < c->ninst; k++) c->any_f32 = c->any_f32 || c->host_desc[k].f32;
    drop_graphs(c);
    return LBE_OK;
}

lbe_status check_nan(lbe_ctx* c)
{
    for (int k = 0; k < c->ninst; k++) {
        int32_t fl = 0;
        hipError_t e = hipMemcpy(&fl, c->host_desc[k].flags, sizeof(int32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return dev_err(c, e, "flag read");
        if (fl) {
            c->nan_latched = true;
            c->err = "non-finite state or non-positive density/temperature in instance " + std::to_string(k);
        }
    }
    return c->nan_latched ? LBE_ENAN : LBE_OK;
}

}  // namespace

static __device__ __align__(256) char scratch[size_t(64) << 20];

namespace {

// Workspace of lbe_init_static: a file-scope device array, one copy per GPU, held by every GPU
// the library runs on until the process ends.  Host code never passes the array's name to the
// device (on the host it is only a stand-in symbol): the device address of each GPU's copy is
// looked up once per device with hipGetSymbolAddress and kept in static_ws_addr.
constexpr size_t kStaticWsBytes = size_t(64) << 20;
constexpr int kStaticMaxDevices = 64;
std::mutex static_ws_mu;
void* static_ws_addr[kStaticMaxDevices] = {};
bool static_ws_busy[kStaticMaxDevices] = {};
static_assert(sizeof(scratch) == kStaticWsBytes, "static workspace size");

}  // namespace

extern "C" {

const char* lbe_status_string(lbe_status s)
{
    switch (s) {
        case LBE_OK: return "ok";
        case LBE_EINVAL: return "invalid argument";
        case LBE_ENOMEM: return "out of memory / workspace too small";
        case LBE_EDEVICE: return "HIP runtime error";
        case LBE_ENOTCONV: return "not converged";
        case LBE_ENAN: return "non-finite state";
        case LBE_ESTATE: return "invalid state";
    }
    return "unknown status";
}

const char* lbe_last_error(const lbe_ctx* c) { return c ? c->err.c_str() : "null context"; }

lbe_status lbe_query(const lbe_params* p, int32_t n_inst, size_t* device_bytes, size_t* host_bytes)
{
    if (!p || n_inst < 1) return LBE_EINVAL;
    size_t total = align256(sizeof(DevInstance) * n_inst) + align256(4 * sizeof(double) * (size_t)n_inst) +
                   align256(sizeof(int32_t) * (size_t)(n_inst + 1)) + align256(sizeof(int32_t) * (size_t)n_inst) +
                   align256(2 * sizeof(double) * (size_t)n_inst) + align256(sizeof(double) * (size_t)n_inst) +
                   align256(sizeof(int32_t) * (size_t)n_inst);
    size_t host = sizeof(lbe_ctx);
    for (int k = 0; k < n_inst; k++) {
        lbe_params q;
        lbe_status st = validate_params(p[k], &q, nullptr);
        if (st != LBE_OK) return st;
        if ((size_t)2 * q.q_radial * q.q_t1 * q.q_t2 > (size_t)kMaxPlane) return LBE_EINVAL;
        StageGroup G = single_group(q);
        if (!slice_group(&G)) return LBE_EINVAL;  // the stage kernel cannot hold this velocity set
        total += instance_bytes_estimate(q);
        host += instance_bytes_estimate(q) / 8 + 4096;
    }
    if (device_bytes) *device_bytes = total;
    if (host_bytes) *host_bytes = host;
    return LBE_OK;
}

lbe_status lbe_init(const lbe_params* p, int32_t n_inst, void* device_ws, size_t ws_bytes, void* hip_stream,
                    lbe_ctx** out)
{
    if (!p || n_inst < 1 || !out || !device_ws) return LBE_EINVAL;
    if (((uintptr_t)device_ws & 255) != 0) return LBE_EINVAL;
    *out = nullptr;
    size_t need = 0;
    lbe_status st = lbe_query(p, n_inst, &need, nullptr);
    if (st != LBE_OK) return st;
    if (ws_bytes < need) return LBE_ENOMEM;
    lbe_ctx* c = new (std::nothrow) lbe_ctx;
    if (!c) return LBE_ENOMEM;
    c->ninst = n_inst;
    c->ws = (char*)device_ws;
    c->ws_bytes = ws_bytes;
    c->stream = (hipStream_t)hip_stream;
    c->tabs.resize(n_inst);
    c->host_desc.resize(n_inst);
    c->steps.assign(n_inst, 0);
    c->active.assign(n_inst, 1);
    c->fraw.resize(n_inst);
    c->promoted_at.assign(n_inst, -1);
    if (const char* g = std::getenv("LBE_GRAPH")) c->use_graph = std::atoi(g) != 0;
    if (const char* g = std::getenv("LBE_FP32_PROMOTE")) c->promote = std::atoi(g) != 0;
    // host tables of the instances, built by a small pool of host threads
    {
        std::vector<lbe_status> sts(n_inst, LBE_OK);
        std::vector<std::string> errs(n_inst);
        std::atomic<int> next(0);
        const int nth = std::max(1, std::min<int>(n_inst, (int)std::thread::hardware_concurrency()));
        auto work = [&]() {
            for (int k = next++; k < n_inst; k = next++) sts[k] = build_instance(p[k], &c->tabs[k], &errs[k]);
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < nth; t++) pool.emplace_back(work);
        work();
        for (auto& th : pool) th.join();
        for (int k = 0; k < n_inst; k++) {
            if (sts[k] != LBE_OK) {
                st = sts[k];
                delete c;
                return st;
            }
            c->maxnr = std::max(c->maxnr, c->tabs[k].nr);
            c->maxn0 = std::max(c->maxn0, c->tabs[k].prm.n_expand[0]);
            c->maxnv = std::max(c->maxnv, c->tabs[k].nv);
            c->maxng = std::max(c->maxng, c->tabs[k].n0 + c->tabs[k].n1 + c->tabs[k].n2);
            if (c->tabs[k].prm.precision == LBE_FP32_STORE) c->any_f32 = true;
        }
    }
    st = plan_groups(c);
    if (st != LBE_OK) {
        delete c;
        return st;
    }
    size_t off = align256(sizeof(DevInstance) * n_inst);
    c->dev_desc = (DevInstance*)c->ws;
    c->dev_items = (WorkItem*)(c->ws + off);
    off = align256(off + c->items_cap * sizeof(WorkItem));
    c->dev_status = (double*)(c->ws + off);
    off = align256(off + 4 * sizeof(double) * (size_t)n_inst);
    c->dev_rowoff = (int32_t*)(c->ws + off);
    off = align256(off + sizeof(int32_t) * (size_t)(n_inst + 1));
    c->dev_mask = (int32_t*)(c->ws + off);
    off = align256(off + sizeof(int32_t) * (size_t)n_inst);
    c->dev_vec = (double*)(c->ws + off);
    off = align256(off + 2 * sizeof(double) * (size_t)n_inst);
    c->dev_mass = (double*)(c->ws + off);
    off = align256(off + sizeof(double) * (size_t)n_inst);
    c->dev_glist = (int32_t*)(c->ws + off);
    off = align256(off + sizeof(int32_t) * (size_t)n_inst);
    c->rowoff.assign(n_inst + 1, 0);
    for (int k = 0; k < n_inst; k++) c->rowoff[k + 1] = c->rowoff[k] + c->tabs[k].nr;
    if (off > ws_bytes) {
        delete c;
        return LBE_ENOMEM;
    }
    hipError_t e = upload_plan(c, nullptr);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->dev_rowoff, c->rowoff.data(), c->rowoff.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           c->stream);
    for (int k = 0; k < n_inst && e == hipSuccess; k++) {
        const InstanceTables& t = c->tabs[k];
        const StageGroup& Gk = c->groups[c->group_of[k]];
        const int nsl = Gk.S;
        if ((size_t)nsl * Gk.img_sz > (size_t)t.n2 * stage_image_bound(t.n0, t.n1, t.n2, t.prm.geometry == LBE_SPH)) {
            delete c;
            return LBE_ENOMEM;
        }
        Layout L = make_layout(t, nsl, (size_t)nsl * Gk.img_sz, off);
        if (L.total > ws_bytes) {
            delete c;
            return LBE_ENOMEM;
        }
        off = L.total;
        DevInstance& d = c->host_desc[k];
        std::memset(&d, 0, sizeof(d));
        d.nr = t.nr;
        d.nv = t.nv;
        d.n0 = t.n0;
        d.n1 = t.n1;
        d.n2 = t.n2;
        d.geometry = t.prm.geometry;
        d.f32 = t.prm.precision == LBE_FP32_STORE;
        d.reduced = t.prm.reduced;
        d.N0 = t.ax[0].N;
        d.N1 = t.ax[1].N;
        d.N2 = t.ax[2].N;
        d.wband = t.wband;
        d.dt = t.dt;
        d.dr = t.dr;
        d.eta0 = t.prm.eta0;
        d.kn = t.prm.kn;
        d.chi0 = t.chi0;
        d.L = t.L;
        d.gin_l = t.gin_l;
        d.gin_r = t.gin_r;
        d.rcl = t.rcl;
        d.rcr = t.rcr;
        d.uw = t.prm.u_wall_inner;
        d.tratio = t.prm.t_wall_outer / t.prm.t_wall_inner;
        char* ws = c->ws;
        for (int b = 0; b < 3; b++) {
            d.f[b] = (double*)(ws + L.f[b]);
            c->fraw[k][b] = ws + L.fraw[b];
        }
        d.mom = (double*)(ws + L.mom);
        d.node = (double*)(ws + L.node);
        d.snap = (double*)(ws + L.snap);
        d.resid = (double*)(ws + L.resid);
        d.flags = (int32_t*)(ws + L.flags);
        d.nw = (double*)(ws + L.nw);
        d.scratch = (double*)(ws + L.scratch);
        d.rest = (const double*)(ws + L.rest);
        for (int b = 0; b < 4; b++) d.base[b] = d.f32 ? (double*)(ws + L.base[b]) : nullptr;
        d.p0 = (const double*)(ws + L.p0);
        d.p1 = (const double*)(ws + L.p1);
        d.p2 = (const double*)(ws + L.p2);
        d.K1 = (const double*)(ws + L.K1);
        d.K2a = (const double*)(ws + L.K2a);
        d.K2b = (const double*)(ws + L.K2b);
        d.w0 = (const double*)(ws + L.w0);
        d.w1 = (const double*)(ws + L.w1);
        d.w2 = (const double*)(ws + L.w2);
        d.poly0 = (const double*)(ws + L.poly0);
        d.poly1 = (const double*)(ws + L.poly1);
        d.poly2 = (const double*)(ws + L.poly2);
        d.qy0 = (const double*)(ws + L.qy0);
        d.qlam0 = (const double*)(ws + L.qlam0);
        d.qrec0 = (const double*)(ws + L.qrec0);
        d.pgx0 = (const double*)(ws + L.pgx0);
        d.pgw0 = (const double*)(ws + L.pgw0);
        d.M0 = (int32_t)t.ax[0].qy.size();
        d.qpw = t.ax[0].qpanel;
        d.nslices = nsl;
        d.geo = (const double*)(ws + L.geo);
        d.r = (const double*)(ws + L.r);
        d.wlo = (const int32_t*)(ws + L.wlo);
        d.wb = (const double*)(ws + L.wb);
        d.gwl = (const double*)(ws + L.gwl);
        d.gwr = (const double*)(ws + L.gwr);
        d.amf = t.amf.empty() ? nullptr : (const double*)(ws + L.amf);
        d.simg = (double*)(ws + L.simg);
        if (e == hipSuccess) e = put(ws, L.p0, t.ax[0].p, c->stream);
        if (e == hipSuccess) e = put(ws, L.p1, t.ax[1].p, c->stream);
        if (e == hipSuccess) e = put(ws, L.p2, t.ax[2].p, c->stream);
        if (e == hipSuccess) e = put(ws, L.K1, t.K1, c->stream);
        if (e == hipSuccess) e = put(ws, L.K2a, t.K2a, c->stream);
        if (e == hipSuccess) e = put(ws, L.K2b, t.K2b, c->stream);
        if (e == hipSuccess) e = put(ws, L.w0, t.ax[0].w, c->stream);
        if (e == hipSuccess) e = put(ws, L.w1, t.ax[1].w, c->stream);
        if (e == hipSuccess) e = put(ws, L.w2, t.ax[2].w, c->stream);
        if (e == hipSuccess) e = put(ws, L.poly0, t.ax[0].poly, c->stream);
        if (e == hipSuccess) e = put(ws, L.poly1, t.ax[1].poly, c->stream);
        if (e == hipSuccess) e = put(ws, L.poly2, t.ax[2].poly, c->stream);
        if (e == hipSuccess) e = put(ws, L.qy0, t.ax[0].qy, c->stream);
        if (e == hipSuccess) e = put(ws, L.qlam0, t.ax[0].qlam, c->stream);
        if (e == hipSuccess) e = put(ws, L.qrec0, t.ax[0].qrec, c->stream);
        if (e == hipSuccess) e = put(ws, L.pgx0, t.ax[0].gx, c->stream);
        if (e == hipSuccess) e = put(ws, L.pgw0, t.ax[0].gw, c->stream);
        if (e == hipSuccess) e = put(ws, L.geo, t.geo, c->stream);
        if (e == hipSuccess) e = put(ws, L.r, t.r, c->stream);
        if (e == hipSuccess) e = put(ws, L.wlo, t.wlo, c->stream);
        if (e == hipSuccess) e = put(ws, L.wb, t.wb, c->stream);
        if (e == hipSuccess) e = put(ws, L.gwl, t.gwl, c->stream);
        if (e == hipSuccess) e = put(ws, L.gwr, t.gwr, c->stream);
        if (e == hipSuccess && !t.amf.empty()) e = put(ws, L.amf, t.amf, c->stream);
        // rest start: n = 1, u = 0, T = 1 (its axis factors are kept for resets on the device)
        if (e == hipSuccess) {
            std::vector<double> g0(t.n0), g1(t.n1), g2(t.n2), f((size_t)t.nr * t.nv);
            equilibrium_axis(t.ax[0], 0.0, 1.0, g0.data());
            equilibrium_axis(t.ax[1], 0.0, 1.0, g1.data());
            equilibrium_axis(t.ax[2], 0.0, 1.0, g2.data());
            std::vector<double> rest(g0);
            rest.insert(rest.end(), g1.begin(), g1.end());
            rest.insert(rest.end(), g2.begin(), g2.end());
            e = hipMemcpy(ws + L.rest, rest.data(), rest.size() * sizeof(double), hipMemcpyHostToDevice);
            for (int v = 0; v < t.nv; v++) {
                const int i0 = v % t.n0, i1 = (v / t.n0) % t.n1, i2 = v / (t.n0 * t.n1);
                const double val = g0[i0] * g1[i1] * g2[i2];
                for (int i = 0; i < t.nr; i++) f[(size_t)i * t.nv + v] = val;
            }
            if (d.f32) {
                // FP32 storage: the rest start is its own base (n = 1), deviations zero
                std::vector<double> b0;
                for (int i = 0; i < t.nr; i++) b0.insert(b0.end(), rest.begin(), rest.end());
                if (e == hipSuccess)
                    e = hipMemcpy(d.base[0], b0.data(), b0.size() * sizeof(double), hipMemcpyHostToDevice);
                if (e == hipSuccess) e = hipMemset(d.f[0], 0, (size_t)t.nr * t.nv * sizeof(float));
            } else if (e == hipSuccess) {
                e = hipMemcpy(d.f[0], f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice);
            }
        }
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->dev_desc, c->host_desc.data(), sizeof(DevInstance) * n_inst, hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess) e = set_stage_smem_limit();
    // constant LDS images of the stage kernel (tables and tile descriptors per slice); the tile
    // height never moves them, so they are built once
    for (size_t q = 0; q < c->groups.size() && e == hipSuccess; q++)
        if (c->gl_cnt[q] > 0)
            e = launch_stage_image(c->dev_desc, c->dev_glist + c->gl_off[q], c->gl_cnt[q], c->groups[q], c->stream);

    if (e != hipSuccess) {
        st = dev_err(c, e, "lbe_init upload");
        delete c;
        return st;
    }
    st = upload_flags(c);
    if (st == LBE_OK) st = dev_err(c, launch_moments(c->dev_desc, n_inst, c->maxnr, 0, 0, 0, -1, c->stream), "moments");
    if (st == LBE_OK) st = dev_err(c, launch_mass(c->dev_desc, n_inst, -1, c->dev_mass, c->stream), "mass");
    if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "lbe_init sync");
    if (st != LBE_OK) {
        delete c;
        return st;
    }
    *out = c;
    return LBE_OK;
}

lbe_status lbe_init_static(const lbe_params* p, int32_t n_inst, void* hip_stream, lbe_ctx** out)
{
    if (!p || n_inst < 1 || !out) return LBE_EINVAL;
    *out = nullptr;
    size_t need = 0;
    lbe_status st = lbe_query(p, n_inst, &need, nullptr);
    if (st != LBE_OK) return st;
    if (need > kStaticWsBytes) return LBE_ENOMEM;  // beyond the static workspace's fixed size
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kStaticMaxDevices) return LBE_EDEVICE;
    std::lock_guard<std::mutex> lock(static_ws_mu);
    if (static_ws_busy[dev]) return LBE_ESTATE;  // one static-workspace context per device at a time
    if (!static_ws_addr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBE_EDEVICE;
        static_ws_addr[dev] = ptr;
    }
    lbe_ctx* c = nullptr;
    st = lbe_init(p, n_inst, static_ws_addr[dev], kStaticWsBytes, hip_stream, &c);
    if (st != LBE_OK) return st;
    c->static_dev = dev;
    static_ws_busy[dev] = true;
    *out = c;
    return LBE_OK;
}

lbe_status lbe_step(lbe_ctx* c, int64_t nsteps)
{
    if (!c || nsteps < 0) return LBE_EINVAL;
    if (c->nan_latched) return LBE_ENAN;
    for (int64_t s = 0; s < nsteps; s++) {
        if (c->any_f32 && ++c->since_fix >= kMassFixEvery) {
            lbe_status st = dev_err(c, launch_mass_fix(c->dev_desc, c->ninst, c->maxnr, c->dev_mass, c->stream),
                                    "mass fix");
            if (st != LBE_OK) return st;
            c->since_fix = 0;
        }
        lbe_status st = enqueue_step(c);
        if (st != LBE_OK) return st;
    }
    for (int k = 0; k < c->ninst; k++)
        if (c->active[k]) c->steps[k] += nsteps;
    return LBE_OK;
}

lbe_status lbe_sync(lbe_ctx* c)
{
    if (!c) return LBE_EINVAL;
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    return check_nan(c);
}

lbe_status lbe_moments(lbe_ctx* c, int32_t inst, double* host_out, int64_t cap)
{
    if (!c || inst < 0 || inst >= c->ninst || !host_out) return LBE_EINVAL;
    const DevInstance& d = c->host_desc[inst];
    if (cap < 9 * (int64_t)d.nr) return LBE_EINVAL;
    // refresh the node block from the moment sums of the state (one node-kernel pass on f[0])
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    std::vector<int32_t> saved = c->active;
    std::fill(c->active.begin(), c->active.end(), 0);
    c->active[inst] = 1;
    st = upload_flags(c);
    if (st == LBE_OK)
        st = dev_err(c, launch_node(c->dev_desc, nullptr, c->ninst, c->maxnr, c->maxn0, 0, 0, c->stream), "moments pass");
    std::vector<double> node((size_t)d.nr * kNodeStride);
    if (st == LBE_OK)
        st = dev_err(c, hipMemcpyAsync(node.data(), d.node, node.size() * sizeof(double), hipMemcpyDeviceToHost,
                                       c->stream),
                     "node read");
    if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    c->active = saved;
    lbe_status st2 = upload_flags(c);
    if (st != LBE_OK) return st;
    if (st2 != LBE_OK) return st2;
    const int fields[11] = {NF_N, NF_U0, NF_U1, NF_U2, NF_T, NF_Q0, NF_P01, NF_NBAR, NF_CHI, NF_PHI, NF_FR};
    const int nf = cap >= 11 * (int64_t)d.nr ? 11 : 9;
    for (int fi = 0; fi < nf; fi++)
        for (int i = 0; i < d.nr; i++) host_out[fi * d.nr + i] = node[(size_t)i * kNodeStride + fields[fi]];
    return check_nan(c);
}

lbe_status lbe_rhs(lbe_ctx* c, int32_t inst, double* host_out, int64_t cap)
{
    if (!c || inst < 0 || inst >= c->ninst || !host_out) return LBE_EINVAL;
    const DevInstance& d = c->host_desc[inst];
    if (cap < (int64_t)d.nr * d.nv) return LBE_EINVAL;
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    std::vector<int32_t> saved = c->active;
    std::fill(c->active.begin(), c->active.end(), 0);
    c->active[inst] = 1;
    st = upload_flags(c);
    if (st == LBE_OK)
        st = dev_err(c, run_stage(c, 0, 0, 0, 0, 0, 1, 0, 0, 1), "rhs");
    if (st == LBE_OK)
        st = dev_err(c, hipMemcpyAsync(host_out, d.scratch, (size_t)d.nr * d.nv * sizeof(double),
                                       hipMemcpyDeviceToHost, c->stream),
                     "rhs read");
    if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    c->active = saved;
    lbe_status st2 = upload_flags(c);
    return st != LBE_OK ? st : st2;
}

lbe_status lbe_run_to_steady(lbe_ctx* c, double tol, int64_t max_steps, int32_t check_every, int64_t* steps_out,
                             double* resid_out)
{
    if (!c || !(tol > 0) || max_steps < 1 || check_every < 1) return LBE_EINVAL;
    if (c->nan_latched) return LBE_ENAN;
    std::fill(c->active.begin(), c->active.end(), 1);
    lbe_status st = upload_flags(c);
    if (st != LBE_OK) return st;
    // per instance: residual (-1 until judged), steps, nan flag, active
    std::vector<double> stv(4 * (size_t)c->ninst, 0.0);
    for (int k = 0; k < c->ninst; k++) {
        stv[4 * k] = -1.0;
        stv[4 * k + 3] = 1.0;
    }
    st = dev_err(c, hipMemcpyAsync(c->dev_status, stv.data(), stv.size() * sizeof(double), hipMemcpyHostToDevice,
                                   c->stream),
                 "status upload");
    if (st != LBE_OK) return st;
    int64_t taken = 0;
    bool all = false;
    int planned = c->ninst;  // instances in the launch plan
    std::vector<int32_t> act(c->ninst, 1);
    // plans with shorter tiles while few work items remain: a tile's nodes are processed in
    // sequence, so with fewer items than two per compute unit the tile height sets the latency
    std::vector<StageGroup> saved = c->groups;
    bool replanned = false;
    auto adapt_tiles = [&](const std::vector<int32_t>* only) {
        for (size_t q = 0; q < c->groups.size(); q++) {
            auto items_at = [&](int nt) {
                long n = 0;
                for (int k = 0; k < c->ninst; k++)
                    if (c->group_of[k] == (int)q && (!only || (*only)[k]))
                        n += (long)((c->tabs[k].nr + nt - 1) / nt) * saved[q].S;
                return n;
            };
            int nt = saved[q].NT;
            while (nt > kMinTileNodes && items_at(nt) < 512) nt /= 2;
            StageGroup G = saved[q];
            if (nt != saved[q].NT && layout_group(&G, nt) && G.NT == nt)
                c->groups[q] = G;
            else
                c->groups[q] = saved[q];
        }
        replanned = true;
        return upload_plan(c, only);
    };
    st = dev_err(c, adapt_tiles(nullptr), "plan");
    if (st != LBE_OK) return st;
    // FP32 storage leaves a residual floor (the rounding of the stored deviations); an instance has
    // stopped improving when the smallest residual of its last `win` check intervals (about 2000
    // steps) is not below 0.8 times the smallest of the `win` intervals before.  A launch group of
    // FP32-storage instances that all stopped improving above tol is switched to FP64 storage in
    // place and the solve continues (LBE_FP32_PROMOTE=0 in the environment turns this off).
    const int win = std::max(2, (int)((2000 + check_every - 1) / check_every));
    std::vector<std::vector<double>> hist(c->ninst);
    while (taken < max_steps && !all) {
        const int chunk = (int)std::min<int64_t>(check_every, max_steps - taken);
        st = enqueue_chunk(c, chunk, tol, chunk == check_every);
        if (st != LBE_OK) break;
        st = dev_err(c, hipMemcpyAsync(stv.data(), c->dev_status, stv.size() * sizeof(double),
                                       hipMemcpyDeviceToHost, c->stream),
                     "status read");
        if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
        if (st != LBE_OK) break;
        taken += chunk;
        all = true;
        int nact = 0;
        for (int k = 0; k < c->ninst; k++) {
            if (stv[4 * k + 2] != 0) {
                c->nan_latched = true;
                c->err = "non-finite state or non-positive density/temperature in instance " + std::to_string(k);
                st = LBE_ENAN;
            }
            act[k] = stv[4 * k + 3] != 0;
            nact += act[k];
            if (act[k]) all = false;
        }
        if (st != LBE_OK) break;
        bool promoted = false;
        if (c->promote && c->any_f32 && chunk == check_every) {
            std::vector<int> stalled(c->groups.size(), 1), members(c->groups.size(), 0);
            for (int k = 0; k < c->ninst; k++) {
                if (!c->host_desc[k].f32 || !act[k]) continue;
                hist[k].push_back(stv[4 * k]);
                const int g = c->group_of[k];
                members[g]++;
                const size_t h = hist[k].size();
                bool flat = h >= (size_t)(2 * win);
                if (flat) {
                    const double recent = *std::min_element(hist[k].end() - win, hist[k].end());
                    const double before = *std::min_element(hist[k].end() - 2 * win, hist[k].end() - win);
                    flat = !(recent < 0.8 * before);
                }
                if (!flat) stalled[g] = 0;
            }
            for (size_t q = 0; q < c->groups.size() && st == LBE_OK; q++) {
                if (!c->groups[q].f32 || !members[q] || !stalled[q]) continue;
                st = promote_group(c, (int)q, taken, &saved);
                promoted = true;
            }
            if (st != LBE_OK) break;
        }
        // once half of the planned instances have converged, launch only the others
        if (nact > 0 && (2 * nact <= planned || promoted)) {
            st = dev_err(c, adapt_tiles(&act), "plan");
            if (st != LBE_OK) break;
            planned = nact;
        }
    }
    if (replanned) {
        c->groups = saved;
        lbe_status stp = dev_err(c, upload_plan(c, nullptr), "plan");
        if (st == LBE_OK) st = stp;
    }
    if (st != LBE_OK) return st;
    std::fill(c->active.begin(), c->active.end(), 1);
    st = upload_flags(c);
    if (st != LBE_OK) return st;
    bool conv = true;
    for (int k = 0; k < c->ninst; k++) {
        const int64_t done = (int64_t)stv[4 * k + 1];
        const double r = stv[4 * k];
        c->steps[k] += done;
        if (steps_out) steps_out[k] = done;
        if (resid_out) resid_out[k] = r;
        if (!(r >= 0 && r <= tol)) conv = false;
    }
    return conv ? LBE_OK : LBE_ENOTCONV;
}

// ---- checkpoint / resume: the exact device state a step reads from one step to the next
namespace {
constexpr char kCkptMagic[8] = {'L', 'B', 'E', 'C', 'K', 'P', 'T', '1'};

// FNV-1a over the problem statements, field by field (the struct has padding).
uint64_t params_fingerprint(const lbe_ctx* c)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < n; i++) h = (h ^ b[i]) * 1099511628211ull;
    };
    for (const InstanceTables& t : c->tabs) {
        const lbe_params& q = t.prm;
        const double dv[8] = {q.r_inner, q.r_outer, q.u_wall_inner, q.t_wall_inner, q.t_wall_outer, q.eta0, q.kn, q.cfl};
        const int32_t iv[7] = {q.geometry, q.nr, q.q_radial, q.q_t1, q.q_t2, q.n_expand[0], q.n_expand[1]};
        mix(dv, sizeof(dv));
        mix(iv, sizeof(iv));
        mix(&q.n_expand[2], sizeof(int32_t));
        mix(&q.reduced, sizeof(int32_t));
        mix(&q.phi_a, sizeof(double));
    }
    return h;
}

struct CkptInst {
    int64_t steps, promoted_at;
    int32_t f32, nr, nv, nslices, ng, pad;
};

size_t inst_state_bytes(const DevInstance& d)
{
    const size_t E = d.f32 ? sizeof(float) : sizeof(double);
    const size_t ng = (size_t)(d.n0 + d.n1 + d.n2);
    return (size_t)d.nr * d.nv * E + (d.f32 ? (size_t)d.nr * ng * sizeof(double) : 0) +
           (size_t)d.nr * d.nslices * kMomStride * sizeof(double) + sizeof(double);
}

size_t checkpoint_bytes(const lbe_ctx* c)
{
    size_t b = sizeof(kCkptMagic) + sizeof(uint64_t) + 3 * sizeof(int64_t) + c->groups.size() * sizeof(int32_t);
    for (int k = 0; k < c->ninst; k++) b += sizeof(CkptInst) + inst_state_bytes(c->host_desc[k]);
    return b;
}
}  // namespace

lbe_status lbe_checkpoint_size(lbe_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return LBE_EINVAL;
    *bytes = checkpoint_bytes(c);
    return LBE_OK;
}

lbe_status lbe_checkpoint_save(lbe_ctx* c, void* host_buf, size_t cap)
{
    if (!c || !host_buf) return LBE_EINVAL;
    if (cap < checkpoint_bytes(c)) return LBE_EINVAL;
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    char* o = (char*)host_buf;
    auto put_h = [&](const void* p, size_t n) {
        std::memcpy(o, p, n);
        o += n;
    };
    const uint64_t fp = params_fingerprint(c);
    const int64_t hdr[3] = {c->ninst, (int64_t)c->groups.size(), c->since_fix};
    put_h(kCkptMagic, sizeof(kCkptMagic));
    put_h(&fp, sizeof(fp));
    put_h(hdr, sizeof(hdr));
    for (const StageGroup& G : c->groups) put_h(&G.NT, sizeof(int32_t));
    std::vector<double> mass(c->ninst);
    st = dev_err(c, hipMemcpy(mass.data(), c->dev_mass, mass.size() * sizeof(double), hipMemcpyDeviceToHost), "mass");
    for (int k = 0; k < c->ninst && st == LBE_OK; k++) {
        const DevInstance& d = c->host_desc[k];
        const CkptInst ci = {c->steps[k], c->promoted_at[k], d.f32, d.nr, d.nv, d.nslices, d.n0 + d.n1 + d.n2, 0};
        put_h(&ci, sizeof(ci));
        const size_t fb = (size_t)d.nr * d.nv * (d.f32 ? sizeof(float) : sizeof(double));
        st = dev_err(c, hipMemcpy(o, d.f[0], fb, hipMemcpyDeviceToHost), "state");
        o += fb;
        if (st == LBE_OK && d.f32) {
            const size_t bb = (size_t)d.nr * ci.ng * sizeof(double);
            st = dev_err(c, hipMemcpy(o, d.base[0], bb, hipMemcpyDeviceToHost), "base table");
            o += bb;
        }
        const size_t mb = (size_t)d.nr * d.nslices * kMomStride * sizeof(double);
        if (st == LBE_OK) st = dev_err(c, hipMemcpy(o, d.mom, mb, hipMemcpyDeviceToHost), "moment sums");
        o += mb;
        put_h(&mass[k], sizeof(double));
    }
    if (st != LBE_OK) return st;
    return check_nan(c);
}

lbe_status lbe_checkpoint_load(lbe_ctx* c, const void* host_buf, size_t len)
{
    if (!c || !host_buf) return LBE_EINVAL;
    const char* o = (const char*)host_buf;
    const char* end = o + len;
    auto get_h = [&](void* p, size_t n) {
        if (o + n > end) return false;
        std::memcpy(p, o, n);
        o += n;
        return true;
    };
    char magic[8];
    uint64_t fp = 0;
    int64_t hdr[3];
    if (!get_h(magic, 8) || std::memcmp(magic, kCkptMagic, 8) != 0 || !get_h(&fp, sizeof(fp)) ||
        !get_h(hdr, sizeof(hdr))) {
        c->err = "not a checkpoint of this library";
        return LBE_EINVAL;
    }
    if (fp != params_fingerprint(c) || hdr[0] != c->ninst || hdr[1] != (int64_t)c->groups.size()) {
        c->err = "checkpoint of different problem statements";
        return LBE_EINVAL;
    }
    std::vector<int32_t> nts(c->groups.size());
    if (!get_h(nts.data(), nts.size() * sizeof(int32_t))) return LBE_EINVAL;
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    // the instances' storage as saved (instances switched to FP64 storage are switched here too)
    {
        const char* scan = o;
        std::vector<int32_t> f32s(c->ninst);
        for (int k = 0; k < c->ninst; k++) {
            CkptInst ci;
            if (scan + sizeof(ci) > end) return LBE_EINVAL;
            std::memcpy(&ci, scan, sizeof(ci));
            const DevInstance& d = c->host_desc[k];
            if (ci.nr != d.nr || ci.nv != d.nv || ci.nslices != d.nslices) {
                c->err = "checkpoint of a different launch plan";
                return LBE_EINVAL;
            }
            f32s[k] = ci.f32;
            scan += sizeof(ci) + (size_t)ci.nr * ci.nv * (ci.f32 ? 4 : 8) + (ci.f32 ? (size_t)ci.nr * ci.ng * 8 : 0) +
                    (size_t)ci.nr * ci.nslices * kMomStride * 8 + 8;
        }
        for (size_t q = 0; q < c->groups.size() && st == LBE_OK; q++) {
            if (!c->groups[q].f32) continue;
            bool promote = false;
            for (int k = 0; k < c->ninst; k++)
                if (c->group_of[k] == (int)q && !f32s[k]) promote = true;
            if (promote) st = promote_group(c, (int)q, 0, nullptr);
        }
        if (st != LBE_OK) return st;
    }
    for (size_t q = 0; q < c->groups.size(); q++) {
        StageGroup G = c->groups[q];
        if (!layout_group(&G, nts[q]) || G.NT != nts[q]) {
            c->err = "checkpoint tile height does not fit";
            return LBE_EINVAL;
        }
        c->groups[q] = G;
    }
    std::vector<double> mass(c->ninst);
    for (int k = 0; k < c->ninst && st == LBE_OK; k++) {
        const DevInstance& d = c->host_desc[k];
        CkptInst ci;
        if (!get_h(&ci, sizeof(ci)) || ci.f32 != d.f32) return LBE_EINVAL;
        const size_t fb = (size_t)d.nr * d.nv * (d.f32 ? sizeof(float) : sizeof(double));
        if (o + fb > end) return LBE_EINVAL;
        st = dev_err(c, hipMemcpy(d.f[0], o, fb, hipMemcpyHostToDevice), "state");
        o += fb;
        if (st == LBE_OK && d.f32) {
            const size_t bb = (size_t)d.nr * ci.ng * sizeof(double);
            if (o + bb > end) return LBE_EINVAL;
            st = dev_err(c, hipMemcpy(d.base[0], o, bb, hipMemcpyHostToDevice), "base table");
            o += bb;
        }
        const size_t mb = (size_t)d.nr * d.nslices * kMomStride * sizeof(double);
        if (o + mb + sizeof(double) > end) return LBE_EINVAL;
        if (st == LBE_OK) st = dev_err(c, hipMemcpy(d.mom, o, mb, hipMemcpyHostToDevice), "moment sums");
        o += mb;
        get_h(&mass[k], sizeof(double));
        c->steps[k] = ci.steps;
        c->promoted_at[k] = ci.promoted_at;
    }
    if (st == LBE_OK)
        st = dev_err(c, hipMemcpy(c->dev_mass, mass.data(), mass.size() * sizeof(double), hipMemcpyHostToDevice), "mass");
    if (st != LBE_OK) return st;
    c->since_fix = hdr[2];
    c->nan_latched = false;
    std::fill(c->active.begin(), c->active.end(), 1);
    st = dev_err(c, upload_plan(c, nullptr), "plan");
    if (st == LBE_OK) st = upload_flags(c);
    return st;
}

lbe_status lbe_get_state(lbe_ctx* c, int32_t inst, double* host_f, int64_t cap)
{
    if (!c || inst < 0 || inst >= c->ninst || !host_f) return LBE_EINVAL;
    const DevInstance& d = c->host_desc[inst];
    if (cap < (int64_t)d.nr * d.nv) return LBE_EINVAL;
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    const double* from = d.f[0];
    if (d.f32) {
        // FP32 storage: deviations plus their base, in FP64, through the scratch
        st = dev_err(c, launch_expand(c->dev_desc, inst, d.nr, c->stream), "expand");
        if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
        if (st != LBE_OK) return st;
        from = d.scratch;
    }
    return dev_err(c, hipMemcpy(host_f, from, (size_t)d.nr * d.nv * sizeof(double), hipMemcpyDeviceToHost),
                   "state read");
}

lbe_status lbe_set_state(lbe_ctx* c, int32_t inst, const double* host_f, int64_t len)
{
    if (!c || inst < 0 || inst >= c->ninst || !host_f) return LBE_EINVAL;
    const DevInstance& d = c->host_desc[inst];
    if (len != (int64_t)d.nr * d.nv) return LBE_EINVAL;
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    st = dev_err(c, hipMemcpy(d.f32 ? d.scratch : d.f[0], host_f, (size_t)len * sizeof(double), hipMemcpyHostToDevice),
                 "state write");
    if (st != LBE_OK) return st;
    c->nan_latched = false;
    if (!d.f32) {
        st = upload_flags(c);
        if (st == LBE_OK)
            st = dev_err(c, launch_moments(c->dev_desc, c->ninst, c->maxnr, 0, 0, 0, inst, c->stream), "moments");
        if (st != LBE_OK) return st;
        return dev_err(c, hipStreamSynchronize(c->stream), "sync");
    }
    // FP32 storage: moments of the FP64 state, its node coefficients and equilibrium projections,
    // then the base table and the deviations, and the moment sums of the stored state
    std::fill(c->active.begin(), c->active.end(), 0);
    c->active[inst] = 1;
    st = upload_flags(c);
    if (st == LBE_OK)
        st = dev_err(c, launch_moments(c->dev_desc, c->ninst, c->maxnr, 0, 0, 1, inst, c->stream), "moments");
    if (st == LBE_OK) st = dev_err(c, launch_node(c->dev_desc, nullptr, c->ninst, c->maxnr, c->maxn0, 0, 0, c->stream), "node");
    if (st == LBE_OK) st = dev_err(c, launch_rebase(c->dev_desc, inst, d.nr, c->stream), "rebase");
    if (st == LBE_OK)
        st = dev_err(c, launch_moments(c->dev_desc, c->ninst, c->maxnr, 0, 0, 0, inst, c->stream), "moments");
    // the state's own mass becomes the mass kept from now on
    if (st == LBE_OK) st = dev_err(c, launch_mass(c->dev_desc, c->ninst, inst, c->dev_mass, c->stream), "mass");
    if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    std::fill(c->active.begin(), c->active.end(), 1);
    lbe_status st2 = upload_flags(c);
    if (st != LBE_OK) return st;
    if (st2 != LBE_OK) return st2;
    return check_nan(c);
}

lbe_status lbe_info(lbe_ctx* c, int32_t inst, double* out, int64_t cap)
{
    if (!c || inst < 0 || inst >= c->ninst || !out || cap < 17) return LBE_EINVAL;
    const InstanceTables& t = c->tabs[inst];
    const double v[19] = {(double)t.nr, (double)t.nv, (double)t.n0, (double)t.n1, (double)t.n2, t.chi0, t.C, t.L,
                          t.sigma, t.rcl, t.rcr, t.dr, t.dt, (double)c->steps[inst], (double)t.ax[0].N,
                          (double)t.ax[1].N, (double)t.ax[2].N, (double)c->host_desc[inst].f32,
                          (double)c->promoted_at[inst]};
    std::memcpy(out, v, sizeof(double) * (cap >= 19 ? 19 : 17));
    return LBE_OK;
}

lbe_status lbe_tables(const lbe_params* p, int32_t which, const double* extra, double* out, int64_t cap,
                      int64_t* len_out)
{
    if (!p) return LBE_EINVAL;
    if (which == 9) {
        if (!extra) return LBE_EINVAL;
        if (len_out) *len_out = 1;
        if (cap < 1 || !out) return LBE_EINVAL;
        out[0] = p->geometry == LBE_CYL   ? ball_in_cylinder(extra[0], extra[1], extra[2])
                 : p->geometry == LBE_SPH ? ball_in_sphere(extra[0], extra[1], extra[2])
                                          : ball_below_plane(extra[0], extra[1], extra[2]);
        return LBE_OK;
    }
    if (which == 13) {
        lbe_params q;
        if (!extra || validate_params(*p, &q, nullptr) != LBE_OK) return LBE_EINVAL;
        if (len_out) *len_out = 1;
        if (cap < 1 || !out) return LBE_EINVAL;
        const double C = 1 / (6 * std::sqrt(2.0) * q.eta0 * chi_cs(q.eta0) * q.kn);
        const double sigma = (q.r_outer - q.r_inner) / C;  // as build_instance
        out[0] = mf_potential(q.geometry, sigma, q.phi_a, extra[1], extra[0]);
        return LBE_OK;
    }
    InstanceTables t;
    std::string err;
    lbe_status st = build_instance(*p, &t, &err);
    if (st != LBE_OK) return st;
    std::vector<double> v;
    switch (which) {
        case 0:
        case 1:
        case 2:
            v = t.ax[which].p;
            v.insert(v.end(), t.ax[which].w.begin(), t.ax[which].w.end());
            break;
        case 3: v = t.K1; break;
        case 4: v = t.K2a; break;
        case 5: v = t.K2b; break;
        case 6:
            v.assign((size_t)t.nr * t.nr, 0.0);
            for (int i = 0; i < t.nr; i++)
                for (int k = 0; k < t.wband; k++) {
                    const int j = t.wlo[i] + k;
                    if (j < t.nr) v[(size_t)i * t.nr + j] = t.wb[(size_t)i * t.wband + k];
                }
            break;
        case 7:
            v = t.gwl;
            v.insert(v.end(), t.gwr.begin(), t.gwr.end());
            break;
        case 8: {
            if (!extra) return LBE_EINVAL;
            v.assign(t.n0 + t.n1 + t.n2, 0.0);
            equilibrium_axis(t.ax[0], extra[0], extra[1], v.data());
            equilibrium_axis(t.ax[1], extra[0], extra[1], v.data() + t.n0);
            equilibrium_axis(t.ax[2], extra[0], extra[1], v.data() + t.n0 + t.n1);
            break;
        }
        case 10: v = t.K2r; break;
        case 11:
            v = t.ax[0].gx;
            v.insert(v.end(), t.ax[0].gw.begin(), t.ax[0].gw.end());
            break;
        case 12:
            v = t.amf;
            if (v.empty()) v.assign((size_t)t.nr * t.nr, 0.0);
            break;
        default: return LBE_EINVAL;
    }
    if (len_out) *len_out = (int64_t)v.size();
    if (!out || cap < (int64_t)v.size()) return LBE_EINVAL;
    std::memcpy(out, v.data(), v.size() * sizeof(double));
    return LBE_OK;
}

lbe_status lbe_features(lbe_ctx* c, float* dev_x, int64_t cap_rows, int64_t* rows_out)
{
    if (!c) return LBE_EINVAL;
    const int rows = c->rowoff[c->ninst];
    if (rows_out) *rows_out = rows;
    if (!dev_x || cap_rows < rows) return LBE_EINVAL;
    lbe_status st = dev_err(c, launch_warm_profile_net(c->dev_desc, c->dev_rowoff, c->ninst, 0, rows, dev_x, nullptr,
                                                       nullptr, nullptr, nullptr, 1, c->stream),
                            "features");
    if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    return st;
}

lbe_status lbe_targets(lbe_ctx* c, float* dev_t, int64_t cap_rows)
{
    if (!c || !dev_t) return LBE_EINVAL;
    const int rows = c->rowoff[c->ninst];
    if (cap_rows < rows) return LBE_EINVAL;
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    std::vector<int32_t> saved = c->active;
    std::fill(c->active.begin(), c->active.end(), 1);
    st = upload_flags(c);
    if (st == LBE_OK) st = dev_err(c, launch_node(c->dev_desc, nullptr, c->ninst, c->maxnr, c->maxn0, 0, 0, c->stream), "node pass");
    std::vector<float> out((size_t)rows * 5);
    const int fields[5] = {NF_N, NF_U1, NF_T, NF_Q0, NF_P01};
    for (int k = 0; k < c->ninst && st == LBE_OK; k++) {
        const DevInstance& d = c->host_desc[k];
        std::vector<double> node((size_t)d.nr * kNodeStride);
        st = dev_err(c, hipMemcpyAsync(node.data(), d.node, node.size() * sizeof(double), hipMemcpyDeviceToHost,
                                       c->stream),
                     "node read");
        if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
        for (int i = 0; i < d.nr && st == LBE_OK; i++)
            for (int q = 0; q < 5; q++)
                out[((size_t)c->rowoff[k] + i) * 5 + q] = (float)node[(size_t)i * kNodeStride + fields[q]];
    }
    if (st == LBE_OK)
        st = dev_err(c, hipMemcpyAsync(dev_t, out.data(), out.size() * sizeof(float), hipMemcpyHostToDevice, c->stream),
                     "target upload");
    if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    c->active = saved;
    lbe_status st2 = upload_flags(c);
    if (st != LBE_OK) return st;
    if (st2 != LBE_OK) return st2;
    return check_nan(c);
}

namespace {

lbe_status upload_mask(lbe_ctx* c, const std::vector<int32_t>& mask)
{
    return dev_err(c, hipMemcpyAsync(c->dev_mask, mask.data(), mask.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                     c->stream),
                   "mask upload");
}

// Grad-13 state of the masked instances from the profiles in their node blocks, then the mass
// renormalisation and the moment sums of the new state.  FP32-storage instances get the FP64
// state in their scratch first; its mass becomes the mass they keep, and it is then stored as
// deviations from the discrete equilibrium of its own moments (as lbe_set_state does).
hipError_t build_warm_state(lbe_ctx* c)
{
    hipError_t e = launch_proj(c->dev_desc, c->ninst, c->maxnr, c->stream);
    if (e == hipSuccess) e = launch_grad13(c->dev_desc, c->ninst, c->maxnr, c->dev_mask, c->stream);
    if (e == hipSuccess) e = launch_moments(c->dev_desc, c->ninst, c->maxnr, 0, 0, 2, -1, c->stream);
    if (e == hipSuccess) e = launch_renorm(c->dev_desc, c->ninst, c->dev_mask, c->stream);
    if (e == hipSuccess) e = launch_moments(c->dev_desc, c->ninst, c->maxnr, 0, 0, 2, -1, c->stream);
    if (c->any_f32) {
        if (e == hipSuccess) e = launch_mass(c->dev_desc, c->ninst, -2, c->dev_mass, c->stream, c->dev_mask);
        if (e == hipSuccess) e = launch_node(c->dev_desc, nullptr, c->ninst, c->maxnr, c->maxn0, 0, 0, c->stream);
        if (e == hipSuccess) e = launch_rebase_masked(c->dev_desc, c->ninst, c->maxnr, c->dev_mask, c->stream);
        if (e == hipSuccess) e = launch_moments(c->dev_desc, c->ninst, c->maxnr, 0, 0, 0, -1, c->stream);
    }
    return e;
}

// Network prediction of every node of the masked instances into their node blocks, in chunks of
// the network's row capacity, then their warm state.
hipError_t predict_warm_state(lbe_ctx* c, lbe_mlp* m)
{
    const int rows = c->rowoff[c->ninst], R = mlp_max_rows(m);
    double mean[5], scale[5];
    mlp_scaling(m, mean, scale);
    hipError_t e = hipSuccess;
    for (int r0 = 0; r0 < rows && e == hipSuccess; r0 += R) {
        const int n = std::min(R, rows - r0);
        e = launch_warm_profile_net(c->dev_desc, c->dev_rowoff, c->ninst, r0, n, mlp_input(m), nullptr, nullptr,
                                    nullptr, nullptr, 1, c->stream);
        if (e == hipSuccess) e = mlp_forward_rows(m, mlp_input(m), n, c->stream);
        if (e == hipSuccess)
            e = launch_warm_profile_net(c->dev_desc, c->dev_rowoff, c->ninst, r0, n, nullptr, mlp_output(m), mean,
                                        scale, c->dev_mask, 0, c->stream);
    }
    if (e == hipSuccess) e = build_warm_state(c);
    return e;
}

// One full step of every instance from its current state and the residual of that step.
lbe_status one_step_residual(lbe_ctx* c, std::vector<double>& out)
{
    lbe_status st = dev_err(c, launch_snapshot(c->dev_desc, c->ninst, c->stream), "snapshot");
    if (st == LBE_OK) st = enqueue_step(c);
    if (st == LBE_OK) st = dev_err(c, launch_residual(c->dev_desc, c->ninst, c->stream), "residual");
    if (st == LBE_OK) st = dev_err(c, launch_collect_resid(c->dev_desc, c->ninst, c->dev_vec, c->stream), "collect");
    out.assign(c->ninst, 0.0);
    if (st == LBE_OK)
        st = dev_err(c, hipMemcpyAsync(out.data(), c->dev_vec, out.size() * sizeof(double), hipMemcpyDeviceToHost,
                                       c->stream),
                     "residual read");
    if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    return st;
}

}  // namespace

lbe_status lbe_set_init_moments(lbe_ctx* c, int32_t inst, const double* host_in, int64_t len)
{
    if (!c || inst < 0 || inst >= c->ninst || !host_in) return LBE_EINVAL;
    const DevInstance& d = c->host_desc[inst];
    if (len != 5 * (int64_t)d.nr) return LBE_EINVAL;
    for (int i = 0; i < d.nr; i++)
        if (!(host_in[i] > 0) || !(host_in[2 * d.nr + i] > 0)) return LBE_EINVAL;
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    st = dev_err(c, hipMemcpy(d.scratch, host_in, (size_t)len * sizeof(double), hipMemcpyHostToDevice), "profile");
    if (st != LBE_OK) return st;
    // only this instance is active while its state is rebuilt
    std::fill(c->active.begin(), c->active.end(), 0);
    c->active[inst] = 1;
    st = upload_flags(c);
    std::vector<int32_t> mask(c->ninst, 0);
    mask[inst] = 1;
    if (st == LBE_OK) st = upload_mask(c, mask);
    if (st == LBE_OK) st = dev_err(c, launch_profile_from_host(c->dev_desc, inst, c->stream), "profile");
    if (st == LBE_OK) st = dev_err(c, build_warm_state(c), "warm state");
    if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    std::fill(c->active.begin(), c->active.end(), 1);
    lbe_status st2 = upload_flags(c);
    c->nan_latched = false;
    return st != LBE_OK ? st : st2;
}

lbe_status lbe_warm_start(lbe_ctx* c, lbe_mlp* m, int32_t judge, int32_t* kept, double* rho)
{
    if (!c || !m) return LBE_EINVAL;
    if (c->nan_latched) return LBE_ENAN;
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    std::fill(c->active.begin(), c->active.end(), 1);
    st = upload_flags(c);
    if (st != LBE_OK) return st;
    std::vector<int32_t> keep(c->ninst, 1);
    std::vector<double> r_rest(c->ninst, -1.0), r_warm(c->ninst, -1.0);
    if (judge) {
        // one step from the rest start and one from the predicted state
        st = dev_err(c, launch_rest(c->dev_desc, c->ninst, c->maxnr, nullptr, c->stream), "rest");
        if (st == LBE_OK) st = dev_err(c, launch_moments(c->dev_desc, c->ninst, c->maxnr, 0, 0, 0, -1, c->stream), "moments");
        if (st == LBE_OK) st = one_step_residual(c, r_rest);
        if (st == LBE_OK) st = upload_mask(c, keep);
        if (st == LBE_OK) st = dev_err(c, predict_warm_state(c, m), "prediction");
        if (st == LBE_OK) st = one_step_residual(c, r_warm);
        if (st != LBE_OK) return st;
        for (int k = 0; k < c->ninst; k++) keep[k] = (r_warm[k] < r_rest[k]) ? 1 : 0;  // NaN falls back
    }
    // final state: the prediction where kept, the rest start elsewhere
    st = upload_mask(c, keep);
    if (st == LBE_OK) st = dev_err(c, predict_warm_state(c, m), "prediction");
    if (st == LBE_OK) st = dev_err(c, launch_rest(c->dev_desc, c->ninst, c->maxnr, c->dev_mask, c->stream), "rest");
    if (st == LBE_OK) st = dev_err(c, launch_moments(c->dev_desc, c->ninst, c->maxnr, 0, 0, 0, -1, c->stream), "moments");
    if (st == LBE_OK && c->any_f32) {
        // FP32-storage instances back at the rest start keep the rest start's mass
        std::vector<int32_t> rest_mask(c->ninst);
        for (int k = 0; k < c->ninst; k++) rest_mask[k] = !keep[k];
        st = upload_mask(c, rest_mask);
        if (st == LBE_OK)
            st = dev_err(c, launch_mass(c->dev_desc, c->ninst, -2, c->dev_mass, c->stream, c->dev_mask), "mass");
    }
    if (st == LBE_OK) st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    // a judged state that went non-finite has been replaced: clear the device flags
    st = upload_flags(c);
    for (int k = 0; k < c->ninst; k++) {
        if (kept) kept[k] = keep[k];
        if (rho) {
            rho[2 * k] = r_warm[k];
            rho[2 * k + 1] = r_rest[k];
        }
    }
    return st;
}

lbe_status lbe_autotune(lbe_ctx* c, int32_t reps, double* out, int64_t cap, int32_t* ngroups_out)
{
    if (!c || reps < 1) return LBE_EINVAL;
    const int ng = (int)c->groups.size();
    if (ngroups_out) *ngroups_out = ng;
    if (out && cap < 4 * (int64_t)ng) return LBE_EINVAL;
    if (c->nan_latched) return LBE_ENAN;
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    // the stage launches below overwrite the moment sums and buffer 1; keep the sums
    std::vector<std::vector<double>> mom(c->ninst);
    for (int k = 0; k < c->ninst && st == LBE_OK; k++) {
        const DevInstance& d = c->host_desc[k];
        mom[k].resize((size_t)d.nr * d.nslices * kMomStride);
        st = dev_err(c, hipMemcpy(mom[k].data(), d.mom, mom[k].size() * sizeof(double), hipMemcpyDeviceToHost),
                     "moment save");
    }
    if (st != LBE_OK) return st;
    // coefficients of the state, so that the timed launches see the real data
    st = dev_err(c, launch_node(c->dev_desc, nullptr, c->ninst, c->maxnr, c->maxn0, 0, 0, c->stream), "node");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == LBE_OK) st = dev_err(c, hipEventCreate(&e0), "event");
    if (st == LBE_OK) st = dev_err(c, hipEventCreate(&e1), "event");
    auto time_group = [&](int q, double* ms) -> lbe_status {
        build_items(c);
        if (c->items.size() > c->items_cap) return LBE_EINVAL;
        hipError_t e = hipMemcpyAsync(c->dev_items, c->items.data(), c->items.size() * sizeof(WorkItem),
                                      hipMemcpyHostToDevice, c->stream);
        auto one = [&]() {
            return launch_stage(c->dev_desc, c->dev_items + c->item_off[q], c->item_cnt[q], c->groups[q], 0, 0, 1,
                                0.0, 1.0, 0, 0, 0, 1, c->stream);
        };
        if (e == hipSuccess) e = one();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; r++) e = one();
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        *ms = t / reps;
        return dev_err(c, e, "autotune launch");
    };
    for (int q = 0; q < ng && st == LBE_OK; q++) {
        const StageGroup base = c->groups[q];
        StageGroup best = base;
        double best_ms = 0, base_ms = 0;
        st = time_group(q, &base_ms);
        best_ms = base_ms;
        for (int cand : kTileCandidates) {
            if (st != LBE_OK || cand == base.NT) continue;
            StageGroup G = base;
            if (!layout_group(&G, cand) || G.NT != cand) continue;
            c->groups[q] = G;
            double ms = 0;
            st = time_group(q, &ms);
            if (st == LBE_OK && ms < best_ms) {
                best_ms = ms;
                best = G;
            }
        }
        c->groups[q] = best;
        if (out) {
            out[4 * q] = base.nv;
            out[4 * q + 1] = best.NT;
            out[4 * q + 2] = best_ms;
            out[4 * q + 3] = base_ms;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    build_items(c);
    lbe_status st2 = dev_err(c, hipMemcpyAsync(c->dev_items, c->items.data(), c->items.size() * sizeof(WorkItem),
                                               hipMemcpyHostToDevice, c->stream),
                             "items upload");
    for (int k = 0; k < c->ninst && st2 == LBE_OK; k++)
        st2 = dev_err(c, hipMemcpyAsync(c->host_desc[k].mom, mom[k].data(), mom[k].size() * sizeof(double),
                                        hipMemcpyHostToDevice, c->stream),
                      "moment restore");
    if (st2 == LBE_OK) st2 = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    drop_graphs(c);
    if (st != LBE_OK) return st;
    if (st2 != LBE_OK) return st2;
    return check_nan(c);
}

lbe_status lbe_timing(lbe_ctx* c, int32_t enable, double* out, int64_t cap)
{
    if (!c) return LBE_EINVAL;
    if (enable) {
        lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
        if (st != LBE_OK) return st;
        c->ev_used = 0;
        c->stage_ev.clear();
        c->node_ev.clear();
        c->timing = true;
        return LBE_OK;
    }
    c->timing = false;
    lbe_status st = dev_err(c, hipStreamSynchronize(c->stream), "sync");
    if (st != LBE_OK) return st;
    if (!out || cap < 4) return LBE_EINVAL;
    double sums[2] = {0, 0};
    for (int which = 0; which < 2; which++) {
        for (auto& pr : which == 0 ? c->stage_ev : c->node_ev) {
            float ms = 0;
            st = dev_err(c, hipEventElapsedTime(&ms, c->ev[pr.first], c->ev[pr.second]), "event time");
            if (st != LBE_OK) return st;
            sums[which] += ms;
        }
    }
    out[0] = sums[0];
    out[1] = (double)c->stage_ev.size();
    out[2] = sums[1];
    out[3] = (double)c->node_ev.size();
    return LBE_OK;
}

void lbe_free(lbe_ctx* c)
{
    if (!c) return;
    if (c->static_dev >= 0) {
        // the static workspace is free for the next lbe_init_static once this context's work is done
        (void)hipStreamSynchronize(c->stream);
        std::lock_guard<std::mutex> lock(static_ws_mu);
        static_ws_busy[c->static_dev] = false;
    }
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipStream_t t : c->gstreams) (void)hipStreamDestroy(t);
    for (hipEvent_t ev : c->gevents) (void)hipEventDestroy(ev);
    delete c;
}

}  // extern "C"
