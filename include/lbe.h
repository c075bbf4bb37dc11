/*
 * lbe.h - C ABI of the MI355X (gfx950) finite-difference lattice Boltzmann solver for the
 * simplified Enskog equation in vielbein (cylindrical / spherical) coordinates.
 *
 * Method: S. Busuioc, "Mesoscopic Lattice Boltzmann modeling of dense gas flows in
 * curvilinear geometries", arXiv:2403.15051.  One time step advances the discrete
 * distribution f(r_i, p_v) on Nr radial cells x a mixed half-range (radial momentum) /
 * full-range (transverse momenta) Gauss-Hermite velocity set with TVD Runge-Kutta 3:
 *   df/dt = - (flux-form radial advection, WENO-5)          Sec. II.B/II.C, Sec. III
 *           - (vielbein inertial terms, K-matrix contractions) Sec. III.B eqs. (force1/2)
 *           + J0 (Shakhov relaxation) + J1 (first-order Enskog) eqs. (j0), (j1)
 * with chi evaluated at the ball-averaged density (eqs. (chi_ret), (fm), Appendix A) and
 * diffuse-reflection walls at R_L + sigma/2 and R_R - sigma/2 (Sec. IV).
 *
 * Conventions
 *   - Units: m = k_B = T_0 = 1; lengths as given (the paper's sigma follows from eta0, Kn
 *     and L = r_outer - r_inner through Kn = 1/(6 sqrt2 eta0 chi(eta0) C), C = L/sigma);
 *     the number density is normalised to mean 1 over the computational domain.
 *   - Velocity index v = i0 + n0 * (i1 + n1 * i2), radial momentum innermost; n0 = 2 Q_r
 *     (positive nodes ascending, then their mirrors), n1 = Q_t1, n2 = Q_t2 (ascending roots
 *     of the probabilists' Hermite polynomials).  Cylinder: axes (R, phi, z); sphere:
 *     (r, theta, phi).
 *   - f of one instance is stored [nr][nv], velocity innermost (coalesced), in device
 *     memory inside the caller's workspace.
 *   - Ownership: the caller owns the device workspace (e.g. a torch uint8 tensor) and the
 *     HIP stream; the context owns only host-side tables and never frees the workspace.
 *     Host arrays passed in are copied; host arrays passed out are filled.
 *   - Errors: every call returns an lbe_status and never throws across the ABI; arguments
 *     are validated before any device work.  A non-finite f or n <= 0 detected on the
 *     device latches LBE_ENAN until lbe_set_state replaces the state.
 *   - Threading: one context per host thread; the library has no global mutable state.
 */
#ifndef LBE_H
#define LBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbe_ctx lbe_ctx; /* opaque */
typedef struct lbe_mlp lbe_mlp; /* opaque: network of the learned warm start */

typedef enum {
    LBE_OK = 0,
    LBE_EINVAL = -1,   /* invalid argument (nothing was done) */
    LBE_ENOMEM = -2,   /* workspace too small / host allocation failed */
    LBE_EDEVICE = -3,  /* HIP runtime error */
    LBE_ENOTCONV = -4, /* lbe_run_to_steady reached max_steps before tol */
    LBE_ENAN = -5,     /* non-finite state or n <= 0 detected (sticky) */
    LBE_ESTATE = -6    /* call not valid in the current state */
} lbe_status;

enum { LBE_CYL = 0, LBE_SPH = 1, LBE_PLANAR = 2 }; /* LBE_PLANAR: the Cartesian model equation of
                                                    * Sec. II between parallel walls at x = r_inner,
                                                    * r_outer (the R_L -> infinity limit)         */
enum { LBE_FP64 = 0, LBE_FP32_STORE = 1 }; /* storage of f (lbe_params.precision) */
enum { LBE_GEMM_BF16 = 0, LBE_GEMM_FP32 = 1 }; /* matrix-core operand type of the network */

/* Problem statement of one instance (Sec. IV set-up of the paper). */
typedef struct {
    int32_t geometry;     /* LBE_CYL (coaxial cylinders) | LBE_SPH (concentric spheres) |
                           * LBE_PLANAR (parallel plates; u_wall_inner moves along axis 1)    */
    double r_inner;       /* physical wall radii R_L < R_R; L = R_R - R_L                     */
    double r_outer;
    double u_wall_inner;  /* tangential (phi) speed of the inner cylinder; must be 0 for LBE_SPH */
    double t_wall_inner;  /* wall temperatures T_L, T_R (> 0)                                  */
    double t_wall_outer;
    double eta0;          /* mean packing fraction, 0 < eta0 < 0.5                            */
    double kn;            /* Knudsen number on L (> 0); requires C = L/sigma > 1             */
    int32_t nr;           /* radial cells, >= 8                                               */
    int32_t q_radial;     /* half-range order Q_r (2 Q_r radial momenta), 2..100 (tables);
                           * the stage kernel holds 2 Q_r x 2 Q_r in LDS: lbe_query rejects
                           * sets it cannot hold (with 8-point transverse orders: Q_r <= 48
                           * for reduced cylinders and plates, Q_r <= 30 for spheres)      */
    int32_t q_t1;         /* full-range orders of the transverse axes, 2..100                 */
    int32_t q_t2;
    int32_t n_expand[3];  /* equilibrium expansion orders N_a; 0 -> min(7, Q_a - 1); N_a < Q_a */
    double cfl;           /* dt = cfl * dr / max|p_r|  (> 0)                                  */
    int32_t precision;    /* LBE_FP64: f stored in FP64.  LBE_FP32_STORE: f stored as FP32
                           * deviations from the discrete equilibrium of per-node FP64 moments
                           * (all arithmetic, moment sums, node coefficients and the residual
                           * stay FP64).  The state buffers are laid out at FP64 size so that
                           * lbe_run_to_steady can switch such an instance to FP64 storage in
                           * place (the bytes streamed per step are those of FP32 storage).   */
    int32_t reduced;      /* cylinder or plates, 0 or 1: integrate p_z out (Sec. III, "Quadrature
                           * choice"): the state holds phi = int f dp_z and chi = int p_z^2 f dp_z
                           * on the (p_R, p_phi) quadrature, as the two planes i2 = 0, 1 of the
                           * velocity index (q_t2 and n_expand[2] are then ignored; n2 = 2).   */
    double phi_a;         /* attractive mean field, beyond the paper (its Sec. V names attractive
                           * forces as the next step): depth, in units of k_B T, of the Sutherland
                           * tail phi(t) = -phi_a (sigma/t)^6 for t > sigma.  The potential energy
                           * Phi(x) = n0 int n(x') phi(|x - x'|) d^3x' (n0 sigma^3 = 6 eta0 / pi,
                           * n = 0 outside the computational domain) gives the radial force
                           * F = -dPhi/dr (fourth-order stencil) and the term F df/dp_r of the
                           * Enskog-Vlasov equation.  0: none (the paper's model); finite.     */
} lbe_params;

/* Device workspace needed for n_inst instances described by p[0..n_inst-1] (device_bytes),
 * and the host memory the context will hold (host_bytes).  Host-only; no device work.
 * LBE_EINVAL for an invalid problem statement or a velocity set the stage kernel cannot hold
 * in its LDS at any slicing (lbe_tables still builds the host tables of such a set). */
lbe_status lbe_query(const lbe_params* p, int32_t n_inst, size_t* device_bytes, size_t* host_bytes);

/* Build the tables of every instance on the host (quadratures Sec. III, force matrices
 * Sec. III.B, averaged-density weights eq. (fm) / Appendix A, wall Maxwellians), upload
 * them into device_ws (>= lbe_query's device_bytes, 256-byte aligned) on hip_stream
 * (a hipStream_t, or NULL for the default stream), derive on the device the stage kernel's
 * per-slice table images (its constant LDS contents, written once), set every instance to the
 * rest start (n = 1, u = 0, T = 1) and compute its moments.  *out receives the context. */
lbe_status lbe_init(const lbe_params* p, int32_t n_inst, void* device_ws, size_t ws_bytes, void* hip_stream,
                    lbe_ctx** out);

/* lbe_init without a caller workspace, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the context
 * lives in a device array inside the library, 64 MiB, one copy per GPU, held by each GPU the
 * library runs on until the process ends.  The call itself allocates no device memory.  Same
 * arguments and effect as lbe_init otherwise.  Returns LBE_ENOMEM when lbe_query's device_bytes
 * exceed 64 MiB, LBE_ESTATE when a context made by this call on the current device has not been
 * freed yet (there is one such workspace per GPU: contexts on it would overwrite each other), and
 * LBE_EDEVICE when the array's address cannot be obtained.  lbe_free releases the workspace for
 * the next call after waiting for the context's stream.  The workspace keeps the previous
 * context's contents; lbe_init writes everything it later reads. */
lbe_status lbe_init_static(const lbe_params* p, int32_t n_inst, void* hip_stream, lbe_ctx** out);

/* Enqueue nsteps full TVD-RK3 steps of every instance on the context's stream (async).  The
 * launches of one step are captured once into a HIP graph and replayed (set LBE_GRAPH=0 in the
 * environment before lbe_init to launch them one by one); instances sharing a velocity set form a
 * launch group, and the groups' launch chains run on forked streams joined back into the
 * context's stream.  FP32-storage instances get their total mass restored every 10 steps (so a
 * window of any multiple of 10 steps holds the same share of these launches). */
lbe_status lbe_step(lbe_ctx* c, int64_t nsteps);

/* Wait for the stream; returns LBE_ENAN if the device flagged a non-finite state. */
lbe_status lbe_sync(lbe_ctx* c);

/* Macroscopic profiles of instance inst (synchronises): host_out[field * nr + i] for
 * fields n, u_r, u_t1, u_t2, T, q_r, P_{r t1}, nbar, chi (eqs. (macro_def), (fm), (chi)),
 * all FP64; cap >= 9 * nr doubles.  With cap >= 11 * nr also the mean-field potential Phi
 * and the radial force F of lbe_params.phi_a (zero without attraction). */
lbe_status lbe_moments(lbe_ctx* c, int32_t inst, double* host_out, int64_t cap);

/* Step every instance until its one-step residual
 *   rho = max_i max(|dn|, |du_r|, |du_t1|, |du_t2|, |dT|) / dt
 * (changes over one full step), evaluated after every check_every-th step, is <= tol, or
 * until max_steps.  Converged instances stop advancing.  steps_out[k], resid_out[k]
 * (n_inst each, may be NULL) receive per-instance steps taken and the last residual.
 * Returns LBE_OK when all converged, LBE_ENOTCONV otherwise.  One check interval (the steps,
 * the residual and the freeze test, all on the device) is one captured HIP graph; the host reads
 * one status array per interval.  Once half of the instances still advancing have converged, the
 * launches cover only the others, with shorter tiles while few work items remain; results agree
 * with lbe_step to rounding.  FP32-storage instances get their total mass restored at the start
 * of every interval.  The rounding of FP32 storage leaves a residual floor of order 1e-6 on hard
 * cases: when every still-advancing instance of an FP32-storage launch group has stopped
 * improving (the smallest residual of its last ~2000 steps is not below 0.8 times the smallest of
 * the ~2000 steps before), above tol, the group is switched to FP64 storage in place (state =
 * stored deviations plus base, in FP64) and continues to tol; the instances stay FP64-storage
 * afterwards (lbe_info reports it).  LBE_FP32_PROMOTE=0 in the environment before lbe_init turns
 * the switch off. */
lbe_status lbe_run_to_steady(lbe_ctx* c, double tol, int64_t max_steps, int32_t check_every, int64_t* steps_out,
                             double* resid_out);

/* Copy the FP64 state f[nr][nv] of instance inst out / in (synchronises).  Setting the
 * state clears a latched LBE_ENAN. */
lbe_status lbe_get_state(lbe_ctx* c, int32_t inst, double* host_f, int64_t cap);
lbe_status lbe_set_state(lbe_ctx* c, int32_t inst, const double* host_f, int64_t len);

/* Checkpoint / resume of the whole context: the exact device state one step reads from the
 * previous one (the stored state buffer in its stored precision, the FP32 base tables, the moment
 * sums, the FP32 mass targets), the step counters, each instance's storage precision and the
 * launch plan's tile heights.  lbe_checkpoint_size gives the bytes; lbe_checkpoint_save fills a
 * host buffer of at least that size (synchronises); lbe_checkpoint_load restores it into a
 * context made by lbe_init with the same problem statements (checked by a fingerprint, else
 * LBE_EINVAL), switching instances that were switched to FP64 storage, after which stepping
 * continues bitwise as the saved context would (the kernels use no atomics and fixed orders). */
lbe_status lbe_checkpoint_size(lbe_ctx* c, size_t* bytes);
lbe_status lbe_checkpoint_save(lbe_ctx* c, void* host_buf, size_t cap);
lbe_status lbe_checkpoint_load(lbe_ctx* c, const void* host_buf, size_t len);

/* Right-hand side L(f)[nr][nv] of the current state of instance inst (one evaluation of
 * every term of one RK stage, without updating the state); synchronises. */
lbe_status lbe_rhs(lbe_ctx* c, int32_t inst, double* host_out, int64_t cap);

/* Derived scalars of instance inst: [nr, nv, n0, n1, n2, chi0, C, L, sigma, rcl, rcr, dr,
 * dt, steps, N0, N1, N2]; cap >= 17.  With cap >= 19 also [fp32_storage_now, step at which the
 * instance was switched from FP32 to FP64 storage or -1]. */
lbe_status lbe_info(lbe_ctx* c, int32_t inst, double* out, int64_t cap);

/* Host-only access to the tables lbe_init builds for one instance (no device needed):
 *   which = 0: radial nodes+weights [2 n0]; 1: transverse-1 nodes+weights [2 n1];
 *           2: transverse-2 nodes+weights [2 n2]; 3: K1 (d/dp_r, n0 x n0);
 *           4: K2 of axis 1 (d(f p)/dp, n1 x n1); 5: K2 of axis 2 (n2 x n2);
 *           6: dense averaged-density weights W (nr x nr); 7: wall Maxwellians [2 nv];
 *           8: equilibrium factors at (u, T) = (extra[0], extra[1]) for the three axes
 *              [n0 + n1 + n2];
 *           9: cell volume of the ball of radius extra[0] centred at distance extra[2] from
 *              the axis/origin inside radius extra[1] (geometry of p) [1];
 *          10: d(f p)/dp matrix of the radial half-range axis (n0 x n0; not used by the
 *              reduced equations, exported for checks);
 *          11: nodes then weights of the 32-point half-range Gauss rule the equilibrium
 *              projection uses at moderate u / sqrt(T) [64];
 *          12: mean-field weights A (nr x nr): Phi_i = sum_j A_ij n_j (zeros when phi_a = 0);
 *          13: integral of the tail phi over the region of radius extra[0] (ball, infinite
 *              cylinder, or the half space x' < extra[0] for plates) seen from radius extra[1],
 *              for the geometry, sigma and phi_a of p [1].
 * len_out receives the number of doubles written (or needed when cap is too small). */
lbe_status lbe_tables(const lbe_params* p, int32_t which, const double* extra, double* out, int64_t cap,
                      int64_t* len_out);

/* Per-launch timing with HIP events on the context's stream.  enable = 1 starts recording
 * (synchronises first); enable = 0 stops, synchronises and fills out[0..3] = [total ms of the
 * stage-kernel launches, their count, total ms of the node-kernel launches, their count]
 * (cap >= 4).  Recording adds two events per launch and is meant for benchmarks. */
lbe_status lbe_timing(lbe_ctx* c, int32_t enable, double* out, int64_t cap);

/* Tile autotuner of the stage kernel (batched sweeps: instances with one velocity set share a
 * launch group).  For every launch group, times `reps` stage launches (after one warm-up) for
 * each candidate tile height (4, 8, 16, 32, 64 nodes per work item, where the LDS allows) and
 * keeps the fastest.  The state and its moment sums are kept.  The tile height changes only
 * the velocity shift of each tile's collision polynomial and moment sums, so results change at
 * rounding level.  out[4 q ..] = (velocities of group q, chosen nodes per tile, its ms per
 * launch, the ms of the tile height in use before the call); cap >= 4 * groups (out may be NULL);
 * *ngroups_out (may be NULL) receives the number of groups.  Synchronises. */
lbe_status lbe_autotune(lbe_ctx* c, int32_t reps, double* out, int64_t cap, int32_t* ngroups_out);

/* ---------------------------------------------------------------- learned warm start
 * Not part of the paper: a network maps (geometry flag, eta0, Kn, u_w, T2/T1, r_hat) to the
 * steady profile (n, u_t1, T, q_r, P_r,t1) at one node, trained on steady states this solver
 * computes.  The solver only starts from its prediction: the state is the Grad 13-moment
 * distribution on the collision term's discrete equilibrium, scaled to the rest start's mass,
 * and it is kept only where its one-step residual beats the rest start's.
 *
 * Network: 6 -> 256 -> 256 -> 256 -> 256 -> 5, SiLU hidden activations, linear output; 200 453
 * FP32 parameters packed per layer as W [fan_out][fan_in] (row-major) then b [fan_out].  Every
 * matrix product runs on the matrix cores with BF16 operands and FP32 accumulation
 * (LBE_GEMM_BF16), or FP32 operands (LBE_GEMM_FP32).  Outputs are standardised targets:
 * profile = mean + scale * output, per field.  Device pointers (dev_*) are float arrays in
 * device memory owned by the caller, row-major [rows][6] inputs and [rows][5] outputs/targets.
 */

/* Device workspace of a network that processes up to max_rows rows per pass; *n_params receives
 * the parameter count (both may be NULL). */
lbe_status lbe_mlp_query(int32_t max_rows, size_t* device_bytes, int64_t* n_params);
/* Network in device_ws (256-byte aligned, >= lbe_mlp_query's bytes; zeroed) on hip_stream. */
lbe_status lbe_mlp_init(int32_t max_rows, int32_t gemm_kind, void* device_ws, size_t ws_bytes, void* hip_stream,
                        lbe_mlp** out);
/* Uniform Glorot initialisation of the weights from a seeded host generator, zero biases; resets
 * the Adam state. */
lbe_status lbe_mlp_init_params(lbe_mlp* m, uint64_t seed);
/* Parameters in / out (host FP32, len / cap >= parameter count); setting resets the Adam state. */
lbe_status lbe_mlp_set_params(lbe_mlp* m, const float* host, int64_t len);
lbe_status lbe_mlp_get_params(lbe_mlp* m, float* host, int64_t cap);
/* Target standardisation (5 means, 5 positive scales, FP64). */
lbe_status lbe_mlp_set_scaling(lbe_mlp* m, const double* mean, const double* scale);
lbe_status lbe_mlp_get_scaling(lbe_mlp* m, double* mean, double* scale);
/* Outputs of rows <= max_rows input rows (async on the network's stream). */
lbe_status lbe_mlp_forward(lbe_mlp* m, const float* dev_x, int32_t rows, float* dev_y);
/* Mean-squared error of the outputs against standardised targets dev_t over rows x 5 and its
 * gradient with respect to every parameter (kept for lbe_mlp_adam_step; copied to host_grad when
 * it is not NULL, cap >= parameter count); synchronises. */
lbe_status lbe_mlp_loss_grad(lbe_mlp* m, const float* dev_x, const float* dev_t, int32_t rows, double* loss,
                             float* host_grad, int64_t cap);
/* Replace the kept gradient (host FP32, len = parameter count). */
lbe_status lbe_mlp_set_grads(lbe_mlp* m, const float* host, int64_t len);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the kept gradient. */
lbe_status lbe_mlp_adam_step(lbe_mlp* m, float lr);
/* Training on n rows (dev_x [n][6], dev_t [n][5] unstandardised profiles): sets the target
 * standardisation from the data (mean and standard deviation per field), then `epochs` passes of
 * minibatches of `batch` rows (<= max_rows) in a seeded affine permutation of the rows, each a
 * forward pass, the loss, the backward pass and an Adam step; the learning rate falls from lr to
 * lr / 10 on a cosine over the epochs.  host_loss[epoch] (may be NULL) receives each epoch's mean
 * loss.  Synchronises once per epoch. */
lbe_status lbe_mlp_train(lbe_mlp* m, const float* dev_x, const float* dev_t, int64_t n, int32_t epochs, int32_t batch,
                         float lr, uint64_t seed, double* host_loss);
const char* lbe_mlp_last_error(const lbe_mlp* m);
void lbe_mlp_free(lbe_mlp* m);

/* Network inputs of every node of every instance, rows instance-major (instance k's nodes start
 * at row sum_{j<k} nr_j): geometry flag, then (eta0 - 0.155) / s1, (log10 Kn + 0.5) / s2,
 * (u_w - 0.25) / s3, (T2/T1 - 1.5) / s4, (r_hat - 0.5) / s5 with s = (b - a) / sqrt(12) of the
 * ranges U(0.01, 0.3), U(-2, 1), U(0, 0.5), U(1, 2), U(0, 1); r_hat = (r_i - R_L - sigma/2) /
 * (L - sigma).  *rows_out (may be NULL) receives the row count; cap_rows >= it; synchronises. */
lbe_status lbe_features(lbe_ctx* c, float* dev_x, int64_t cap_rows, int64_t* rows_out);
/* Profiles (n, u_t1, T, q_r, P_r,t1) of the current states, rows as in lbe_features (training
 * targets); synchronises. */
lbe_status lbe_targets(lbe_ctx* c, float* dev_t, int64_t cap_rows);
/* Start instance inst from a given profile host_in[field * nr + i], fields n, u_t1, T, q_r,
 * P_r,t1 (n, T > 0; u_r = u_t2 = 0): Grad-13 state, scaled to the rest start's total mass
 * sum_i V_i n_i = sum_i V_i.  An FP32-storage instance gets the FP64 state re-based into
 * deviations from the discrete equilibrium of its own moments, and keeps that state's mass.
 * Synchronises; clears a latched LBE_ENAN. */
lbe_status lbe_set_init_moments(lbe_ctx* c, int32_t inst, const double* host_in, int64_t len);
/* Start every instance from the network's prediction (n, T kept within [0.05, 20]).  With judge
 * set, one step is taken from the rest start and one from the predicted state, and an instance
 * keeps the prediction only if its residual (as in lbe_run_to_steady) is the smaller; the others
 * get the rest start.  kept[k] (may be NULL) receives 1 / 0; rho[2k], rho[2k+1] (may be NULL)
 * the two residuals (-1 without judge).  Step counters are unchanged.  FP32-storage instances are
 * handled as in lbe_set_init_moments (the rest start as lbe_init sets it).  Synchronises. */
lbe_status lbe_warm_start(lbe_ctx* c, lbe_mlp* m, int32_t judge, int32_t* kept, double* rho);

const char* lbe_last_error(const lbe_ctx* c);
const char* lbe_status_string(lbe_status s);
void lbe_free(lbe_ctx* c);

#ifdef __cplusplus
}
#endif
#endif
