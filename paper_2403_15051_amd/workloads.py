"""Seeded synthetic workloads: the problem statements the solver is run on.

This module only describes inputs (geometry, radii, walls, packing fraction, Knudsen number,
grid and quadrature orders); it holds none of the method's arithmetic except the closed-form
confinement ratio C = 1/(6 sqrt2 eta0 chi(eta0) Kn) (Sec. II of arXiv:2403.15051), which the
parameter sweep uses only to reject draws with sigma >= L / 1.5 and the paper's grid to state Kn
for a given C.  The paper measures on no public dataset; its own set-ups (Sec. IV) are reproduced
as synthetic problem statements.
"""
from __future__ import annotations

import numpy as np

# Cylindrical Couette, FP64: R1 = 1, R2 = 2, inner wall u_phi = 0.1, T = 1 walls, eta0 = 0.05,
# Kn = 0.1, Nr = 32, half-range order 4 in p_R, orders 4 (p_phi) and 2 (p_z), 1000 RK3 steps.
COUETTE_SMALL = dict(geometry=0, r_inner=1.0, r_outer=2.0, u_wall_inner=0.1, t_wall_inner=1.0, t_wall_outer=1.0,
                     eta0=0.05, kn=0.1, nr=32, q_radial=4, q_t1=4, q_t2=2, cfl=0.25)
COUETTE_SMALL_STEPS = 1000

# Cylindrical Fourier: walls at rest, T1 = 1, T2 = 1.5, eta0 = 0.1, Kn = 0.5, Nr = 128,
# half-range order 8, orders 8 (p_phi) and 4 (p_z).
FOURIER_CYL = dict(geometry=0, r_inner=1.0, r_outer=2.0, u_wall_inner=0.0, t_wall_inner=1.0, t_wall_outer=1.5,
                   eta0=0.1, kn=0.5, nr=128, q_radial=8, q_t1=8, q_t2=4, cfl=0.25)

# Spherical Fourier: T1 = 1, T2 = 2, eta0 = 0.2, Kn = 0.05, Nr = 256, half-range order 16,
# orders 12 (p_theta) and 12 (p_phi): 32 x 12 x 12 = 4608 velocities.
FOURIER_SPH = dict(geometry=1, r_inner=1.0, r_outer=2.0, u_wall_inner=0.0, t_wall_inner=1.0, t_wall_outer=2.0,
                   eta0=0.2, kn=0.05, nr=256, q_radial=16, q_t1=12, q_t2=12, cfl=0.25)

# The paper's own parameter grid (Sec. IV set-up), in units of sigma = 1: inner radius R_L in
# {1, 3, 5}, outer radius R_L + C with C in {4, 7, 10}, mean packing fraction eta0 in {0.01, 0.1,
# 0.2}, Kn on L = C from the Kn map of Sec. II (Table 1 lists these values), radial spacing sigma/10
# over the computational gap C - 1, time step 1e-3.  Couette: inner wall speed 1, walls at T = 1;
# Fourier: walls at 1 + 0.1 and 1 - 0.1; rest (App. B): walls at T = 1 at rest.  Velocity sets:
# cylinder HHLB(7, Q_R) x HLB(7, 8) with p_z integrated out (reduced = 1), sphere HHLB(7, Q_R) x
# HLB(7, 8) x HLB(7, 8); the planar limit (geometry 2, plates at R_L and R_L + C, the R_L -> infinity
# end of the radius sweeps) takes the cylinder's reduced set; Q_R = 20 for eta0 in {0.1, 0.2} (the paper's 100 / 60 at eta0 = 0.01 are
# passed as given: the host tables take them, the GPU stage kernel holds the radial force matrix in
# LDS and takes Q_R <= 48 with these transverse sets).
PAPER_ETA0 = (0.01, 0.1, 0.2)
PAPER_C = (4, 7, 10)
PAPER_RL = (1, 3, 5)


def paper_case(flow: str, geometry: int, eta0: float, C: float, R_L: float, q_radial: int | None = None,
               dt: float = 1e-3, precision: int = 0) -> dict:
    """One problem statement of the paper's grid (flow: 'couette', 'fourier' or 'rest'; geometry 0
    cylinder, 1 sphere, 2 plates)."""
    kn = 1.0 / (6 * np.sqrt(2.0) * eta0 * ((2 - eta0) / (2 * (1 - eta0) ** 3)) * C)
    if q_radial is None:
        q_radial = 20 if eta0 >= 0.1 else (100 if flow == "couette" else 60)
    nr = int(round(10 * (C - 1)))
    tl, tr = (1.1, 0.9) if flow == "fourier" else (1.0, 1.0)
    uw = 1.0 if flow == "couette" else 0.0
    d = dict(geometry=geometry, r_inner=float(R_L), r_outer=float(R_L + C), u_wall_inner=uw, t_wall_inner=tl,
             t_wall_outer=tr, eta0=eta0, kn=kn, nr=nr, q_radial=q_radial, q_t1=8, q_t2=8, cfl=0.25,
             reduced=0 if geometry == 1 else 1, precision=precision)
    # dt = cfl dr / max|p_R|: the largest half-range node of order Q_R is close to sqrt(4 Q_R + 2) (the
    # solver's own tables fix it exactly; dt_target is met to within that estimate)
    d["cfl"] = float(dt * np.sqrt(4 * q_radial + 2) / 0.1)
    return d


def attraction_case(geometry: int, phi_a: float = 0.5, eta0: float = 0.2, C: float = 5.0, R_L: float = 1.0,
                    nr: int = 40, q: int = 4, flow: str = "rest", precision: int = 0) -> dict:
    """A problem with the attractive mean field (beyond the paper: Enskog-Vlasov force of a
    Sutherland tail of depth phi_a k_B T), in units of sigma = 1 like the paper's grid: walls at
    R_L and R_L + C, Kn from the Kn map, half-range order q and full-range order q (p_z integrated
    out for cylinders and plates).  flow 'rest' (walls at T = 1), 'fourier' (T 1.1 / 0.9) or
    'couette' (inner wall speed 0.3)."""
    kn = 1.0 / (6 * np.sqrt(2.0) * eta0 * ((2 - eta0) / (2 * (1 - eta0) ** 3)) * C)
    tl, tr = (1.1, 0.9) if flow == "fourier" else (1.0, 1.0)
    uw = 0.3 if (flow == "couette" and geometry != 1) else 0.0
    return dict(geometry=geometry, r_inner=float(R_L), r_outer=float(R_L + C), u_wall_inner=uw, t_wall_inner=tl,
                t_wall_outer=tr, eta0=eta0, kn=kn, nr=nr, q_radial=q, q_t1=q, q_t2=q, cfl=0.25,
                reduced=0 if geometry == 1 else 1, precision=precision, phi_a=phi_a)


SWEEP_SEED = 240315051
SWEEP_ORDERS = (4, 8, 12, 16)


def _confinement(eta0: float, kn: float) -> float:
    chi = (2 - eta0) / (2 * (1 - eta0) ** 3)
    return 1.0 / (6 * np.sqrt(2.0) * eta0 * chi * kn)


def sweep(n: int = 256, seed: int = SWEEP_SEED, nr_range=(64, 512), c_min: float = 1.5):
    """Parameter sweep of uneven instances (Couette/Fourier 50/50).

    Per instance, in this order: geometry flag (Bernoulli 1/2: 0 Couette, 1 Fourier), Nr ~ U{64..512},
    eta0 ~ U(0.01, 0.3), Kn = 10^U(-2, 1) (eta0, Kn redrawn together while C < c_min),
    u_w ~ U(0, 0.5), T2/T1 ~ U(1, 2), Q ~ U{4, 8, 12, 16}.  Couette instances use u_w with
    T2/T1 = 1, Fourier instances T2/T1 with u_w = 0; both draws are always consumed.
    Velocities (2Q, Q, max(Q/2, 4)); cylindrical geometry, R1 = 1, R2 = 2, CFL 0.25.
    Returns (params list, acceptance rate of the (eta0, Kn) draws).
    """
    rng = np.random.default_rng(seed)
    out = []
    draws = 0
    for _ in range(n):
        flag = int(rng.integers(0, 2))
        nr = int(rng.integers(nr_range[0], nr_range[1] + 1))
        while True:
            eta0 = float(rng.uniform(0.01, 0.3))
            kn = float(10 ** rng.uniform(-2, 1))
            draws += 1
            if _confinement(eta0, kn) >= c_min:
                break
        uw = float(rng.uniform(0, 0.5))
        tr = float(rng.uniform(1, 2))
        q = int(SWEEP_ORDERS[int(rng.integers(0, 4))])
        out.append(dict(geometry=0, r_inner=1.0, r_outer=2.0, u_wall_inner=uw if flag == 0 else 0.0,
                        t_wall_inner=1.0, t_wall_outer=1.0 if flag == 0 else tr, eta0=eta0, kn=kn, nr=nr,
                        q_radial=q, q_t1=q, q_t2=max(q // 2, 4), cfl=0.25, flag=flag))
    return out, n / draws


def solver_params(d: dict) -> dict:
    """Drop bookkeeping keys that are not part of the problem statement."""
    return {k: v for k, v in d.items() if k != "flag"}


def oracle_params(d: dict) -> dict:
    """The problem statement without the storage precision (the oracle is FP64)."""
    return {k: v for k, v in d.items() if k not in ("flag", "precision")}


# ---------------------------------------------------------------- learned warm start inputs
MLP_LAYERS = ((6, 256), (256, 256), (256, 256), (256, 256), (256, 5))
WARM_TRAIN_SEED = 240315052
WARM_HELDOUT_SEED = 240315053


def mlp_params(seed: int) -> np.ndarray:
    """Random network parameters (uniform, Glorot scale, FP32-representable), packed layer by
    layer as W [fan_out][fan_in] then b [fan_out]."""
    rng = np.random.default_rng(seed)
    parts = []
    for fin, fout in MLP_LAYERS:
        a = np.sqrt(6.0 / (fin + fout))
        parts.append(rng.uniform(-a, a, size=fin * fout))
        parts.append(rng.uniform(-0.1, 0.1, size=fout))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def mlp_batch(seed: int, rows: int):
    """Random inputs (rows x 6) and targets (rows x 5), FP32-representable."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((rows, 6)).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((rows, 5)).astype(np.float32).astype(np.float64)
    return X, T


def mlp_grad_vector(seed: int, n: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(n) * 1e-2).astype(np.float32).astype(np.float64)


def smooth_profile(nr: int, seed: int) -> dict:
    """A smooth synthetic profile (n, u_t1, T, q_r, P_rt1) on nr nodes, for the warm-start state."""
    rng = np.random.default_rng(seed)
    x = (np.arange(nr) + 0.5) / nr
    a = rng.uniform(-1, 1, size=5)
    return {"n": 1.0 + 0.2 * a[0] * np.cos(np.pi * x), "u_t1": 0.1 * a[1] * (1 - x),
            "T": 1.0 + 0.3 * abs(a[2]) * x, "q_r": 0.02 * a[3] * np.sin(np.pi * x),
            "P_rt1": 0.01 * a[4] * (1 + x)}


def warm_sweep(n: int, seed: int, nr_range=(24, 48), orders=(4,)):
    """Training / held-out instances of the warm start: the sweep's physical draws (flag, eta0, Kn,
    u_w, T2/T1) with a reduced grid and velocity set (Nr and Q drawn from the given ranges)."""
    ps, acc = sweep(n, seed=seed, nr_range=nr_range)
    rng = np.random.default_rng(seed + 1)
    for p in ps:
        q = int(orders[int(rng.integers(0, len(orders)))])
        p.update(q_radial=q, q_t1=q, q_t2=max(q // 2, 4))
    return ps, acc
