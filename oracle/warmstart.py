"""Plain FP64 reference of the warm-start state (Grad-13 reconstruction and mass renormalisation).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Not part of the paper.  Given the profile (n, u_t1, T, q_r, P_r,t1) at every radial node, with the
radial and second transverse velocities zero, the state is the Grad 13-moment distribution built
on the discrete equilibrium of Sec. III.C (the same n g_r g_1 g_2 as the collision term):
    f_v = f^MB_v [1 + P xi_r xi_1 / (n T^2) + (q xi_r / (n T^2)) (|xi|^2 / (5 T) - 1)],  xi = p - u,
whose moments reproduce the five inputs when the quadrature is exact for them.  The whole state
is then scaled by one factor so that the total mass sum_i V_i n_i equals that of the rest start
(n = 1 at every node), because the closed system's steady state depends on its mass.
"""
from __future__ import annotations

import numpy as np

from . import Solver, geq


def grad13_state(params: dict, prof: dict) -> np.ndarray:
    """f [nr][nv] for the profile prof = {n, u_t1, T, q_r, P_rt1} (arrays of nr), renormalised."""
    s = Solver(params)
    info = s.info()
    g = s.grid()
    nr = s.nr
    n0, n1, n2 = int(info["n0"]), int(info["n1"]), int(info["n2"])
    N0, N1, N2 = int(info["N0"]), int(info["N1"]), int(info["N2"])
    Q0, Q1, Q2 = n0 // 2, n1, n2
    f = np.zeros((nr, n2, n1, n0))
    for i in range(nr):
        n, ut, T = prof["n"][i], prof["u_t1"][i], prof["T"][i]
        q, P = prof["q_r"][i], prof["P_rt1"][i]
        g0 = geq(True, Q0, N0, 0.0, T)
        g1 = geq(False, Q1, N1, ut, T)
        g2 = geq(False, Q2, N2, 0.0, T)
        fmb = n * g2[:, None, None] * g1[None, :, None] * g0[None, None, :]
        xr = g["p0"][None, None, :]
        xt = (g["p1"] - ut)[None, :, None]
        xz = g["p2"][:, None, None]
        xi2 = xr * xr + xt * xt + xz * xz
        f[i] = fmb * (1 + P * xr * xt / (n * T * T) + (q * xr / (n * T * T)) * (xi2 / (5 * T) - 1))
    f = f.reshape(nr, n0 * n1 * n2)
    vol = g["vol"]
    mass = (vol * f.sum(axis=1)).sum()
    return f * (vol.sum() / mass)


def profile_moments(params: dict, f: np.ndarray) -> dict:
    """(n, u_t1, T, q_r, P_rt1) of a state by direct quadrature sums (two passes)."""
    s = Solver(params)
    info = s.info()
    g = s.grid()
    n0, n1, n2 = int(info["n0"]), int(info["n1"]), int(info["n2"])
    F = f.reshape(-1, n2, n1, n0)
    pr = g["p0"][None, None, None, :]
    p1 = g["p1"][None, None, :, None]
    p2 = g["p2"][None, :, None, None]
    n = F.sum(axis=(1, 2, 3))
    ur = (F * pr).sum(axis=(1, 2, 3)) / n
    ut = (F * p1).sum(axis=(1, 2, 3)) / n
    uz = (F * p2).sum(axis=(1, 2, 3)) / n
    xr = pr - ur[:, None, None, None]
    xt = p1 - ut[:, None, None, None]
    xz = p2 - uz[:, None, None, None]
    xi2 = xr * xr + xt * xt + xz * xz
    T = (F * xi2).sum(axis=(1, 2, 3)) / (3 * n)
    q = 0.5 * (F * xi2 * xr).sum(axis=(1, 2, 3))
    P = (F * xr * xt).sum(axis=(1, 2, 3))
    return {"n": n, "u_r": ur, "u_t1": ut, "T": T, "q_r": q, "P_rt1": P}
