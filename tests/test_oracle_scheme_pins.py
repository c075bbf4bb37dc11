"""Pins of the oracle's time integrator, first-order Enskog term and whole-scheme steady states.

Each pin ties a part of the oracle to a fact fixed outside it:
  * the TVD Runge-Kutta step (Sec. III) is third order in time: self-convergence of the same
    semi-discretisation at four time steps;
  * the discrete J1 (eq. (j1) with the discrete equilibrium) has the same low-order velocity
    moments as the continuous eq. (j1) in its vector form, with the velocity gradient taken
    as the Cartesian Jacobian of the axisymmetric (or radial) field, so the covariant terms of
    the reduced equations are checked against plain calculus;
  * a rigidly rotating gas has no shear: J1 vanishes where the averaged density is flat;
  * converged steady states conserve the radial heat flux (Fourier, Sec. IV) and the
    angular-momentum flux (Couette, Sec. IV).
The tests marked "mutant" plant a deliberate mistake in a copy of the oracle and check that
the pin it guards fails.
"""
import os

import mpmath as mp
import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _build_oracle():
    oracle.build(force=False)
    # the problems here are small: one thread avoids the OpenMP start-up cost of every stage
    n = oracle.get_threads()
    oracle.set_threads(1)
    yield
    oracle.set_threads(n)


def equilibrium_state(s, prof):
    """f[i, v] = n_i g_R(u_r, T) g_1(u_t1, T) g_2(u_t2, T) on the oracle's discrete equilibrium."""
    info = s.info()
    n0, n1, n2 = int(info["n0"]), int(info["n1"]), int(info["n2"])
    Q = (n0 // 2, n1, n2)
    N = (int(info["N0"]), int(info["N1"]), int(info["N2"]))
    f = np.zeros((s.nr, n2, n1, n0))
    for i in range(s.nr):
        T = prof["T"][i]
        g0 = oracle.geq(True, Q[0], N[0], prof["u_r"][i], T)
        g1 = oracle.geq(False, Q[1], N[1], prof["u_t1"][i], T)
        g2 = oracle.geq(False, Q[2], N[2], prof["u_t2"][i], T)
        f[i] = prof["n"][i] * g2[:, None, None] * g1[None, :, None] * g0[None, None, :]
    return f.reshape(s.nr, -1)


def velocity_grid(s):
    g = s.grid()
    P2, P1, P0 = np.meshgrid(g["p2"], g["p1"], g["p0"], indexing="ij")
    return np.stack([P0.reshape(-1), P1.reshape(-1), P2.reshape(-1)])


# ------------------------------------------------------------------ TVD RK3 order (Sec. III)
RK_CASE = dict(geometry=0, r_inner=1.0, r_outer=2.0, u_wall_inner=0.3, t_wall_inner=1.0, t_wall_outer=1.4,
               eta0=0.1, kn=0.3, nr=16, q_radial=4, q_t1=4, q_t2=4, cfl=0.4)


def pin_rk3_third_order(lib=None):
    """Same semi-discretisation, same physical time, CFL c, c/2, c/4, c/8: a third-order step
    has error ratios e(c)/e(c/2) -> (1 - 8^-3)/(2^-3 - 8^-3) = 8.1 and e(c/2)/e(c/4) -> 9.0
    against the c/8 run."""
    s = oracle.Solver(RK_CASE, lib=lib)
    s.step(30)  # a non-equilibrium state near the moving, heated walls
    f0 = s.get_f()
    finals = []
    for k in range(4):
        t = oracle.Solver(dict(RK_CASE, cfl=RK_CASE["cfl"] / 2**k), lib=lib)
        t.set_f(f0)
        t.step(6 * 2**k)
        finals.append(t.get_f())
    e = [np.abs(finals[k] - finals[3]).max() for k in range(3)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 7.0 < r1 < 9.5 and 7.8 < r2 < 10.5, (e, r1, r2)


def test_rk3_is_third_order_in_time():
    pin_rk3_third_order()


RK_MUTANTS = {
    "stage2 weights swapped": [("0.75 * s->f[k] + 0.25 * (s->fs1[k]", "0.25 * s->f[k] + 0.75 * (s->fs1[k]")],
    "stage3 weights swapped": [("s->f[k] / 3 + 2.0 / 3 * (s->fs2[k]", "2.0 / 3 * s->f[k] + 1.0 / 3 * (s->fs2[k]")],
    "stage3 from f1": [("2.0 / 3 * (s->fs2[k] + dt", "2.0 / 3 * (s->fs1[k] + dt")],
}


@pytest.mark.parametrize("name", sorted(RK_MUTANTS))
def test_mutant_rk3_pin_fails(name, tmp_path):
    lib = oracle.load_variant(RK_MUTANTS[name], str(tmp_path))
    with pytest.raises(AssertionError):
        pin_rk3_third_order(lib)


# ------------------------------------------------------------------ J1, eq. (j1)
def cartesian_velocity_gradient(geometry, r, u, du):
    """Jacobian G[a][b] = d u_b / d x_a at the point (r, 0, 0), where the local orthonormal
    frame is (x, y, z) = (e_R, e_phi, e_z) (cylinder) or (e_r, ., .) (sphere), of the field whose
    frame components are u_a(rho) = u_a + du_a (rho - r) (cylinder: radial, azimuthal, axial;
    sphere: radial only).  Computed by numerical differentiation in 40 digits, not by the
    covariant-derivative formulas of the reduced equations."""
    mp.mp.dps = 40
    r = mp.mpf(r)
    uu = [mp.mpf(x) for x in u]
    dd = [mp.mpf(x) for x in du]

    def field(x, y, z):
        if geometry == 0:
            rho = mp.sqrt(x * x + y * y)
            ur = uu[0] + dd[0] * (rho - r)
            up = uu[1] + dd[1] * (rho - r)
            uz = uu[2] + dd[2] * (rho - r)
            return [ur * x / rho - up * y / rho, ur * y / rho + up * x / rho, uz]
        rho = mp.sqrt(x * x + y * y + z * z)
        ur = uu[0] + dd[0] * (rho - r)
        return [ur * x / rho, ur * y / rho, ur * z / rho]

    G = np.zeros((3, 3))
    pt = [r, mp.mpf(0), mp.mpf(0)]
    for a in range(3):
        for b in range(3):
            def comp(t, a=a, b=b):
                q = list(pt)
                q[a] = q[a] + t
                return field(*q)[b]
            G[a, b] = float(mp.diff(comp, 0))
    return G


def continuous_j1_moments(n, u, T, brhochi, dlog_nnchiT, dlogT, G, psis):
    """Moments int J1 psi d^3p of eq. (j1) in vector form,
        J1 = -b rho chi f^MB { xi . [grad ln(n^2 chi T) + 3/5 (zeta^2 - 5/2) grad ln T]
                              + 2/5 [2 zeta zeta : grad u + (zeta^2 - 5/2) div u] },
    zeta = xi / sqrt(2T), with the continuous Maxwellian f^MB (density n, velocity u,
    temperature T), by a 14-point Gauss-Hermite product rule (exact for these polynomial
    integrands).  Gradients are radial: grad = e_1 d/dr."""
    x, w = np.polynomial.hermite_e.hermegauss(14)
    w = w / np.sqrt(2 * np.pi)
    X0, X1, X2 = np.meshgrid(x, x, x, indexing="ij")
    W3 = (w[:, None, None] * w[None, :, None] * w[None, None, :]).reshape(-1)
    xi = np.sqrt(T) * np.stack([X0.reshape(-1), X1.reshape(-1), X2.reshape(-1)])
    p = xi + np.asarray(u)[:, None]
    zeta = xi / np.sqrt(2 * T)
    z2 = (zeta**2).sum(0)
    zGz = np.einsum("ak,ab,bk->k", zeta, G, zeta)
    div = np.trace(G)
    S = xi[0] * (dlog_nnchiT + 0.6 * (z2 - 2.5) * dlogT) + 0.4 * (2 * zGz + (z2 - 2.5) * div)
    J = -brhochi * n * S
    return np.array([(W3 * J * psi(p)).sum() for psi in psis]), np.array([(W3 * np.abs(J * psi(p))).sum()
                                                                         for psi in psis])


def monomials(maxdeg=3):
    out = []
    for a in range(maxdeg + 1):
        for b in range(maxdeg + 1 - a):
            for c in range(maxdeg + 1 - a - b):
                out.append(((a, b, c), lambda p, a=a, b=b, c=c: p[0] ** a * p[1] ** b * p[2] ** c))
    return out


J1_CASES = {
    0: dict(geometry=0, r_inner=1.0, r_outer=2.0, u_wall_inner=0.0, t_wall_inner=1.0, t_wall_outer=1.0, eta0=0.2,
            kn=0.1, nr=14, q_radial=8, q_t1=8, q_t2=8, cfl=0.25),
    1: dict(geometry=1, r_inner=1.0, r_outer=2.0, u_wall_inner=0.0, t_wall_inner=1.0, t_wall_outer=1.0, eta0=0.2,
            kn=0.1, nr=14, q_radial=8, q_t1=8, q_t2=8, cfl=0.25),
}


def j1_profiles(s, geometry):
    x = (np.arange(s.nr) + 0.5) / s.nr
    return {"n": 1.0 + 0.3 * np.sin(2.0 * x) - 0.1 * x**2, "T": 1.0 + 0.4 * x + 0.15 * np.cos(3 * x),
            "u_r": 0.12 * np.sin(2.5 * x) + 0.03, "u_t1": (0.25 - 0.2 * x**2) if geometry == 0 else 0 * x,
            "u_t2": (0.1 * np.cos(2 * x)) if geometry == 0 else 0 * x}


def pin_j1_moments(geometry, lib=None, nodes=None):
    s = oracle.Solver(J1_CASES[geometry], lib=lib)
    prof = j1_profiles(s, geometry)
    s.set_f(equilibrium_state(s, prof))
    m = s.moments()
    nc = s.node_coeffs()
    gr = s.node_grads()
    J1 = s.rhs_terms()["J1"]
    P = velocity_grid(s)
    r = s.grid()["r"]
    mons = monomials(3)
    psis = [f for _, f in mons]
    for i in (nodes if nodes is not None else range(s.nr)):
        u = [m["u_r"][i], m["u_t1"][i], m["u_t2"][i]]
        du = [gr["du_r"][i], gr["du_t1"][i], gr["du_t2"][i]]
        G = cartesian_velocity_gradient(geometry, r[i], u, du)
        C, scale = continuous_j1_moments(m["n"][i], u, m["T"][i], nc["brhochi"][i], gr["dlog_nnchiT"][i],
                                         gr["dlogT"][i], G, psis)
        D = np.array([(J1[i] * psi(P)).sum() for psi in psis])
        err = np.abs(D - C) / scale
        assert err.max() < 1e-11, (i, [mons[k][0] for k in np.argsort(-err)[:3]], err.max())


@pytest.mark.parametrize("geometry", [0, 1])
def test_j1_moments_match_continuous_eq_j1(geometry):
    pin_j1_moments(geometry)


def test_j1_gradients_are_the_fourth_order_derivatives_of_the_moments():
    """The gradients J1 uses are the (separately pinned) 4th-order differences of
    ln(n^2 chi(nbar) T), ln T and the velocity components of the current moments."""
    s = oracle.Solver(J1_CASES[0])
    prof = j1_profiles(s, 0)
    s.set_f(equilibrium_state(s, prof))
    m = s.moments()
    gr = s.node_grads()
    dr = s.info()["dr"]
    checks = {"dlog_nnchiT": np.log(m["n"] ** 2 * m["chi"] * m["T"]), "dlogT": np.log(m["T"]), "du_r": m["u_r"],
              "du_t1": m["u_t1"], "du_t2": m["u_t2"]}
    for key, phi in checks.items():
        ref = np.array([oracle.fd4(phi, i, dr) for i in range(s.nr)])
        assert np.abs(gr[key] - ref).max() <= 1e-12 * np.abs(ref).max(), key
    # the profiles really carry gradients of every kind
    for key in checks:
        assert np.abs(gr[key]).max() > 0.05, key


J1_MUTANTS = {
    "drop -u_phi/R": (0, [("(du[1 * nr + i] - m->u[1] / s->r[i])", "(du[1 * nr + i])")]),
    "drop u_R/R in shear (cyl)": (0, [("zeta[1] * zeta[1] * m->u[0] / s->r[i] + ", "")]),
    "sign of grad ln T": (0, [("0.6 * (z2 - 2.5) * dg2[i]", "-0.6 * (z2 - 2.5) * dg2[i]")]),
    "shear factor 2 dropped": (0, [("0.4 * (2 * zzgu", "0.4 * (zzgu")]),
    "div u coefficient": (0, [("(z2 - 2.5) * divu", "(z2 - 1.5) * divu")]),
    "div u without u_R/R": (0, [("divu = dur + m->u[0] / s->r[i];", "divu = dur;")]),
    "sphere div u factor": (1, [("divu = dur + 2 * m->u[0] / s->r[i];", "divu = dur + m->u[0] / s->r[i];")]),
    "sphere transverse shear dropped": (1, [
        ("zeta[0] * zeta[0] * dur + (zeta[1] * zeta[1] + zeta[2] * zeta[2]) * m->u[0] / s->r[i]",
         "zeta[0] * zeta[0] * dur")]),
    "axial shear dropped": (0, [("m->u[0] / s->r[i] + zeta[0] * zeta[2] * du[2 * nr + i]", "m->u[0] / s->r[i]")]),
}


@pytest.mark.parametrize("name", sorted(J1_MUTANTS))
def test_mutant_j1_pin_fails(name, tmp_path):
    geometry, subs = J1_MUTANTS[name]
    lib = oracle.load_variant(subs, str(tmp_path))
    with pytest.raises(AssertionError):
        pin_j1_moments(geometry, lib=lib, nodes=range(3, 11))


# ------------------------------------------------------------------ rigid rotation
def pin_rigid_rotation(lib=None):
    """u_phi = Omega r, u_R = 0, uniform n and T: the covariant shear d_R u_phi - u_phi/R and
    div u vanish, so J1 = 0 wherever the averaged density is flat (rows of W summing to one over
    the whole fourth-order stencil), while the rotation itself is not small."""
    p = dict(J1_CASES[0], eta0=0.1, kn=0.05, nr=40, q_radial=4, q_t1=6, q_t2=4)
    s = oracle.Solver(p, lib=lib)
    r = s.grid()["r"]
    om = 0.3
    prof = {"n": np.ones(s.nr), "T": np.ones(s.nr), "u_r": np.zeros(s.nr), "u_t1": om * r, "u_t2": np.zeros(s.nr)}
    f = equilibrium_state(s, prof)
    s.set_f(f)
    rows = s.W().sum(1)
    flat = np.array([all(abs(rows[j] - 1) < 1e-14 for j in range(i - 2, i + 3) if 0 <= j < s.nr) and 2 <= i < s.nr - 2
                     for i in range(s.nr)])
    assert flat.sum() >= 8
    J1 = s.rhs_terms()["J1"]
    nc = s.node_coeffs()
    for i in np.nonzero(flat)[0]:
        assert np.abs(J1[i]).max() <= 1e-12 * nc["brhochi"][i] * np.abs(f[i]).max(), i
    assert np.abs(J1[~flat]).max() > 1e-3 * np.abs(f).max()  # the walls' averaged density does act


def test_rigid_rotation_has_no_enskog_shear_term():
    pin_rigid_rotation()


def test_mutant_rigid_rotation_pin_fails(tmp_path):
    lib = oracle.load_variant(J1_MUTANTS["drop -u_phi/R"][1], str(tmp_path))
    with pytest.raises(AssertionError):
        pin_rigid_rotation(lib)


# ------------------------------------------------------------------ converged steady states
def load_fixture(name):
    path = os.path.join(HERE, "golden", name + ".txt")
    if not os.path.exists(path):
        pytest.skip(f"fixture {name} not generated")
    d = {}
    for line in open(path):
        if line.startswith("# steps"):
            d["steps"] = int(line.split()[2])
            continue
        if line[0] == "#":
            continue
        k, *v = line.split()
        d[k] = np.array([float(x) for x in v])
    return d


FOURIER = {  # problem, tolerance on the whole channel, on the interior (two cells from each wall)
    "steady_fourier_cyl": (dict(geometry=0, r_inner=1.0, r_outer=2.0, u_wall_inner=0.0, t_wall_inner=1.0,
                                t_wall_outer=1.5, eta0=0.1, kn=0.5, nr=128, q_radial=8, q_t1=8, q_t2=4, cfl=0.25),
                           5e-4, 1e-4),
    "steady_fourier_cyl_small": (dict(geometry=0, r_inner=1.0, r_outer=2.0, u_wall_inner=0.0, t_wall_inner=1.0,
                                      t_wall_outer=1.5, eta0=0.1, kn=0.5, nr=32, q_radial=4, q_t1=4, q_t2=4,
                                      cfl=0.25), 2e-3, 1e-4),
    "steady_fourier_sph": (dict(geometry=1, r_inner=1.0, r_outer=2.0, u_wall_inner=0.0, t_wall_inner=1.0,
                                t_wall_outer=2.0, eta0=0.2, kn=0.05, nr=256, q_radial=16, q_t1=12, q_t2=12,
                                cfl=0.25), 1e-2, 1e-3),
}


@pytest.mark.parametrize("name", sorted(FOURIER))
def test_fourier_steady_heat_flux_times_area_is_constant(name):
    """Sec. IV Fourier flow: at steady state the energy equation reduces to d(r^{D-1} q_r)/dr = 0
    (the inertial terms and the Shakhov term conserve energy, J1's energy moment vanishes with
    u_r), so r^{D-1} q_r is constant up to truncation error, while q_r itself varies.  The cells
    next to the walls carry the largest truncation error (the wall ghosts enter their WENO
    stencils; up to 0.5 % on the dense sphere), the interior is held tighter."""
    p, tol, tol_in = FOURIER[name]
    d = load_fixture(name)
    r = oracle.Solver(dict(p, q_radial=4, q_t1=4, q_t2=4)).grid()["r"]  # the grid does not depend on the orders
    D = 2 if p["geometry"] == 0 else 3
    flux = d["q_r"] * r ** (D - 1)
    assert np.ptp(d["q_r"]) > 0.1 * np.abs(d["q_r"]).max()
    assert np.ptp(flux) < tol * np.abs(flux.mean()), np.ptp(flux) / np.abs(flux.mean())
    assert np.ptp(flux[2:-2]) < tol_in * np.abs(flux.mean()), np.ptp(flux[2:-2]) / np.abs(flux.mean())
    assert np.abs(d["u_r"]).max() < 1e-3 * np.sqrt(p["t_wall_outer"])


def test_couette_steady_angular_momentum_flux_is_constant():
    """Sec. IV Couette flow near the Boltzmann limit (eta0 = 1e-4, so J1 is negligible): the
    phi-momentum balance at steady state is d(R^2 P_R phi)/dR = 0, so R^2 P_R phi is constant up
    to truncation error."""
    d = load_fixture("steady_couette_dilute")
    p = dict(geometry=0, r_inner=1.0, r_outer=2.0, u_wall_inner=0.1, t_wall_inner=1.0, t_wall_outer=1.0, eta0=1e-4,
             kn=0.1, nr=32, q_radial=8, q_t1=8, q_t2=4, cfl=0.25)
    r = oracle.Solver(p).grid()["r"]
    flux = d["P_rt1"] * r**2
    assert np.ptp(d["P_rt1"]) > 0.2 * np.abs(d["P_rt1"]).max()
    # the cells next to the walls (Knudsen layers, wall ghosts in their stencils) to 2 %, the
    # interior to 1e-3
    assert np.ptp(flux) < 2e-2 * np.abs(flux.mean()), np.ptp(flux) / np.abs(flux.mean())
    assert np.ptp(flux[2:-2]) < 1e-3 * np.abs(flux.mean()), np.ptp(flux[2:-2]) / np.abs(flux.mean())
