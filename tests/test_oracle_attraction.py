"""Pins of the oracle's attractive mean field (Enskog-Vlasov force of a Sutherland tail).

Beyond the paper: Sec. V names attractive forces between molecules as the next step.  The
oracle integrates the tail -phi_a (sigma/t)^6 (t > sigma) about the point (spheres of radius t
about it, the cylinder's axial direction first); each pin reaches the same numbers another way:
  * the plane: a closed form from integrating over the transverse plane first;
  * the sphere: shells about the origin (the shell theorem), integrated in mpmath;
  * the cylinder: polar coordinates about the axis with the line integral in closed form, in
    mpmath;
  * special cases: the point on the axis / at the centre, and the bulk limit (the van der Waals
    value -2 a n with a = 2 pi sigma^3 phi_a / 3, i.e. Phi = -8 eta0 phi_a n);
  * the solver: Phi in a wide channel, the force within sigma of a wall (3 eta0 phi_a), its
    sign (into the fluid), Newton's third law in the plane, and the velocity moments of the
    force term (mass 0, radial momentum n F, transverse momentum 0), and the steady channel's
    momentum balance (the Enskog pressure gradient equals n F).
Tests marked "mutant" plant a mistake in a copy of the oracle and check that a pin fails.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module", autouse=True)
def _build_oracle():
    oracle.build(force=False)
    n = oracle.get_threads()
    oracle.set_threads(1)
    yield
    oracle.set_threads(n)


def _U(lib, geo, sigma, phi_a, r, s):
    if lib is None:
        return oracle.mf_potential(geo, sigma, phi_a, r, s)
    return lib.orc_mf_potential(geo, sigma, phi_a, r, s)


# ------------------------------------------------------------------ the plane
def plane_closed_form(h, sigma, phi_a):
    """U of the half space x' < x - h... written as the transverse-plane integral first:
    g(D) = 2 pi int_0^inf phi(sqrt(D^2 + rho^2)) rho drho = -(pi/2) phi_a sigma^6 / max(D^2, sigma^2)^2,
    then U = int_t^inf g(D) dD with t = x - s, piecewise in t."""
    t = h
    if t >= sigma:
        k = t ** -3 / 3
    elif t >= -sigma:
        k = (sigma - t) / sigma ** 4 + 1 / (3 * sigma ** 3)
    else:
        k = 8 / (3 * sigma ** 3) + t ** -3 / 3
    return -(math.pi / 2) * phi_a * sigma ** 6 * k


def pin_plane(lib=None):
    for sigma in (1.0, 0.3):
        for phi_a in (0.7, -0.4):
            for h in (-3.0, -1.2, -1.0, -0.5, 0.0, 0.4, 1.0, 2.5, 7.0):
                x = 5.0
                s = x - h * sigma
                u = _U(lib, 2, sigma, phi_a, x, s)
                ref = plane_closed_form(x - s, sigma, phi_a)
                assert abs(u - ref) <= 1e-14 * abs(phi_a) + 1e-14 * abs(ref), (sigma, phi_a, h, u, ref)


def test_plane_potential_closed_form():
    pin_plane()


# ------------------------------------------------------------------ the sphere
def sphere_shells(r, s, sigma, phi_a, lo=0.0):
    """int over lo < |x'| < s by shells about the origin: a shell of radius rho seen from distance r
    contributes (2 pi rho / r) int_{|r - rho|}^{r + rho} t phi(t) dt (shell theorem)."""
    mp.mp.dps = 25
    r, s, sigma, lo = mp.mpf(r), mp.mpf(s), mp.mpf(sigma), mp.mpf(lo)

    def inner(rho):
        a, b = max(abs(r - rho), sigma), max(r + rho, sigma)
        return -phi_a * sigma ** 6 * (a ** -4 - b ** -4) / 4

    pts = sorted(set([lo, s] + [x for x in (r - sigma, r + sigma, sigma - r) if lo < x < s]))
    return float(mp.quad(lambda rho: rho * 2 * mp.pi / r * inner(rho), pts))


SPHERE_POINTS = [(3.3, 4.1), (2.0, 1.5), (1.7, 1.2), (5.0, 9.0), (0.4, 2.0), (1.0, 1.0), (0.6, 0.3)]


def pin_sphere(lib=None):
    for r, s in SPHERE_POINTS:
        u = _U(lib, 1, 1.0, 0.8, r, s)
        ref = sphere_shells(r, s, 1.0, 0.8)
        assert abs(u - ref) <= 2e-14, (r, s, u, ref)


def test_sphere_potential_shells():
    pin_sphere()


def test_sphere_potential_centre_and_bulk():
    # at the centre: -4 pi phi_a sigma^6 int_sigma^s t^-4 dt
    for s in (1.5, 3.0, 10.0):
        ref = -4 * math.pi * 0.9 * (1 - s ** -3) / 3
        assert abs(oracle.mf_potential(1, 1.0, 0.9, 0.0, s) - ref) < 1e-13
    # far inside a large ball: the whole tail integral -(4 pi / 3) phi_a sigma^3 less the part
    # beyond the surface, which is below (sigma / (s - r))^3 of it
    full = -(4 * math.pi / 3) * 0.9 * 0.5 ** 3
    u = oracle.mf_potential(1, 0.5, 0.9, 10.0, 1000.0)
    assert abs(u / full - 1) < (0.5 / 990) ** 3


# ------------------------------------------------------------------ the cylinder
def line_closed_form(d, sigma, phi_a):
    """int phi(sqrt(d^2 + z^2)) dz over |z| > z0 = sqrt(max(sigma^2 - d^2, 0)), with the
    antiderivative of (d^2 + z^2)^-3."""
    d = mp.mpf(d)
    z0 = mp.sqrt(sigma ** 2 - d ** 2) if d < sigma else mp.mpf(0)

    def F(z):
        return z / (4 * d ** 2 * (d ** 2 + z ** 2) ** 2) + 3 * z / (8 * d ** 4 * (d ** 2 + z ** 2)) + \
            3 * mp.atan(z / d) / (8 * d ** 5)

    return -phi_a * sigma ** 6 * 2 * (3 * mp.pi / (16 * d ** 5) - F(z0))


def cylinder_axis_polar(r, s, sigma, phi_a):
    """int over the disk R' < s in polar coordinates about the axis, of the line integral."""
    mp.mp.dps = 20
    r, s, sigma = mp.mpf(r), mp.mpf(s), mp.mpf(sigma)

    def inner(rho):
        pts = [mp.mpf(0), mp.pi]
        if rho > 0:
            c = (r * r + rho * rho - sigma * sigma) / (2 * r * rho)
            if -1 < c < 1:
                pts = [mp.mpf(0), mp.acos(c), mp.pi]
        return 2 * mp.quad(lambda th: line_closed_form(mp.sqrt(r * r + rho * rho - 2 * r * rho * mp.cos(th)), sigma,
                                                       phi_a), pts)

    pts = sorted(set([mp.mpf(0), s] + [x for x in (r - sigma, r + sigma, sigma - r) if 0 < x < s]))
    return float(mp.quad(lambda rho: rho * inner(rho), pts))


CYL_POINTS = [(3.3, 4.1), (2.0, 1.5), (1.7, 1.2), (1.5, 2.49)]  # the last: |r - s| close to sigma


def pin_cylinder(lib=None, points=CYL_POINTS):
    for r, s in points:
        u = _U(lib, 0, 1.0, 0.8, r, s)
        ref = cylinder_axis_polar(r, s, 1.0, 0.8)
        assert abs(u - ref) <= 2e-14, (r, s, u, ref)


def test_cylinder_potential_axis_polar():
    pin_cylinder()


def test_cylinder_potential_on_axis():
    # on the axis: spheres of radius t > s lie inside the cylinder on the band |cos| > sqrt(1 - s^2/t^2),
    # so U = -4 pi phi_a sigma^6 (sigma^-3 / 3 - s^-3 int_0^1 u^2 sqrt(1 - u^2) du), the integral pi / 16
    for s in (1.5, 3.0, 10.0):
        ref = -4 * math.pi * 0.6 * (1 / 3 - math.pi / (16 * s ** 3))
        assert abs(oracle.mf_potential(0, 1.0, 0.6, 0.0, s) - ref) < 1e-13


def test_curved_potentials_reach_the_plane():
    # far from the axis / centre, a thin layer looks planar: the difference is of order sigma / R
    for geo in (0, 1):
        for h in (-2.0, -0.5, 0.7, 3.0):
            R = 1e4
            u = oracle.mf_potential(geo, 1.0, 1.0, R, R - h)
            ref = plane_closed_form(h, 1.0, 1.0)
            assert abs(u - ref) < 1e-3 * abs(ref), (geo, h, u, ref)


# ------------------------------------------------------------------ the solver
def channel(geo=2, nr=312, phi_a=0.5, eta0=0.2, C=40.0, reduced=1, L=None):
    """Walls at 1 and 1 + L (L = C: sigma = 1)."""
    kn = 1.0 / (6 * math.sqrt(2.0) * eta0 * oracle.chi(eta0) * C)
    L = C if L is None else L
    return dict(geometry=geo, r_inner=1.0, r_outer=1.0 + L, u_wall_inner=0.0, t_wall_inner=1.0, t_wall_outer=1.0,
                eta0=eta0, kn=kn, nr=nr, q_radial=4, q_t1=4, q_t2=4, cfl=0.25, reduced=reduced, phi_a=phi_a)


def pin_wide_channel(lib=None):
    """Uniform n = 1 between plates 40 sigma apart (sigma = 1/2): far from the walls Phi is the bulk
    value -8 eta0 phi_a n, less the tail beyond each edge of the fluid (a fraction (sigma/D)^3 / 8
    per side at distance D); within sigma of a wall F = 3 eta0 phi_a n / sigma, pointing into the
    fluid."""
    p = channel(L=20.0)
    s = oracle.Solver(p, lib=lib)
    phi, F = s.mean_field()
    info = s.info()
    r = s.grid()["r"]
    sig = info["sigma"]
    for i in (s.nr // 2, s.nr // 3):
        dl, dr_ = r[i] - info["rcl"], info["rcr"] - r[i]
        ref = -8 * 0.2 * 0.5 * (1 - (sig / dl) ** 3 / 8 - (sig / dr_) ** 3 / 8)
        assert abs(phi[i] - ref) < 1e-12, (i, phi[i], ref)
    # the fourth-order stencils of these nodes stay on the side of the kink of Phi'' at sigma;
    # the other wall pulls back by a fraction (sigma / distance)^4
    near = r - info["rcl"] < sig - 2 * info["dr"]
    other = (sig / (info["rcr"] - info["rcl"] - sig)) ** 4
    assert near.sum() >= 4
    assert abs(sig - 0.5) < 1e-15
    assert np.all(np.abs(F[near] / (3 * 0.2 * 0.5 / sig) - 1) < 1.01 * other + 1e-12), F[near]
    assert np.all(F[near] > 0) and np.all(F[::-1][near] < 0)
    assert np.max(np.abs(F + F[::-1])) < 1e-12


def test_wide_channel_bulk_and_walls():
    pin_wide_channel()


def pin_sphere_uniform(lib=None):
    """Uniform n = 1 between spheres: Phi_i is n0 times the tail integral over the fluid shell, by
    shells about the origin."""
    p = channel(geo=1, nr=24, C=5.0, reduced=0)
    s = oracle.Solver(p, lib=lib)
    phi, _ = s.mean_field()
    info = s.info()
    r = s.grid()["r"]
    sig = info["sigma"]
    n0 = 6 * 0.2 / (math.pi * sig ** 3)
    for i in (0, 5, 17, 23):
        ref = n0 * sphere_shells(r[i], info["rcr"], sig, 0.5, lo=info["rcl"])
        assert abs(phi[i] - ref) < 1e-12, (i, phi[i], ref)


def test_sphere_uniform_potential():
    pin_sphere_uniform()


def test_third_law_in_the_plane():
    """Pair forces cancel: sum_i n_i F_i dr vanishes up to the gradient stencil's truncation, for a
    lopsided profile (300 steps of a channel with unequal wall temperatures)."""
    p = dict(channel(nr=40, C=5.0), t_wall_outer=1.4, u_wall_inner=0.3)
    s = oracle.Solver(p)
    s.step(300)
    n = s.moments()["n"]
    _, F = s.mean_field()
    vol = s.grid()["vol"]
    assert np.max(np.abs(n - n.mean())) > 0.02
    assert abs(np.sum(vol * n * F)) < 1e-5 * np.sum(vol * np.abs(n * F))


def force_moments(p, lib=None):
    """(mass, radial momentum - n F, transverse momentum) rates of the force term of a
    non-equilibrium state, relative to max |n F|."""
    s = oracle.Solver(p, lib=lib)
    s.step(300)
    s0 = oracle.Solver(dict(p, phi_a=0.0), lib=lib)
    s0.set_f(s.get_f())
    _, F = s.mean_field()
    n = s.moments()["n"]
    dL = -(s.rhs_terms()["I"] - s0.rhs_terms()["I"])
    info = s.info()
    n0, n1, n2 = int(info["n0"]), int(info["n1"]), int(info["n2"])
    g = s.grid()
    pr = np.tile(g["p0"], n1 * n2)
    p1 = np.repeat(np.tile(g["p1"], n2), n0)
    mask = np.ones(s.nv)
    if p.get("reduced"):
        mask[n0 * n1:] = 0  # chi carries no mass
    scale = np.max(np.abs(n * F))
    assert scale > 0.1
    return (np.max(np.abs(dL @ mask)) / scale, np.max(np.abs((dL * mask) @ pr - n * F)) / scale,
            np.max(np.abs((dL * mask) @ p1)) / scale)


MOMENT_CASES = {
    "plane, reduced": (2, 1),
    "cylinder, reduced": (0, 1),
    "cylinder": (0, 0),
    "sphere": (1, 0),
}


def pin_force_moments(geo, red, lib=None):
    p = dict(channel(geo=geo, nr=40, C=5.0, reduced=red), t_wall_outer=1.4, u_wall_inner=0.0 if geo == 1 else 0.3)
    m, pr, pt = force_moments(p, lib)
    assert m < 1e-14 and pr < 1e-13 and pt < 1e-14, (m, pr, pt)


@pytest.mark.parametrize("name", sorted(MOMENT_CASES))
def test_force_term_moments(name):
    pin_force_moments(*MOMENT_CASES[name])


def test_attraction_matrix_entries():
    """Entries of A (Phi = A n) against the cell integrals by shells (sphere) and the closed form
    (plane), with n0 = 6 eta0 / (pi sigma^3)."""
    p = channel(geo=1, nr=24, C=5.0, reduced=0)
    s = oracle.Solver(p)
    A = s.attraction()
    info = s.info()
    g = s.grid()
    sig = info["sigma"]
    n0 = 6 * 0.2 / (math.pi * sig ** 3)
    for i, j in ((0, 0), (3, 5), (12, 2), (23, 17), (7, 23)):
        ref = n0 * sphere_shells(g["r"][i], g["ri"][j + 1], sig, 0.5, lo=g["ri"][j])
        assert abs(A[i, j] - ref) < 1e-13 * n0, (i, j, A[i, j], ref)
    p = channel(geo=2, nr=24, C=5.0)
    s = oracle.Solver(p)
    A = s.attraction()
    g = s.grid()
    for i, j in ((0, 0), (3, 5), (12, 2), (23, 17)):
        x = g["r"][i]
        ref = n0 * (plane_closed_form(x - g["ri"][j + 1], sig, 0.5) - plane_closed_form(x - g["ri"][j], sig, 0.5))
        assert abs(A[i, j] - ref) < 1e-13 * n0, (i, j, A[i, j], ref)
    assert not np.any(oracle.Solver(dict(p, phi_a=0.0)).attraction())


def test_attraction_thins_the_wall_layer():
    """Gas at rest between plates at T = 1 (eta0 0.2): hard spheres pile up against a hard wall
    (contact density above the middle), while the mean field pulls molecules back into the bulk,
    so with phi_a = 0.5 the wall layer is thinner than the middle.  Both steady states keep the
    mass of the uniform start."""
    from paper_2403_15051_amd import workloads

    p = workloads.attraction_case(2, nr=40, C=5.0)
    prof = {}
    for pa in (0.0, 0.5):
        s = oracle.Solver(workloads.oracle_params(dict(p, phi_a=pa)))
        m0 = s.mass()
        rc, steps, res = s.run_to_steady(1e-8, 100000, 50)
        assert rc == 0
        assert abs(s.mass() / m0 - 1) < 1e-12
        prof[pa] = s.moments()["n"]
    n0, n1 = prof[0.0], prof[0.5]
    mid = len(n0) // 2
    assert n0[0] > n0[mid] + 0.05 and n0[-1] > n0[mid] + 0.05
    assert n1[0] < n1[mid] and n1[-1] < n1[mid]
    assert n0[0] - n1[0] > 0.05


def pin_steady_balance(lib=None):
    """Steady gas at rest between plates with the mean field: the momentum equation leaves
    d P / dx = n F, with P the local Enskog pressure n T (1 + 4 eta0 n chi) (n on the mean density),
    so P minus the integral of n F from the first node is flat.  Here P varies by about 0.36 across
    the channel; the balance holds to the truncation level that P keeps without the field (7e-4)."""
    from paper_2403_15051_amd import workloads

    p = workloads.attraction_case(2, nr=40, C=5.0)
    s = oracle.Solver(workloads.oracle_params(p), lib=lib)
    rc, steps, res = s.run_to_steady(1e-8, 100000, 50)
    assert rc == 0
    m = s.moments()
    _, F = s.mean_field()
    n, T, chi = m["n"], m["T"], m["chi"]
    P = n * T * (1 + 4 * p["eta0"] * n * chi)
    dx = s.grid()["r"][1] - s.grid()["r"][0]
    nF = n * F
    work = np.concatenate([[0.0], np.cumsum(0.5 * (nF[1:] + nF[:-1]) * dx)])
    assert np.ptp(P) > 0.3
    assert np.ptp(P - work) < 3e-3, (np.ptp(P), np.ptp(P - work))


def test_steady_momentum_balance():
    pin_steady_balance()


def test_rejects_non_finite_depth():
    with pytest.raises(ValueError):
        oracle.Solver(channel(phi_a=float("nan"), nr=16))


# ------------------------------------------------------------------ planted mistakes
MUTANTS = {
    "cap measure sign": ((("return 2 * PI * t * t * (1 + mu);", "return 2 * PI * t * t * (1 - mu);"),), "sphere"),
    "half-space measure": ((("return 2 * PI * t * (t + h);", "return 2 * PI * t * (t - h);"),), "plane"),
    "arc angle": ((("return 2 * acos(cz);", "return acos(cz);"),), "cylinder"),
    "line integrand": ((("acc += h * GL10W[k] * sb * sb * sb * sb;", "acc += h * GL10W[k] * sb * sb;"),), "cylinder"),
    "density scale": ((("const double n0 = 6 * prm.eta0 / (PI * s->sigma * s->sigma * s->sigma);",
                        "const double n0 = 6 * prm.eta0 / (PI * s->sigma * s->sigma);"),), "channel"),
    "force sign": ((("nd[i].F = s->Amf ? -fd4(phi, i, nr, s->dr) : 0;", "nd[i].F = s->Amf ? fd4(phi, i, nr, s->dr) : 0;"),),
                   "channel"),
    "force term sign (plane)": ((("if (s->Amf) I = m->F * d0;", "if (s->Amf) I = -m->F * d0;"),), "moments plane"),
    "force term sign (curved)": ((("if (s->Amf && !planar) I += m->F * d0;", "if (s->Amf && !planar) I -= m->F * d0;"),),
                                 "moments sphere"),
    "force term scale": ((("if (s->Amf) I = m->F * d0;", "if (s->Amf) I = 0.5 * m->F * d0;"),), "steady balance"),
    "force on the wrong axis": ((("if (s->Amf && !planar) I += m->F * d0;", "if (s->Amf && !planar) I += m->F * d1;"),),
                                "moments sphere"),
    "transposed weights": ((("for (int j = 0; j < nr; j++) acc += s->Amf[i * nr + j] * nd[j].n;",
                             "for (int j = 0; j < nr; j++) acc += s->Amf[j * nr + i] * nd[j].n;"),), "sphere uniform"),
}


def _run_pin(kind, lib):
    if kind == "sphere":
        pin_sphere(lib)
    elif kind == "plane":
        pin_plane(lib)
    elif kind == "cylinder":
        pin_cylinder(lib, points=CYL_POINTS[:1])
    elif kind == "channel":
        pin_wide_channel(lib)
    elif kind == "sphere uniform":
        pin_sphere_uniform(lib)
    elif kind == "moments plane":
        pin_force_moments(2, 1, lib)
    elif kind == "moments sphere":
        pin_force_moments(1, 0, lib)
    elif kind == "steady balance":
        pin_steady_balance(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_attraction_pin_fails(name, tmp_path):
    subs, kind = MUTANTS[name]
    lib = oracle.load_variant(list(subs), str(tmp_path))
    with pytest.raises(AssertionError):
        _run_pin(kind, lib)
