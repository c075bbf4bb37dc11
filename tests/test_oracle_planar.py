"""Pins of the oracle's planar channel (the Cartesian model equation of Sec. II, the R_L -> infinity
limit of the curvilinear set-ups): cap volumes against numerical integration, the averaged-density
weights, mass conservation, the dilute-limit stationary Maxwellian, the approach of the cylinder to
the planar right-hand side as R_L grows (curvature terms ~ L / R_L), and the App. B rest state."""
import mpmath as mp
import numpy as np
import pytest

import oracle

PLANE = dict(geometry=2, r_inner=1.0, r_outer=2.0, u_wall_inner=0.2, t_wall_inner=1.0, t_wall_outer=1.2, eta0=0.15,
             kn=0.2, nr=24, q_radial=6, q_t1=6, q_t2=4, cfl=0.25)


@pytest.fixture(scope="module", autouse=True)
def _build_oracle():
    oracle.build(force=False)
    n = oracle.get_threads()
    oracle.set_threads(1)
    yield
    oracle.set_threads(n)


def test_cap_volume_against_integration():
    """Volume of {x < X} inside the ball of radius s at x = b: the integral of the disk areas
    pi (s^2 - (x - b)^2) over x < X."""
    for s, X, b in ((0.3, 1.3, 1.2), (0.3, 1.0, 1.2), (0.5, 0.9, 1.0), (0.2, 2.0, 1.0), (0.4, 0.1, 1.0)):
        lo, hi = b - s, min(X, b + s)
        ref = float(mp.quad(lambda x: mp.pi * (s * s - (x - b) ** 2), [lo, hi])) if hi > lo else 0.0
        assert oracle.vol_slab(s, X, b) == pytest.approx(ref, rel=1e-14, abs=1e-16)


def test_planar_averaged_density_weights():
    p = dict(PLANE, eta0=0.2, kn=0.05, nr=40)
    s = oracle.Solver(p)
    W = s.W()
    info, r = s.info(), s.grid()["r"]
    far = (r - info["rcl"] > info["sigma"]) & (info["rcr"] - r > info["sigma"])
    assert far.any() and (~far).any()
    assert np.allclose(W.sum(1)[far], 1.0, atol=1e-14)
    # a node at the computational wall sees exactly half of its ball inside the domain
    assert W.sum(1)[0] == pytest.approx(0.5 + 0.75 * (s.info()["dr"] / 2) / info["sigma"]
                                        - 0.25 * ((s.info()["dr"] / 2) / info["sigma"]) ** 3, rel=1e-12)


@pytest.mark.parametrize("reduced", [0, 1])
def test_planar_mass_conserved_to_roundoff(reduced):
    s = oracle.Solver(dict(PLANE, reduced=reduced))
    m0 = s.mass()
    s.step(150)
    assert abs(s.mass() / m0 - 1) < 1e-13


def test_planar_uniform_maxwellian_is_stationary_in_the_dilute_limit():
    s = oracle.Solver(dict(PLANE, u_wall_inner=0.0, t_wall_outer=1.0, eta0=1e-12))
    f0 = s.get_f()
    s.step(50)
    assert np.abs(s.get_f() - f0).max() <= 4e-16 * np.abs(f0).max()


def test_cylinder_approaches_the_plates_as_the_radius_grows():
    """The same gap, state and problem on coaxial cylinders of inner radius R_L and on plates: the
    right-hand sides differ by the curvature terms, of order L / R_L."""
    plane = oracle.Solver(PLANE)
    plane.step(20)
    f = plane.get_f()
    L = PLANE["r_outer"] - PLANE["r_inner"]
    diffs = []
    for RL in (1e2, 1e3, 1e4):
        cyl = oracle.Solver(dict(PLANE, geometry=0, r_inner=RL, r_outer=RL + L))
        cyl.set_f(f)
        diffs.append(np.abs(cyl.rhs() - plane.rhs()).max() / np.abs(plane.rhs()).max())
    assert diffs[0] < 2e-2 and 8 < diffs[0] / diffs[1] < 12 and 8 < diffs[1] / diffs[2] < 12, diffs


def test_planar_rest_state_enskog_pressure_balance():
    """App. B between plates: layering of n at both walls with n (1 + 4 eta0 n chi) flat to a small
    fraction of the layering amplitude, T and u_x at their truncation level."""
    p = dict(PLANE, u_wall_inner=0.0, t_wall_outer=1.0, eta0=0.2, kn=0.05)
    s = oracle.Solver(p)
    rc, steps, res = s.run_to_steady(1e-6, 40000, 200)
    assert rc == 0
    m = s.moments()
    pr = m["n"] * (1 + 4 * 0.2 * m["n"] * m["chi"])
    assert np.ptp(m["n"]) > 0.08
    assert np.ptp(pr) < 0.1 * np.ptp(m["n"])
    # the plates are symmetric: the profile is mirror-symmetric
    assert np.abs(m["n"] - m["n"][::-1]).max() < 1e-6
