"""Pins of the oracle's reduced distributions (cylinder with p_z integrated out, Sec. III
"Quadrature choice"): phi = int f dp_z and chi = int p_z^2 f dp_z on the (p_R, p_phi) quadrature.

The reduction commutes with every linear part of the scheme, and the collision integrals over p_z
are exact for a p_z quadrature of order 5 with expansion order 4 (the polynomials in xi_z are at
most quadratic, times p_z^2 quartic).  So on a full three-axis state f and its reduction
(phi, chi) = sum_k (1, p_k^2) f_k, the force terms, the Shakhov and Enskog terms and the moments
of the reduced model equal the same sums of the three-axis model's, to rounding.  The face
reconstruction (WENO-5) is nonlinear, so the advection terms agree only to the reconstruction's
accuracy: exactly where the data are smooth as the grid is refined, not at the wall faces where
the nonlinear weights act on the ghost jump."""
import numpy as np
import pytest

import oracle

BASE = dict(geometry=0, r_inner=1.0, r_outer=2.0, u_wall_inner=0.3, t_wall_inner=1.0, t_wall_outer=1.3, eta0=0.15,
            kn=0.2, nr=16, q_radial=8, q_t1=8, q_t2=5, cfl=0.25, n_expand=(0, 0, 4))


@pytest.fixture(scope="module", autouse=True)
def _build_oracle():
    oracle.build(force=False)
    n = oracle.get_threads()
    oracle.set_threads(1)
    yield
    oracle.set_threads(n)


def pair(nr=16, steps=20):
    full = oracle.Solver(dict(BASE, nr=nr))
    red = oracle.Solver(dict(BASE, nr=nr, reduced=1))
    full.step(steps)
    pz = full.grid()["p2"]

    def reduce(f):
        F = f.reshape(full.nr, len(pz), -1)
        return np.concatenate([F.sum(1), (F * pz[None, :, None] ** 2).sum(1)], axis=1)

    red.set_f(reduce(full.get_f()))
    return full, red, reduce


def test_reduced_shape():
    full, red, _ = pair()
    assert red.shape == (2, 8, 16) and red.nv == 2 * 8 * 16
    assert red.info()["n2"] == 2


def test_reduced_collision_force_terms_and_moments_equal_the_pz_moments_of_the_full_model():
    full, red, reduce = pair()
    tf, tr = full.rhs_terms(), red.rhs_terms()
    for k in ("I", "J0", "J1"):
        a, b = reduce(tf[k]), tr[k]
        e = np.abs(a - b).max() / np.abs(b).max()
        assert e < 5e-13, (k, e)
    mf, mr = full.moments(), red.moments()
    for f in ("n", "u_r", "u_t1", "T", "q_r", "P_rt1", "nbar", "chi"):
        assert np.abs(mf[f] - mr[f]).max() <= 1e-14 * max(1.0, np.abs(mf[f]).max()), f
    assert np.abs(mr["u_t2"]).max() == 0.0
    assert np.abs(mr["T"] - 1).max() > 1e-3  # the state is not isothermal: chi carries T


def test_reduced_advection_agrees_where_the_reconstruction_is_linear():
    """Interior cells (away from the walls' ghost jump): the difference falls with refinement
    far faster than the grid spacing; it vanishes in the limit where WENO-5's weights are the
    linear ones."""
    inner = []
    for nr in (16, 32, 64):
        full, red, reduce = pair(nr=nr, steps=20 * nr // 16)
        a, b = reduce(full.rhs_terms()["A"]), red.rhs_terms()["A"]
        d = np.abs(a - b).max(axis=1) / np.abs(b).max()
        inner.append(d[nr // 2 - 2:nr // 2 + 2].max())
    assert inner[0] < 1e-2 and inner[1] < 1e-4 and inner[2] < 0.05 * inner[1], inner


def test_reduced_mass_conserved_to_roundoff():
    red = oracle.Solver(dict(BASE, reduced=1))
    m0 = red.mass()
    red.step(150)
    assert abs(red.mass() / m0 - 1) < 1e-13


def test_reduced_uniform_maxwellian_is_stationary_in_the_dilute_limit():
    red = oracle.Solver(dict(BASE, reduced=1, u_wall_inner=0.0, t_wall_outer=1.0, eta0=1e-12))
    f0 = red.get_f()
    red.step(50)
    assert np.abs(red.get_f() - f0).max() <= 4e-16 * np.abs(f0).max()


def test_reduced_rest_start_is_phi_and_T_phi():
    red = oracle.Solver(dict(BASE, reduced=1))
    f = red.get_f().reshape(red.nr, 2, -1)
    assert np.array_equal(f[:, 0], f[:, 1])  # chi = T phi with T = 1
    m = red.moments()
    assert np.allclose(m["T"], 1.0, atol=1e-15) and np.allclose(m["n"], 1.0, atol=1e-15)
