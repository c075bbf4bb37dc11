"""CPU checks of liblbe's host side against the oracle: the library loads and exports every
entry point of include/lbe.h, rejects invalid problem statements before any device work, and
its once-per-solve tables (quadratures, force matrices, averaged-density weights, equilibrium
factors, volumes) equal the oracle's, which were built by different algorithms."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2403_15051_amd import lbe, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _libs():
    oracle.build(force=False)
    if not os.path.exists(lbe.LIB_PATH):
        pytest.skip("liblbe.so not built")
    lbe.load()


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "lbe.h")).read()
    declared = set(re.findall(r"\b(lbe_[a-z_]+)\s*\(", header))
    assert {"lbe_init", "lbe_step", "lbe_moments", "lbe_run_to_steady"} <= declared
    lib = lbe.load()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(lbe.EXPORTS) == declared


BAD = [
    dict(eta0=0.0), dict(eta0=0.5), dict(kn=-1.0), dict(nr=7), dict(q_radial=1), dict(q_radial=101), dict(q_t1=101),
    dict(n_expand=(4, 0, 0)), dict(cfl=0.0), dict(t_wall_outer=0.0), dict(r_outer=0.5),
    dict(geometry=1, u_wall_inner=0.1), dict(geometry=3), dict(geometry=-1),
    dict(geometry=1, u_wall_inner=0.0, reduced=1), dict(reduced=2), dict(eta0=0.01, kn=100.0),  # C < 1
    dict(phi_a=float("nan")), dict(phi_a=float("inf")),
]


@pytest.mark.parametrize("bad", BAD)
def test_invalid_problem_statements_are_rejected(bad):
    p = dict(workloads.COUETTE_SMALL, **bad)
    with pytest.raises(lbe.LbeError) as e:
        lbe.query([p])
    assert e.value.status == lbe.LBE_EINVAL


@pytest.mark.parametrize("reduced", [0, 1])
def test_stage_kernel_radial_order_limit(reduced):
    """The host tables take Q_R up to 100; the GPU stage kernel holds the radial force matrix in
    LDS, so lbe_query (and lbe_init) accept Q_R <= 48 with HLB(7,8) transverse sets and reject
    larger radial orders with LBE_EINVAL rather than failing at launch."""
    for q in (20, 32, 48, 56, 60, 100):
        p = dict(workloads.paper_case("couette", 0, 0.01, 4, 1, q_radial=q), reduced=reduced, q_t2=4)
        if q <= 48:
            lbe.query([p])
        else:
            with pytest.raises(lbe.LbeError) as e:
                lbe.query([p])
            assert e.value.status == lbe.LBE_EINVAL
        assert lbe.tables(p, 0).size == 4 * q


def test_stage_kernel_radial_order_limit_on_spheres():
    """Spheres keep both transverse axes (HLB(7,8) x HLB(7,8)): the stage kernel holds Q_R <= 30."""
    for q, ok in ((20, True), (30, True), (32, False), (48, False)):
        p = workloads.paper_case("fourier", 1, 0.1, 4, 1, q_radial=q)
        if ok:
            lbe.query([p])
        else:
            with pytest.raises(lbe.LbeError) as e:
                lbe.query([p])
            assert e.value.status == lbe.LBE_EINVAL


def test_query_sizes_scale():
    d1, _ = lbe.query([workloads.FOURIER_CYL])
    d2, _ = lbe.query([workloads.FOURIER_CYL] * 2)
    assert d1 > 4 * 128 * 512 * 8 and 1.9 * d1 < d2 < 2.1 * d1


CASES = [workloads.COUETTE_SMALL, workloads.FOURIER_CYL, dict(workloads.FOURIER_SPH, nr=32),
         dict(workloads.COUETTE_SMALL, q_radial=12, q_t1=6, q_t2=3, n_expand=(5, 4, 2)),
         # the paper's largest radial orders (eta0 = 0.01: Q_R = 60 Fourier, 100 Couette)
         dict(workloads.COUETTE_SMALL, q_radial=64, q_t1=8, q_t2=4),
         dict(workloads.COUETTE_SMALL, q_radial=100, q_t1=8, q_t2=4)]


@pytest.mark.parametrize("p", CASES)
def test_quadratures_match_oracle(p):
    Q = (p["q_radial"], p["q_t1"], p["q_t2"])
    for axis in range(3):
        t = lbe.tables(p, axis)
        n = t.size // 2
        x, w = oracle.quad_half(Q[0]) if axis == 0 else oracle.quad_full(Q[axis])
        assert np.allclose(t[:n], x, rtol=4e-16, atol=4e-16)
        assert np.allclose(t[n:], w, rtol=1e-14, atol=0)


@pytest.mark.parametrize("p", CASES)
def test_force_matrices_match_oracle(p):
    K1 = lbe.tables(p, 3).reshape(2 * p["q_radial"], -1)
    assert np.allclose(K1, oracle.kmat_half(p["q_radial"], 1), rtol=1e-12, atol=1e-13 * np.abs(K1).max())
    K2r = lbe.tables(p, 10).reshape(2 * p["q_radial"], -1)
    assert np.allclose(K2r, oracle.kmat_half(p["q_radial"], 2), rtol=1e-12, atol=1e-13 * np.abs(K2r).max())
    for axis, which in ((1, 4), (2, 5)):
        Q = p["q_t1"] if axis == 1 else p["q_t2"]
        K = lbe.tables(p, which).reshape(Q, Q)
        assert np.allclose(K, oracle.kmat_full(Q, 2), rtol=1e-12, atol=1e-14 * max(1, np.abs(K).max()))


def test_projection_gauss_rule_matches_oracle_rule():
    """The equilibrium projection's 32-point half-range rule is the half-range quadrature of
    order 32 (Sec. III), built here by the library's own algorithm: nodes and weights against the
    oracle's."""
    t = lbe.tables(workloads.COUETTE_SMALL, 11)
    x, w = oracle.quad_half(32)
    assert np.allclose(t[:32], x[:32], rtol=1e-15, atol=1e-15)
    assert np.allclose(t[32:], w[:32], rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("p", CASES)
def test_equilibrium_factors_match_oracle(p):
    N = p.get("n_expand", (0, 0, 0))
    Q = (p["q_radial"], p["q_t1"], p["q_t2"])
    Ns = [N[a] if N[a] else min(7, Q[a] - 1) for a in range(3)]
    for u, T in ((0.0, 1.0), (0.31, 1.37), (-0.22, 0.81)):
        g = lbe.tables(p, 8, [u, T, 0.0])
        o = [oracle.geq(True, Q[0], Ns[0], u, T), oracle.geq(False, Q[1], Ns[1], u, T),
             oracle.geq(False, Q[2], Ns[2], u, T)]
        ref = np.concatenate(o)
        # normwise per axis to a few ulps (the oracle is correctly rounded); pointwise the tail
        # nodes (weights down to 1e-15) keep only the absolute accuracy of the projection sum
        n0, n1 = len(o[0]), len(o[1])
        for sl in (slice(0, n0), slice(n0, n0 + n1), slice(n0 + n1, None)):
            assert np.abs(g[sl] - ref[sl]).max() <= 2e-15 * np.abs(ref[sl]).max()
        assert np.allclose(g, ref, rtol=1e-13, atol=2e-17)


@pytest.mark.parametrize("geometry", [0, 1])
def test_averaged_density_weights_match_oracle(geometry):
    for p in (dict(workloads.COUETTE_SMALL, geometry=geometry, u_wall_inner=0.0),
              dict(workloads.FOURIER_CYL, geometry=geometry, nr=48), dict(workloads.FOURIER_SPH, geometry=geometry,
                                                                           nr=64)):
        W = lbe.tables(p, 6).reshape(p["nr"], p["nr"])
        Wo = oracle.Solver(oracle.make_params(**{k: v for k, v in p.items()})).W()
        assert np.abs(W - Wo).max() < 2e-13, np.abs(W - Wo).max()


def test_ball_cylinder_volume_elliptic_matches_slice_integral():
    p = dict(workloads.COUETTE_SMALL)
    s = 0.3
    for R, b in ((1.0, 0.8), (1.0, 0.999), (1.0, 1.2), (1.3, 1.05), (2.0, 1.71), (1.0, 0.69), (1.0, 1.31), (1.5, 1.5001)):
        v = lbe.tables(p, 9, [s, R, b])[0]
        assert v == pytest.approx(oracle.vol_cyl(s, R, b), rel=5e-14, abs=1e-17)
    p = dict(workloads.FOURIER_SPH)
    for R, b in ((1.0, 0.8), (1.0, 1.2), (1.3, 1.05), (1.0, 1.31)):
        assert lbe.tables(p, 9, [s, R, b])[0] == pytest.approx(oracle.vol_sph(s, R, b), rel=1e-14, abs=1e-17)


@pytest.mark.parametrize("geometry", [0, 1, 2])
def test_mean_field_potential_matches_oracle(geometry):
    """The tail integral U(r; s): closed forms (plane, sphere) and the graded theta rule (cylinder)
    against the oracle's adaptive quadrature about the point."""
    p = workloads.attraction_case(geometry, phi_a=0.7)
    sig = lbe.tables(p, 13, [2.0, 2.0])  # any point: checks the call
    assert sig.shape == (1,)
    C = oracle.confinement(p["eta0"], p["kn"])
    sigma = (p["r_outer"] - p["r_inner"]) / C
    pts = [(0.0, 2.5), (0.3, 1.9), (1.0, 1.0), (2.0, 1.5), (3.3, 4.1), (5.0, 9.0), (9.0, 5.0), (1.7, 1.2),
           (4.0, 4.0 + 1e-9), (50.0, 51.5), (51.5, 50.0)]
    for r, s in pts:
        if geometry == 2 and r == 0.0:
            continue
        u = lbe.tables(p, 13, [s * sigma, r * sigma])[0]
        ref = oracle.mf_potential(geometry, sigma, 0.7, r * sigma, s * sigma)
        assert abs(u - ref) <= 3e-14 * 0.7 * sigma ** 3 + 1e-14 * abs(ref), (geometry, r, s, u, ref)


@pytest.mark.parametrize("geometry", [0, 1, 2])
def test_mean_field_weights_match_oracle(geometry):
    for kw in (dict(), dict(C=10.0, R_L=5.0, nr=90, phi_a=-0.3)):
        p = workloads.attraction_case(geometry, **kw)
        nr = p["nr"]
        A = lbe.tables(p, 12).reshape(nr, nr)
        Ao = oracle.Solver(workloads.oracle_params(p)).attraction()
        assert np.abs(A - Ao).max() < 1e-13 * np.abs(Ao).max(), np.abs(A - Ao).max()
    assert not lbe.tables(dict(p, phi_a=0.0), 12).any()


def test_sweep_generator_is_seeded_and_valid():
    a, acc = workloads.sweep(64)
    b, _ = workloads.sweep(64)
    assert a == b
    assert 0.3 < acc < 0.8
    for d in a:
        lbe.query([workloads.solver_params(d)])
