"""The planar channel (the Cartesian model equation of Sec. II, the limit R_L -> infinity of the
curved set-ups) on the GPU through the C ABI against the oracle: the paper's units and velocity sets
(HHLB(7,20) x HLB(7,8) reduced, and the three-axis set), FP64 at 1e-12 normwise, FP32 storage
profiles at 1e-5; and the approach of the cylinder to the plates as R_L grows, GPU only."""
import numpy as np
import pytest

import oracle
from paper_2403_15051_amd import lbe, workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-12

COUETTE = W.paper_case("couette", 2, 0.1, 4, 1)
FOURIER = W.paper_case("fourier", 2, 0.2, 7, 3)
FOURIER_3D = dict(W.paper_case("fourier", 2, 0.1, 4, 1), reduced=0, q_radial=8, q_t1=6, q_t2=4)


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    lbe.load()


def nrel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def profile_errors(mg, mo):
    uscale = max(np.abs(mo[k]).max() for k in ("u_r", "u_t1"))
    nT = np.abs(mo["n"]).max() * np.abs(mo["T"]).max()
    out = {}
    for k in ("n", "u_r", "u_t1", "T", "q_r", "P_rt1", "nbar", "chi"):
        scale = uscale if k.startswith("u_") else np.abs(mo[k]).max()
        if k == "q_r":
            scale = max(scale, nT * np.sqrt(np.abs(mo["T"]).max()))
        elif k == "P_rt1":
            scale = max(scale, nT)
        out[k] = float(np.abs(mg[k] - mo[k]).max() / scale)
    return out


@pytest.mark.parametrize("p", [COUETTE, FOURIER, FOURIER_3D])
def test_planar_rhs_of_an_oracle_state(p):
    print("case", p, flush=True)
    o = oracle.Solver(W.oracle_params(p))
    o.step(30)
    g = lbe.Solver(p)
    g.set_state(0, o.get_f())
    e = nrel(g.rhs(), o.rhs())
    print("rhs", e, flush=True)
    assert e <= TOL


@pytest.mark.parametrize("p", [COUETTE, FOURIER, FOURIER_3D])
def test_planar_500_steps_fp64(p):
    print("case", p, flush=True)
    o = oracle.Solver(W.oracle_params(p))
    g = lbe.Solver(p)
    o.step(500)
    g.step(500)
    e = nrel(g.get_state(), o.get_f())
    errs = profile_errors(g.moments(), o.moments())
    print("f", e, {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    assert e <= TOL
    for k, v in errs.items():
        assert v <= TOL, (k, v)


def test_planar_500_steps_fp32_storage():
    p = dict(FOURIER, precision=lbe.FP32_STORE)
    o = oracle.Solver(W.oracle_params(p))
    g = lbe.Solver(p)
    o.step(500)
    g.step(500)
    errs = profile_errors(g.moments(), o.moments())
    print({k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)


def test_plates_cylinders_and_spheres_in_one_batch():
    ps = [COUETTE, W.paper_case("couette", 0, 0.1, 4, 1), W.paper_case("fourier", 1, 0.1, 4, 1), FOURIER_3D]
    g = lbe.Solver(ps)
    g.step(100)
    for k, p in enumerate(ps):
        o = oracle.Solver(W.oracle_params(p))
        o.step(100)
        e = nrel(g.get_state(k), o.get_f())
        print("instance", k, "f", e, flush=True)
        assert e <= TOL, k


def test_planar_mass_conserved():
    g = lbe.Solver(FOURIER)
    m0 = g.moments()["n"].sum()
    g.step(300)
    assert abs(g.moments()["n"].sum() / m0 - 1) < 1e-13


def test_cylinder_rhs_tends_to_the_plates_as_the_radius_grows():
    """One state on plates and on cylinders of the same gap with R_L = 1e2, 1e3, 1e4 (one batch):
    the right-hand sides differ by the curvature terms, which fall as 1 / R_L."""
    L = COUETTE["r_outer"] - COUETTE["r_inner"]
    ps = [COUETTE] + [dict(COUETTE, geometry=0, r_inner=RL, r_outer=RL + L) for RL in (1e2, 1e3, 1e4)]
    g = lbe.Solver(ps)
    plane = lbe.Solver(COUETTE)
    plane.step(40)
    f = plane.get_state()
    for k in range(len(ps)):
        g.set_state(k, f)
    r = [g.rhs(k) for k in range(len(ps))]
    d = [nrel(r[k], r[0]) for k in (1, 2, 3)]
    print("rhs differences", d, flush=True)
    assert d[0] < 5e-2 and 8 < d[0] / d[1] < 12 and 8 < d[1] / d[2] < 12, d
