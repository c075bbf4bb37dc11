"""Batched sweep machinery on the GPU (through the C ABI): the captured HIP graphs of the RK3
step and of the steady-state check interval, the device-side freeze of converged instances, and
the tile autotuner.  Graph replay changes no arithmetic, so that comparison is bitwise; the tile
height changes each tile's velocity shift (rounding only, compared at 1e-12 normwise); batched
steady solves are compared with solo solves of the oracle."""
import numpy as np
import pytest

import oracle
from paper_2403_15051_amd import lbe, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    lbe.load()


def uneven_batch():
    """Five instances, two geometries, three velocity sets, ragged Nr."""
    return [
        dict(workloads.COUETTE_SMALL, nr=37),
        dict(workloads.FOURIER_SPH, nr=29, q_radial=4, q_t1=4, q_t2=4),
        dict(workloads.FOURIER_CYL, nr=70, q_radial=6, q_t1=6, q_t2=4),
        dict(workloads.COUETTE_SMALL, nr=21, u_wall_inner=0.3),
        dict(workloads.FOURIER_CYL, nr=45, q_radial=6, q_t1=6, q_t2=4, kn=0.5),
    ]


def states(g):
    return [g.get_state(k).copy() for k in range(g.n_inst)]


def test_graph_replay_is_bitwise_equal_to_eager_launches(monkeypatch):
    ps = uneven_batch()
    g = lbe.Solver(ps)
    monkeypatch.setenv("LBE_GRAPH", "0")
    e = lbe.Solver(ps)
    monkeypatch.delenv("LBE_GRAPH")
    g.step(25)
    e.step(25)
    g.sync()
    e.sync()
    for k, (a, b) in enumerate(zip(states(g), states(e))):
        assert np.array_equal(a, b), k


def nrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_autotune_keeps_results_to_rounding():
    ps = uneven_batch()
    a = lbe.Solver(ps)
    b = lbe.Solver(ps)
    a.step(3)
    b.step(3)
    rep = a.autotune(reps=2)
    print("autotune", rep, flush=True)
    assert 3 <= len(rep) <= 6  # three velocity sets; a large one is split in two
    for r in rep:
        assert r["tile_nodes"] in (4, 8, 16, 32, 64) and r["ms"] > 0 and r["ms"] <= r["ms_before"]
    a.step(20)
    b.step(20)
    for k, (x, y) in enumerate(zip(states(a), states(b))):
        assert nrel(x, y) <= 1e-13, k
    for k in range(len(ps)):
        ma, mb = a.moments(k), b.moments(k)
        for f in ("n", "T", "q_r"):
            assert nrel(ma[f], mb[f]) <= 1e-12, (k, f)


def test_batched_steady_state_freezes_each_instance_on_its_own_step():
    """Each instance of an uneven batch stops on the step where its own residual first drops
    below tol, with the oracle's step count and profile."""
    ps = [
        dict(workloads.COUETTE_SMALL, nr=16, q_t2=4, kn=0.3),
        dict(workloads.COUETTE_SMALL, nr=20, q_t2=4, kn=1.0, u_wall_inner=0.2),
        dict(workloads.FOURIER_CYL, nr=16, q_radial=4, q_t1=4, q_t2=4, kn=0.5),
    ]
    g = lbe.Solver(ps)
    st, steps, res = g.run_to_steady(1e-5, 20000, 50)
    assert st == lbe.LBE_OK
    print("steps", steps, "res", res, flush=True)
    for k, p in enumerate(ps):
        o = oracle.Solver(p)
        rc, so, ro = o.run_to_steady(1e-5, 20000, 50)
        assert rc == 0
        assert steps[k] == so, (k, steps[k], so)
        assert res[k] == pytest.approx(ro, rel=1e-6)
        mg, mo = g.moments(k), o.moments()
        # velocities are j/n with j a sum of O(sqrt T) terms, so their rounding floor is about
        # eps sqrt(T): a flow speed that is only truncation-small (Fourier) is measured against
        # 1e-3 of the thermal speed
        uscale = max(max(np.abs(mo[f]).max() for f in ("u_r", "u_t1", "u_t2")), 1e-3 * np.sqrt(mo["T"].max()))
        for f in ("n", "T", "u_r", "u_t1"):
            scale = uscale if f.startswith("u_") else np.abs(mo[f]).max()
            assert np.abs(mg[f] - mo[f]).max() / scale <= 1e-12, (k, f)
    assert len(set(steps.tolist())) > 1  # the instances froze on different steps


def test_run_to_steady_reports_not_converged_and_partial_chunk():
    p = dict(workloads.COUETTE_SMALL, nr=16, q_t2=4)
    g = lbe.Solver(p)
    st, steps, res = g.run_to_steady(1e-14, 130, 50)
    assert st == lbe.LBE_ENOTCONV
    assert steps[0] == 130 and res[0] > 1e-14
    assert g.info()["steps"] == 130


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_full_sweep_sampled_instances_match_oracle(precision, tol):
    """The 256-instance sweep at its full size, in the configuration bench.py times (autotuned
    tiles, captured steps, forked group chains): after 200 steps, the smallest, the largest, the
    first instance and the first of each velocity order (so every launch group, with its own
    workgroup size and tile mode, is checked) match the oracle run on their own: FP64 1e-12
    normwise on f and on the six profiles; FP32 storage 1e-5 on the six profiles (velocities
    against the largest velocity component, q and P floored at n T^(3/2) and n T)."""
    steps = 200
    ps, _ = workloads.sweep(256)
    ps = [dict(workloads.solver_params(p), precision=precision) for p in ps]
    g = lbe.Solver(ps)
    g.autotune(reps=1)
    g.step(steps)
    g.sync()
    size = [p["nr"] * (2 * p["q_radial"]) * p["q_t1"] * p["q_t2"] for p in ps]
    first_of_order = {next(k for k, p in enumerate(ps) if p["q_radial"] == q) for q in workloads.SWEEP_ORDERS}
    for k in sorted({0, int(np.argmin(size)), int(np.argmax(size))} | first_of_order):
        p = {kk: v for kk, v in ps[k].items() if kk != "precision"}
        print("sweep instance", k, "size", size[k], p, flush=True)
        o = oracle.Solver(p)
        o.step(steps)
        if precision == 0:
            f_o = o.get_f()
            e = nrel(g.get_state(k), f_o)
            print("sweep instance", k, "f", e, flush=True)
            assert e <= tol, k
        mg, mo = g.moments(k), o.moments()
        uscale = max(np.abs(mo[f]).max() for f in ("u_r", "u_t1", "u_t2"))
        nT = np.abs(mo["n"]).max() * np.abs(mo["T"]).max()
        for f in ("n", "u_r", "u_t1", "T", "q_r", "P_rt1"):
            scale = uscale if f.startswith("u_") else np.abs(mo[f]).max()
            if f == "q_r":
                scale = max(scale, nT * np.sqrt(np.abs(mo["T"]).max()))
            elif f == "P_rt1":
                scale = max(scale, nT)
            e = float(np.abs(mg[f] - mo[f]).max() / scale)
            print("sweep instance", k, f, e, flush=True)
            assert e <= tol, (k, f)
