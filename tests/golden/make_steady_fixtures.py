"""Write the converged oracle profiles used by the steady-state parity tests and invariant pins.

Calls only the CPU oracle (oracle/).  Cases:
  steady_fourier_cyl        cylindrical Fourier (R 1..2, T 1 / 1.5, eta0 0.1, Kn 0.5, Nr 128, orders 8, 8, 4)
  steady_fourier_cyl_small  the same physics on Nr 32, orders 4, 4, 4
  steady_fourier_sph        spherical Fourier (R 1..2, T 1 / 2, eta0 0.2, Kn 0.05, Nr 256, orders 16, 12, 12)
  steady_couette_dilute     cylindrical Couette near the Boltzmann limit (eta0 1e-4), orders 8, 8, 4
  rest_state_nr24, _nr48    gas at rest between walls at T = 1 (App. B), eta0 0.2, Kn 0.05, orders 6, 6, 4
The Fourier and Couette cases are solved to a residual of 1e-8 checked every 50 steps, the rest
states to 1e-6 checked every 200.  Output: one text file per case with the step count, the last
residual and the profiles n, u_r, u_t1, T, q_r, P_rt1, nbar, chi (one row per field).

The solve runs in chunks of whole check intervals, so it stops on the same step as one long call;
with --ckpt-dir the state after each chunk is saved there and a restarted run resumes from it.

    python tests/golden/make_steady_fixtures.py [case ...] [--threads N] [--ckpt-dir DIR]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2403_15051_amd import workloads as W  # noqa: E402

REST = dict(geometry=0, r_inner=1.0, r_outer=2.0, u_wall_inner=0.0, t_wall_inner=1.0, t_wall_outer=1.0, eta0=0.2,
            kn=0.05, q_radial=6, q_t1=6, q_t2=4, cfl=0.25)
CASES = {  # name: (problem, residual tolerance, check interval)
    "steady_fourier_cyl": (dict(W.FOURIER_CYL), 1e-8, 50),
    "steady_fourier_cyl_small": (dict(W.FOURIER_CYL, nr=32, q_radial=4, q_t1=4, q_t2=4), 1e-8, 50),
    "steady_fourier_sph": (dict(W.FOURIER_SPH), 1e-8, 50),
    "steady_couette_dilute": (dict(W.COUETTE_SMALL, eta0=1e-4, q_radial=8, q_t1=8, q_t2=4), 1e-8, 50),
    "rest_state_nr24": (dict(REST, nr=24), 1e-6, 200),
    "rest_state_nr48": (dict(REST, nr=48), 1e-6, 200),
}
DEFAULT = ("steady_fourier_cyl", "steady_fourier_cyl_small")
FIELDS = ("n", "u_r", "u_t1", "T", "q_r", "P_rt1", "nbar", "chi")


def solve(name, p, tol, check, ckpt_dir):
    s = oracle.Solver(p)
    done = 0
    ck = os.path.join(ckpt_dir, name + ".ckpt.npz") if ckpt_dir else None
    if ck and os.path.exists(ck):
        z = np.load(ck)
        s.set_f(z["f"])
        done = int(z["steps"])
        print(f"{name}: resumed at step {done}", flush=True)
    while True:
        rc, steps, res = s.run_to_steady(tol, 100 * check, check)
        done += steps
        print(f"{name}: step {done} residual {res:.3e}", flush=True)
        if rc == 0:
            return s, done, res
        assert rc == 1 and done < 2_000_000, (name, rc, done, res)
        if ck:
            np.savez(ck + ".tmp.npz", f=s.get_f(), steps=done)
            os.replace(ck + ".tmp.npz", ck)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=list(DEFAULT))
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--ckpt-dir", default="")
    a = ap.parse_args()
    oracle.build(force=False)
    if a.threads:
        oracle.set_threads(a.threads)
    for name in a.cases:
        p, tol, check = CASES[name]
        t0 = time.time()
        s, steps, res = solve(name, p, tol, check, a.ckpt_dir)
        m = s.moments()
        path = os.path.join(HERE, name + ".txt")
        with open(path, "w") as fh:
            fh.write(f"# oracle steady state, residual {tol:g} checked every {check} steps; params {p}\n")
            fh.write(f"# steps {steps} residual {res!r}\n")
            for f in FIELDS:
                fh.write(f + " " + " ".join(repr(float(x)) for x in m[f]) + "\n")
        print(name, steps, res, f"{time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
