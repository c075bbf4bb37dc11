"""Write the converged oracle profiles used by the steady-state parity tests and invariant pins.

Calls only the CPU oracle (oracle/).  Cases:
  steady_fourier_cyl        cylindrical Fourier (R 1..2, T 1 / 1.5, eta0 0.1, Kn 0.5, Nr 128, orders 8, 8, 4)
  steady_fourier_cyl_small  the same physics on Nr 32, orders 4, 4, 4
  steady_fourier_sph        spherical Fourier (R 1..2, T 1 / 2, eta0 0.2, Kn 0.05, Nr 256, orders 16, 12, 12)
  steady_couette_dilute     cylindrical Couette near the Boltzmann limit (eta0 1e-4), orders 8, 8, 4
Each is solved to a residual of 1e-8 checked every 50 steps.  Output: one text file per case with
the step count, the last residual and the profiles n, u_r, u_t1, T, q_r, P_rt1 (one row per field).

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

CASES = {
    "steady_fourier_cyl": dict(W.FOURIER_CYL),
    "steady_fourier_cyl_small": dict(W.FOURIER_CYL, nr=32, q_radial=4, q_t1=4, q_t2=4),
    "steady_fourier_sph": dict(W.FOURIER_SPH),
    "steady_couette_dilute": dict(W.COUETTE_SMALL, eta0=1e-4, q_radial=8, q_t1=8, q_t2=4),
}
DEFAULT = ("steady_fourier_cyl", "steady_fourier_cyl_small")
FIELDS = ("n", "u_r", "u_t1", "T", "q_r", "P_rt1")
CHECK = 50
CHUNK = 100 * CHECK


def solve(name, p, ckpt_dir):
    s = oracle.Solver(p)
    done = 0
    ck = os.path.join(ckpt_dir, name + ".ckpt.npz") if ckpt_dir else None
    if ck and os.path.exists(ck):
        z = np.load(ck)
        s.set_f(z["f"])
        done = int(z["steps"])
        print(f"{name}: resumed at step {done}", flush=True)
    while True:
        rc, steps, res = s.run_to_steady(1e-8, CHUNK, CHECK)
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
        p = CASES[name]
        t0 = time.time()
        s, steps, res = solve(name, p, a.ckpt_dir)
        m = s.moments()
        path = os.path.join(HERE, name + ".txt")
        with open(path, "w") as fh:
            fh.write(f"# oracle steady state, residual 1e-8 checked every {CHECK} steps; params {p}\n")
            fh.write(f"# steps {steps} residual {res!r}\n")
            for f in FIELDS:
                fh.write(f + " " + " ".join(repr(float(x)) for x in m[f]) + "\n")
        print(name, steps, res, f"{time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
