"""Write the converged oracle profiles used by the FP32-storage parity tests.

Calls only the CPU oracle (oracle/): the cylindrical Fourier set-up (R 1..2, T 1 / 1.5, eta0 0.1,
Kn 0.5, Nr 128, half-range order 8, orders 8 and 4), solved to a residual of 1e-8 checked every
50 steps, and a small variant for quick tests.  Output: one text file per case with the step
count, the last residual and the profiles n, u_r, u_t1, T, q_r, P_rt1 (one row per field).

    python tests/golden/make_steady_fixtures.py
"""
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
}
FIELDS = ("n", "u_r", "u_t1", "T", "q_r", "P_rt1")


def main():
    oracle.build(force=False)
    for name, p in CASES.items():
        t0 = time.time()
        s = oracle.Solver(p)
        rc, steps, res = s.run_to_steady(1e-8, 400000, 50)
        assert rc == 0, (name, rc, steps, res)
        m = s.moments()
        path = os.path.join(HERE, name + ".txt")
        with open(path, "w") as fh:
            fh.write(f"# oracle steady state, residual 1e-8 checked every 50 steps; params {p}\n")
            fh.write(f"# steps {steps} residual {res!r}\n")
            for f in FIELDS:
                fh.write(f + " " + " ".join(repr(float(x)) for x in m[f]) + "\n")
        print(name, steps, res, f"{time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
