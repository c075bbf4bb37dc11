"""Train the warm-start network on steady states computed by this solver (needs the GPU).

    python -m paper_2403_15051_amd.train_warmstart [--instances 4096] [--out FILE]

Training instances come from the parameter sweep's generator (geometry flag, eta0, Kn, u_w,
T2/T1 drawn as in the 256-instance sweep, seed 240315052) on a reduced grid and velocity set
(Nr in [32, 64], half-range order 4 or 8), solved together to a residual of 1e-8; every node of
every converged instance is one training row (inputs from lbe_features, targets from
lbe_targets).  The network is trained with its own kernels (BF16 matrix-core products, FP32
accumulation, Adam) and saved with its target standardisation as an .npz of plain arrays.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import lbe
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_FILE = os.path.join(HERE, "warmstart_net.npz")
NR_RANGE = (32, 64)
ORDERS = (4, 8)
TOL = 1e-8
CHECK_EVERY = 50


def instances(n: int, seed: int):
    ps, _ = W.warm_sweep(n, seed, nr_range=NR_RANGE, orders=ORDERS)
    return [W.solver_params(p) for p in ps]


def solve_in_rounds(s: lbe.Solver, tol: float, max_steps: int, log=print, round_steps: int = 20000):
    """Steady solve of every instance in rounds of at most round_steps steps (a line per round).
    Instances already converged re-converge within one check interval of the next round."""
    steps = np.zeros(s.n_inst, dtype=np.int64)
    ok = np.zeros(s.n_inst, dtype=bool)
    done = 0
    while done < max_steps:
        n = min(round_steps, max_steps - done)
        st, taken, res = s.run_to_steady(tol, n, CHECK_EVERY)
        conv = (res >= 0) & (res <= tol)
        steps += np.where(ok, 0, taken)
        ok |= conv
        done += n
        log(f"[train_warmstart]   {done} steps: {int(ok.sum())}/{s.n_inst} converged", flush=True)
        if st == lbe.LBE_OK:
            break
    return steps, ok


def steady_rows(params, tol: float, max_steps: int, chunk: int, log=print):
    """Solve the instances in batches of `chunk`; returns (X, T) device tensors of the rows of the
    converged instances and the step counts."""
    import torch

    xs, ts, all_steps = [], [], []
    for b0 in range(0, len(params), chunk):
        ps = params[b0:b0 + chunk]
        t0 = time.perf_counter()
        s = lbe.Solver(ps)
        steps, ok = solve_in_rounds(s, tol, max_steps, log)
        X, T = s.features(), s.targets()
        rows, r = [], 0
        for k, p in enumerate(ps):
            if ok[k]:
                rows.append(np.arange(r, r + p["nr"]))
            r += p["nr"]
        idx = torch.tensor(np.concatenate(rows), device="cuda")
        xs.append(X[idx])
        ts.append(T[idx])
        all_steps.append(steps)
        log(f"[train_warmstart] solved {b0 + len(ps)}/{len(params)}: {int(ok.sum())} converged, "
            f"max steps {int(steps.max())}, {time.perf_counter() - t0:.1f} s", flush=True)
        del s
    return torch.cat(xs).contiguous(), torch.cat(ts).contiguous(), np.concatenate(all_steps)


def save(path: str, net: lbe.Mlp, meta: dict) -> None:
    mean, scale = net.get_scaling()
    np.savez(path, params=net.get_params(), mean=mean, scale=scale, meta=np.array(json.dumps(meta)))


def load(path: str = DEFAULT_FILE, max_rows: int = 8192) -> tuple[lbe.Mlp, dict]:
    """The saved network on the current device (plain arrays only, nothing executed on load)."""
    with np.load(path, allow_pickle=False) as z:
        net = lbe.Mlp(max_rows=max_rows, gemm=lbe.GEMM_BF16)
        net.set_params(z["params"])
        net.set_scaling(z["mean"], z["scale"])
        meta = json.loads(str(z["meta"]))
    return net, meta


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--chunk", type=int, default=1024)
    ap.add_argument("--max-steps", type=int, default=300000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=DEFAULT_FILE)
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    params = instances(args.instances, W.WARM_TRAIN_SEED)
    t0 = time.perf_counter()
    X, T, steps = steady_rows(params, TOL, args.max_steps, args.chunk)
    t_data = time.perf_counter() - t0
    print(f"[train_warmstart] {X.shape[0]} rows from {int((steps < args.max_steps).sum())} steady states "
          f"in {t_data:.1f} s", flush=True)
    net = lbe.Mlp(max_rows=args.batch, gemm=lbe.GEMM_BF16, seed=W.WARM_TRAIN_SEED)
    t1 = time.perf_counter()
    hist = net.train(X, T, epochs=args.epochs, batch=args.batch, lr=args.lr, seed=W.WARM_TRAIN_SEED)
    t_train = time.perf_counter() - t1
    print(f"[train_warmstart] loss {hist[0]:.4g} -> {hist[-1]:.4g} in {t_train:.1f} s", flush=True)
    meta = {"instances": args.instances, "seed": W.WARM_TRAIN_SEED, "nr_range": NR_RANGE, "orders": ORDERS,
            "tol": TOL, "rows": int(X.shape[0]), "converged": int((steps < args.max_steps).sum()),
            "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "loss_first": float(hist[0]),
            "loss_last": float(hist[-1]), "data_seconds": t_data, "train_seconds": t_train}
    save(args.out, net, meta)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    sys.exit(main())
