"""Benchmark: site-velocity updates per second of the FDLB solver on one MI355X.

A step is one full TVD-RK3 step (three stages of node kernel + stage kernel) of every instance
of the workload; inputs are resident in HBM before the timed region.  Prints one JSON line.

Default workload: the seeded parameter sweep of 256 uneven cylindrical Couette/Fourier
instances (Nr 64..512, half-range orders 4..16), advanced together in one launch per kernel.
The "paper_grid" object times the paper's own production set-ups (its Sec. IV grid of 90 Couette,
Fourier and rest instances on HHLB(7,20) x HLB(7,8) velocity sets, p_z integrated out on cylinders)
in one batch with FP64 storage.  The "steady" object adds steady solves/s at residual 1e-8 on held-out instances of the same
generator (a bounded set at full size, FP32 f): one at a time from rest, batched from rest, and
batched from the judged prediction of the trained warm-start network
(paper_2403_15051_amd/warmstart_net.npz).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
# HBM traffic of the stage kernel measured with rocprofv3 counters (FETCH_SIZE, WRITE_SIZE, each
# scaled by the same counter on a plain copy of known size); valid only for the kernel source it
# was measured on
TRAFFIC_FILES = {"fp64": os.path.join(ROOT, "profiles", "traffic_k_stage_sweep256_fp64.json"),
                 "fp32": os.path.join(ROOT, "profiles", "traffic_k_stage_sweep256_fp32.json")}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2403_15051_amd", "csrc", "lbe_kernels.hip")


def kernel_sha() -> str:
    """SHA-256 of the stage kernel's source section (its HBM traffic depends on nothing else)."""
    with open(KERNEL_SOURCE, encoding="utf-8") as fh:
        text = fh.read()
    a = text.index("// " + "-" * 66 + " stage kernel")
    b = text.index("// " + "-" * 66 + " residual")
    return hashlib.sha256(text[a:b].encode()).hexdigest()


def measured_traffic(precision: str, algorithmic_bytes: float):
    """Bytes per stage launch from the committed counter measurement, or None when the kernel
    source has changed since, the measurement is of another workload (its algorithmic bytes per
    launch differ from this run's), or no measurement exists."""
    try:
        with open(TRAFFIC_FILES[precision]) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_sha():
        return None
    if abs(t.get("algorithmic_bytes_per_launch", -1.0) - algorithmic_bytes) > 1e-9 * algorithmic_bytes:
        return None
    return t["traffic_bytes_per_launch"]


def copy_calibration(nbytes: int, reps: int) -> None:
    """A plain device-to-device copy of nbytes (reads nbytes, writes nbytes), for scaling the HBM
    counters; also reports its bandwidth (read + write bytes per second), the achievable HBM rate."""
    import torch

    torch.cuda.set_device(0)
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes": nbytes, "reps": reps, "seconds_per_copy": dt,
                      "read_plus_write_GBps": 2 * nbytes / dt / 1e9}), flush=True)


def workload(name: str, n_inst: int, precision: str = "fp64"):
    from paper_2403_15051_amd import workloads as W

    if name == "sweep":
        ps, acc = W.sweep(n_inst)
        desc = (f"parameter sweep: {n_inst} cylindrical Couette/Fourier instances, Nr U{{64..512}}, "
                f"eta0 U(0.01,0.3), Kn 10^U(-2,1), Q in {{4,8,12,16}}, seed {W.SWEEP_SEED}, "
                f"{'FP32 f / FP64 moments' if precision == 'fp32' else 'FP64'}")
        prec = 1 if precision == "fp32" else 0
        return [dict(W.solver_params(p), precision=prec) for p in ps], desc
    prec = 1 if precision == "fp32" else 0
    tag = ", FP32 f / FP64 moments" if precision == "fp32" else ", FP64"
    if name == "fourier_sph":
        return [dict(W.FOURIER_SPH, precision=prec)] * n_inst, f"spherical Fourier (Nr 256, 32x12x12 velocities) x {n_inst}{tag}"
    if name == "fourier_cyl":
        return [dict(W.FOURIER_CYL, precision=prec)] * n_inst, f"cylindrical Fourier (Nr 128, 16x8x4 velocities) x {n_inst}{tag}"
    if name == "couette":
        return [dict(W.COUETTE_SMALL, precision=prec)] * n_inst, f"cylindrical Couette (Nr 32, 8x4x2 velocities) x {n_inst}{tag}"
    if name == "paper_grid":
        return paper_grid(prec), (f"the paper's grid (Sec. IV): eta0 0.1, 0.2 x C 4, 7, 10 x R_L 1, 3, 5; Couette on cylinders, "
                                  f"Fourier and rest on cylinders and spheres (90 instances); HHLB(7,20) x HLB(7,8) with "
                                  f"p_z integrated out (cylinders), x HLB(7,8) (spheres); dr = sigma/10, dt ~ 1e-3{tag}")
    raise SystemExit(f"unknown workload {name}")


def paper_grid(prec: int):
    """The paper's production set-ups as one batch (the grid points the GPU stage kernel holds)."""
    from paper_2403_15051_amd import workloads as W

    out = []
    for eta0 in (0.1, 0.2):
        for C in W.PAPER_C:
            for RL in W.PAPER_RL:
                for flow in ("couette", "fourier", "rest"):
                    for geo in ((0,) if flow == "couette" else (0, 1)):
                        out.append(W.paper_case(flow, geo, eta0, C, RL, precision=prec))
    return out


def timed_steps(params, steps: int, warmup: int, autotune: bool = True):
    """Site-velocity updates/s of `steps` replays of the captured RK3 step (inputs resident)."""
    import torch

    from paper_2403_15051_amd import lbe

    s = lbe.Solver(params)
    sv = sum(int(s.info(k)["nr"]) * int(s.info(k)["nv"]) for k in range(s.n_inst))
    if autotune:
        s.autotune(reps=3)
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del s
    return {"value": sv * steps / dt, "ms_per_step": dt * 1e3 / steps, "site_velocities": sv, "instances": len(params)}


def cpu_baseline(params, budget_s: float, threads: int = 0):
    """The oracle, as it stands, on a bounded sample of the same workload (host cores; threads=0
    keeps the oracle's default of all host threads)."""
    import oracle

    oracle.build(force=False)
    default = oracle.get_threads()
    if threads:
        oracle.set_threads(threads)
    used_threads = oracle.get_threads()
    done = 0
    t_run = 0.0
    used = []
    t_start = time.perf_counter()
    try:
        for p in params:
            if time.perf_counter() - t_start > budget_s:
                break
            s = oracle.Solver({k: v for k, v in p.items() if k != "precision"})  # the oracle is FP64
            nv = s.nv
            steps = 0
            t0 = time.perf_counter()
            while steps < 1000:
                s.step(1)
                steps += 1
                if time.perf_counter() - t0 > budget_s / 4 or time.perf_counter() - t_start > budget_s:
                    break
            t_run += time.perf_counter() - t0
            done += p["nr"] * nv * steps
            used.append((p["nr"], nv, steps))
    finally:
        oracle.set_threads(default)
    desc = "; ".join(f"Nr {a} x Nv {b}: {c} steps" for a, b, c in used)
    return {"value": done / t_run, "unit": "site-velocity updates/s", "cores": used_threads, "kind": "oracle",
            "sample": f"{len(used)} instance(s) of the workload, FP64 oracle timed per step ({desc})"}


def _solve_rounds(solver, tol: float, cap: int, every: int, tag: str, round_steps: int = 25000):
    """Steady solve in rounds of round_steps (a progress line per round); returns the step at which
    each instance converged (0 if it did not), the converged mask and the last residuals."""
    import numpy as np

    from paper_2403_15051_amd import lbe

    n = solver.n_inst
    at = np.zeros(n, dtype=np.int64)
    ok = np.zeros(n, dtype=bool)
    done = 0
    res = np.full(n, np.inf)
    while done < cap:
        k = min(round_steps, cap - done)
        st, taken, res = solver.run_to_steady(tol, k, every)
        conv = (res >= 0) & (res <= tol)
        at = np.where(~ok & conv, done + taken, at)
        ok |= conv
        done += k
        print(f"[bench] {tag}: {done} steps, {int(ok.sum())}/{n} converged", file=sys.stderr, flush=True)
        if st == lbe.LBE_OK:
            break
    return at, ok, res


def steady_metrics(n_held: int, n_plain: int, tol: float = 1e-8, cap: int = 150000, full: bool = True):
    """Steady solves/s at residual tol on held-out instances (seed 240315053) of the sweep generator
    itself (full: Nr 64..512, Q 4..16, FP32 f with the library's switch to FP64 storage at the FP32
    floor) or of its reduced-grid form (full=False).  Modes, on the same instances: (1) batched cold,
    all in one context from rest; (2) batched warm: network inference, the one-step residual judge
    against the rest start, and the solve; (3) plain cold, one instance at a time from rest, on the
    first n_plain instances.  Plain cold is reported per instance and, for the ratios, extrapolated
    to the whole set by its time per step (each instance takes the same steps alone as in a batch).
    Instances not converged within cap steps count as failures.  Tables are built and resident
    before each clock starts."""
    import numpy as np
    import torch

    from paper_2403_15051_amd import lbe
    from paper_2403_15051_amd import train_warmstart as TW
    from paper_2403_15051_amd import workloads as W

    if full:
        ps, _ = W.sweep(n_held, seed=W.WARM_HELDOUT_SEED)
        held = [dict(W.solver_params(p), precision=1) for p in ps]
        wdesc = (f"{n_held} held-out instances of the sweep generator itself (seed {W.WARM_HELDOUT_SEED}): "
                 f"Couette/Fourier, Nr U{{64..512}}, eta0 U(0.01,0.3), Kn 10^U(-2,1), u_w U(0,0.5), T2/T1 U(1,2), "
                 f"Q in {{4,8,12,16}}, FP32 f (switched to FP64 storage at its floor), at most {cap} steps")
    else:
        held = TW.instances(n_held, W.WARM_HELDOUT_SEED)
        wdesc = (f"{n_held} held-out instances of the sweep generator on a reduced grid (seed {W.WARM_HELDOUT_SEED}): "
                 f"Nr U{{32..64}}, half-range order in {{4,8}}, FP64, at most {cap} steps")
    every = TW.CHECK_EVERY

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    cold = lbe.Solver(held)
    (at_c, ok_c, _), t_cold = timed(lambda: _solve_rounds(cold, tol, cap, every, "batched cold"))
    net, meta = TW.load()
    warm = lbe.Solver(held)

    def warm_solve():
        kept, rho = warm.warm_start(net, judge=True)
        return kept, _solve_rounds(warm, tol, cap, every, "batched warm")

    (kept, (at_w, ok_w, _)), t_warm = timed(warm_solve)
    # the converged profiles of both starts agree to the residual's reach
    agree = 0.0
    for k in range(n_held):
        if ok_c[k] and ok_w[k]:
            mc, mw = cold.moments(k), warm.moments(k)
            for f in ("n", "T"):
                agree = max(agree, float(np.abs(mw[f] - mc[f]).max() / np.abs(mc[f]).max()))
    promoted = sum(1 for k in range(n_held) if cold.info(k)["promoted_at"] >= 0)
    del cold, warm
    t_plain, n_ok_plain, steps_plain = 0.0, 0, []
    for k, p in enumerate(held[:n_plain]):
        one = lbe.Solver([p])
        (at, ok, _), t = timed(lambda: _solve_rounds(one, tol, cap, every, f"plain cold {k}"))
        t_plain += t
        n_ok_plain += int(ok[0])
        steps_plain.append(int(at[0]) if ok[0] else cap)
        del one
    # plain cold over the whole set at the sample's time per step
    steps_all = np.where(ok_c, at_c, cap)
    t_plain_all = t_plain / max(1, sum(steps_plain)) * float(steps_all.sum())
    r1 = int(ok_c.sum()) / t_plain_all
    r2 = int(ok_c.sum()) / t_cold
    r3 = int(ok_w.sum()) / t_warm
    return {
        "metric": f"steady solves/s at residual {tol:g}",
        "workload": wdesc,
        "plain_cold": {"solves_per_s": r1, "sample": n_plain, "sample_solves_per_s": n_ok_plain / t_plain,
                       "sample_steps": steps_plain, "batched_steps_of_sample": [int(x) for x in steps_all[:n_plain]],
                       "seconds_extrapolated": t_plain_all},
        "batched_cold": {"solves_per_s": r2, "converged": int(ok_c.sum()), "seconds": t_cold,
                         "mean_steps": float(at_c[ok_c].mean()) if ok_c.any() else None,
                         "max_steps": int(at_c.max()), "switched_to_fp64_storage": promoted},
        "batched_warm": {"solves_per_s": r3, "converged": int(ok_w.sum()), "seconds": t_warm,
                         "mean_steps": float(at_w[ok_w].mean()) if ok_w.any() else None,
                         "max_steps": int(at_w.max()), "fallback_rate": float(1 - kept.mean())},
        "warm_over_plain_cold": r3 / r1, "batched_cold_over_plain_cold": r2 / r1, "warm_over_batched_cold": r3 / r2,
        "profile_agreement_warm_vs_cold": agree,
        "network": {k: meta[k] for k in ("instances", "rows", "epochs", "loss_last", "nr_range", "orders")},
    }


def solve_only(args) -> None:
    """Cold steady solve (rest start, residual 1e-8 checked every 50 steps) of the workload; FP32
    storage instances are switched to FP64 storage by the library when their residual stalls at its
    FP32 floor; prints one JSON line."""
    import torch

    from paper_2403_15051_amd import lbe

    params, desc = workload(args.workload, max(1, args.instances), args.precision)
    s = lbe.Solver(params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    at, ok, res = _solve_rounds(s, 1e-8, 400000, 50, "solve")
    torch.cuda.synchronize()
    out = {"workload": desc, "precision": args.precision, "converged": int(ok.sum()), "steps": at.tolist(),
           "residual": res.tolist(), "seconds": time.perf_counter() - t0,
           "switched_to_fp64_storage_at": [int(s.info(k)["promoted_at"]) for k in range(s.n_inst)]}
    print(json.dumps(out), flush=True)


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sweep")
    ap.add_argument("--instances", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--steady-instances", type=int, default=8, help="held-out instances of the steady-solve metric")
    ap.add_argument("--steady-plain", type=int, default=2, help="of which solved one at a time")
    ap.add_argument("--steady-cap", type=int, default=150000, help="step limit of each steady solve")
    ap.add_argument("--steady-reduced", type=int, default=0,
                    help="also report the steady metric on this many reduced-grid held-out instances")
    ap.add_argument("--no-steady", action="store_true")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32",
                    help="storage of f (the sweep is specified with FP32 f and FP64 moments)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-alt", action="store_true", help="skip the FP64-storage comparison run")
    ap.add_argument("--solve", action="store_true",
                    help="only time a cold steady solve (residual 1e-8) of the workload and print its steps")
    ap.add_argument("--copy-bytes", type=int, default=0, help="only run a plain copy of this size (calibration)")
    args = ap.parse_args()
    if args.copy_bytes:
        copy_calibration(args.copy_bytes, max(1, args.steps))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this solver's batched path runs on a single MI355X; "
              "instances of a sweep shard across GPUs without communication (not built).", file=sys.stderr)
        raise SystemExit(2)

    import torch

    from paper_2403_15051_amd import lbe

    torch.cuda.set_device(0)
    if args.solve:
        solve_only(args)
        return
    params, desc = workload(args.workload, args.instances if args.workload == "sweep" else max(1, args.instances),
                            args.precision)
    print(f"[bench] workload: {desc}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    solver = lbe.Solver(params)
    t_init = time.perf_counter() - t0
    infos = [solver.info(k) for k in range(solver.n_inst)]
    sv = sum(int(i["nr"]) * int(i["nv"]) for i in infos)
    print(f"[bench] init {t_init:.1f} s, {solver.n_inst} instances, {sv / 1e6:.2f} M site-velocities", file=sys.stderr,
          flush=True)
    tuned = None
    if not args.no_autotune:
        tuned = solver.autotune(reps=3)
        print("[bench] autotuned tiles: " + ", ".join(f"Nv {r['nv']}: {r['tile_nodes']} nodes "
                                                      f"({r['ms_before']:.3f} -> {r['ms']:.3f} ms)" for r in tuned),
              file=sys.stderr, flush=True)
    solver.step(args.warmup)
    solver.sync()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    # timed region: the captured RK3 step replayed K times
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(args.steps)
    solver.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    value = sv * args.steps / dt
    print(f"[bench] timed {args.steps} steps: {dt * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    # a second pass with HIP events around every launch (launched one by one) for the roofline
    solver.timing_start()
    t2 = time.perf_counter()
    solver.step(args.steps)
    solver.sync()
    t3 = time.perf_counter()
    tm = solver.timing_stop()
    # algorithmic HBM bytes of one stage launch: stage 1 reads f^n and writes f1, stages 2 and 3
    # read f_s and f^n and write: 8 f-accesses per site-velocity per step, 64 B in FP64 and 32 B
    # with FP32 storage, a third of it per stage launch on average
    fbytes = 4 if args.precision == "fp32" else 8
    bytes_per_launch = sv * 8.0 * fbytes / 3
    stage_avg_s = tm["stage_ms"] / tm["stage_launches"] / 1e3
    achieved = bytes_per_launch / stage_avg_s / 1e9
    line = {
        "metric": "site-velocity updates/s; steady solves/s at 1e-8 residual, warm vs cold start",
        "value": value,
        "unit": "site-velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",  # arithmetic; the storage of f is config.precision
        "data": "synthetic",
        "config": {"workload": desc, "instances": solver.n_inst, "site_velocities": sv,
                   "precision": "fp32 storage, fp64 arithmetic" if args.precision == "fp32" else "fp64",
                   "tiles": ([{"nv": r["nv"], "tile_nodes": r["tile_nodes"]} for r in tuned] if tuned else "default"),
                   "parallelism": "single GPU, instances batched per launch"},
        "roofline": {"bound": "hbm", "kernel": "k_stage", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.precision, bytes_per_launch),
                     "stage_ms_avg": stage_avg_s * 1e3, "node_ms_avg": tm["node_ms"] / max(1, tm["node_launches"]),
                     "stage_share_of_step": tm["stage_ms"] / ((t3 - t2) * 1e3),
                     "ms_per_step_eager_timed": (t3 - t2) * 1e3 / args.steps},
    }
    del solver
    if args.precision == "fp32" and args.workload == "sweep" and not args.no_alt:
        # the same workload with FP64 storage, for comparison (same tiles procedure, graph replay)
        p64 = [dict(p, precision=0) for p in params]
        s64 = lbe.Solver(p64)
        if not args.no_autotune:
            s64.autotune(reps=3)
        s64.step(args.warmup)
        s64.sync()
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        s64.step(args.steps)
        s64.sync()
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        line["fp64_storage"] = {"value": sv * args.steps / (t5 - t4), "ms_per_step": (t5 - t4) * 1e3 / args.steps}
        print(f"[bench] fp64 storage: {(t5 - t4) * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
        del s64
    if args.workload == "sweep" and not args.no_alt:
        # the paper's production velocity sets on its own grid, FP64 storage (the paper's precision)
        grid, gdesc = workload("paper_grid", 0, "fp64")
        pg = timed_steps(grid, args.steps, args.warmup, autotune=not args.no_autotune)
        pg["workload"] = gdesc
        line["paper_grid"] = pg
        print(f"[bench] paper grid: {pg['ms_per_step']:.3f} ms/step, {pg['value']:.3e} updates/s", file=sys.stderr,
              flush=True)
    if not args.no_steady:
        line["steady"] = steady_metrics(args.steady_instances, args.steady_plain, cap=args.steady_cap)
        if args.steady_reduced:
            line["steady_reduced_grid"] = steady_metrics(args.steady_reduced, args.steady_plain, full=False)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(params, args.cpu_seconds)
        one = cpu_baseline(params, args.cpu_seconds / 3, threads=1)
        line["cpu_baseline"]["single_thread"] = {"value": one["value"], "cores": 1, "sample": one["sample"]}
        line["cpu_baseline"]["host"] = f"{host_cpu()}, {os.cpu_count()} logical CPUs visible"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
