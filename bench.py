"""Benchmark: preconditioned-OMM solves/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

A step is one complete eigenspace solve through the C ABI: ommSetup (shift,
pole set, sparsifying stencils, assembly and direct factorization of every
P_j), ommSolve (filter X1 = P X0, then preconditioned nonlinear CG with the
exact quartic line search until a stop rule fires) and ommDestroy.  The
orbital block X0 is resident in HBM before the timed region; V (n doubles) is
read from host memory by ommSetup as the C ABI defines.

Kernel classes are timed live with HIP events on the library's stream during
the timed steps (ommSetProfiling); the roofline object reports the class with
the largest total time.  An H.X leg times ommApplyH on one Krylov-sized batch
(all pole x column systems).  The CPU baseline times the oracle on a bounded
sample of the same solve.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    "lattice8_2d_m128_N64": ("lattice_2d", "2D 128x128 grid, N=64, 8x8 jittered Gaussian-well lattice, complex128"),
    "well4_2d_m32_N8": ("small_2d", "2D 32x32 grid, N=8, four random Gaussian wells, complex128"),
}

PEAK_FP64_TFLOPS = 78.6       # 256 CUs x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz (FMA), vector and matrix
PEAK_HBM_GBPS = 8000.0


def load_window(name, inst):
    with open(os.path.join(ROOT, "tests", "golden", "spectra.json")) as f:
        rec = json.load(f)[name]
    import numpy as np
    fp = hashlib.sha256(np.ascontiguousarray(inst.V, dtype=np.float64).tobytes()).hexdigest()[:16]
    if fp != rec["v_sha256_16"]:
        raise SystemExit("stored spectrum does not belong to this potential (fingerprint mismatch)")
    lam = rec["lambda"]
    N = inst.N
    return (float(inst.V.min()), float(lam[N - 1]), float(lam[N])), lam


def roofline_for(profile: dict):
    """Dominant kernel class -> roofline object (algorithmic work / measured time)."""
    name, rec = max(profile.items(), key=lambda kv: kv[1]["ms"])
    secs = rec["ms"] * 1e-3
    if name in ("spp_solve_gemm", "omm_outer", "spp_setup") and rec["flops"] > 0:
        achieved = rec["flops"] / secs / 1e12
        return name, {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                      "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                      "kernel": name, "launches": rec["launches"],
                      "avg_launch_us": 1e3 * rec["ms"] / max(1, rec["launches"])}
    achieved = rec["bytes"] / secs / 1e9
    return name, {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                  "frac": achieved / PEAK_HBM_GBPS, "traffic": None, "kernel": name,
                  "launches": rec["launches"], "avg_launch_us": 1e3 * rec["ms"] / max(1, rec["launches"])}


def hx_leg(pomm, torch, inst, win, systems: int):
    """ommApplyH on `systems` columns, FP64 and FP32: algorithmic GB/s (read X, write HX, read V)."""
    import numpy as np
    opts = pomm.default_options(inner=pomm.INNER_PP, npoles=30)
    h = pomm.Handle(2, inst.m, inst.V, inst.N, win, options=opts)
    out = {}
    n = inst.n
    for name, dt, esz in (("fp64", torch.complex128, 16), ("fp32", torch.complex64, 8)):
        cols = systems if name == "fp32" else min(systems, 30 * inst.N)
        X = torch.randn(cols, n, dtype=dt, device="cuda:0")
        Y = torch.empty_like(X)
        h.apply_h(X, Y)
        torch.cuda.synchronize()
        reps = 5
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            h.apply_h(X, Y)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        gbs = (2.0 * esz * n * cols + (esz // 2) * n) / sec / 1e9
        out[name] = {"columns": cols, "us_per_apply": sec * 1e6, "GB/s": gbs, "frac": gbs / PEAK_HBM_GBPS}
    h.close()
    return out


def cpu_baseline(inst, win, precond_calls: int, seconds_cap: float = 30.0):
    """The oracle's preconditioned solve, timed on a bounded sample and scaled to one solve.

    Sample: the oracle's preconditioner setup for every pole (stencils, sparse P_j,
    SuperLU factorization), then preconditioner applications on single columns
    until the time cap.  One solve = setup + precond_calls x N x (time per column)."""
    from oracle import poles as opoles, solve as osolve
    import numpy as np
    t0 = time.perf_counter()
    opts = osolve.SolveOptions(gmres_rtol=1e-8, filter_rtol=1e-10, npoles=opoles.auto_npoles(*win))
    P = osolve.FermiPreconditioner(2, inst.m, inst.V, *win, opts)
    t_setup = time.perf_counter() - t0
    cols = 0
    t1 = time.perf_counter()
    while True:
        P(inst.X0[:, cols:cols + 1], 1e-8)
        cols += 1
        if time.perf_counter() - t1 > seconds_cap - t_setup or cols >= inst.N:
            break
    t_col = (time.perf_counter() - t1) / cols
    per_solve = t_setup + precond_calls * inst.N * t_col
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "oracle setup for all %d poles (%.1f s) + %d single-column preconditioner "
                      "applications (%.2f s each), scaled to %d applications x %d columns per solve"
                      % (len(P.z), t_setup, cols, t_col, precond_calls, inst.N),
            "seconds_per_solve_estimate": per_solve}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lattice8_2d_m128_N64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU (the solve is not sharded); use --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1603_09724_amd import inputs, pomm

    gen, desc = WORKLOADS[args.workload]
    inst = getattr(inputs, gen)()
    win, lam = load_window(args.workload, inst)
    N = inst.N
    opts = pomm.default_options(filter_rtol=1e-10, gmres_rtol=1e-8, npoles=0)
    dev = torch.device("cuda:0")
    X0 = torch.from_numpy(np.ascontiguousarray(inst.X0.T)).to(dev)
    X = torch.empty_like(X0)
    infos, times, profiles = [], [], []

    def step(profile: bool):
        t = time.perf_counter()
        X.copy_(X0)
        h = pomm.Handle(2, inst.m, inst.V, N, win, options=opts)
        if profile:
            h.set_profiling(True)
        info = h.solve(X)
        info["sigma"] = h.sigma
        info["npoles"] = h.npoles
        if profile:
            profiles.append(h.profile())
        h.close()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        infos.append(info)

    for _ in range(args.warmup):
        step(False)
    times.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = (t1 - t0) / args.steps
    last = infos[-1]
    Estar = 0.5 * sum(l - last["sigma"] for l in lam[:N])
    e_rel = abs(last["energy"] - Estar) / abs(Estar)
    if e_rel > 1e-10:
        print("bench.py: energy error %.3e above 1e-10" % e_rel, file=sys.stderr)
    # aggregate kernel-class profile over the timed steps
    agg = {}
    for prof in profiles:
        for k, v in prof.items():
            a = agg.setdefault(k, {"ms": 0.0, "bytes": 0.0, "flops": 0.0, "launches": 0})
            for f in a:
                a[f] += v[f]
    dom, roof = roofline_for(agg)
    hx = hx_leg(pomm, torch, inst, win, systems=last["npoles"] * N)
    st = sorted(times)
    out = {
        "metric": "preconditioned-OMM solves/s at 1e-10 relative energy error",
        "value": 1.0 / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": inst.n, "N": N,
                   "npoles": last["npoles"], "inner": "sparsifying", "gmres_rtol": 1e-8, "filter_rtol": 1e-10},
        "accuracy": {"energy_rel_err": e_rel, "iters": last["iters"], "stop_rule": last["stop_rule"],
                     "gmres_steps": last["gmres_steps"], "precond_calls": last["precond_calls"]},
        "latency_ms": {"p50": 1e3 * st[len(st) // 2], "p99": 1e3 * st[min(len(st) - 1, math.ceil(0.99 * len(st)) - 1)]},
        "roofline": roof,
        "kernel_classes_ms_per_step": {k: v["ms"] / args.steps for k, v in agg.items()},
        "hx": hx,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, win, int(last["precond_calls"]))
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
