"""Benchmark: preconditioned-OMM solves/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu] [--legs mixed,...]

Five forms of the solve are timed, each for K steps after W warmup steps: the
mixed-precision form (the headline `value`), the plain FP64 form, the
precomputed-preconditioner form of Section 3.3, the mixed form with fp16
sparse-solve factors, and the mixed form on a spectral window estimated on the
GPU inside every step instead of the stored exact spectrum (under "legs").  A step is one
complete eigenspace solve through the C ABI: ommSetup (shift, pole set,
sparsifying stencils, assembly and direct factorization of every P_j), for the
precomputed form ommPrecompute (the pole expansion applied by GMRES to N + 8
Gaussian columns, then the rank-revealing QR), ommSolve (filter X1 = P X0, then
preconditioned nonlinear CG with the exact quartic line search until a stop rule
fires) and ommDestroy.  The orbital block X0 and the Gaussian block are resident
in HBM before the timed region; V (n doubles) is read from host memory by
ommSetup as the C ABI defines.

Kernel classes are timed live with HIP events on the library's stream: the last
warmup step records every class (the per-class breakdown), the timed steps only
the class with the largest total time (ommSetProfilingClasses), which the
roofline object reports; profiling starts after ommSetup, so the setup is reported
as the median host wall time of that synchronous call (phase_ms_p50, with the window
estimate where a leg runs one).  An H.X leg times ommApplyH on one Krylov-sized batch
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

PEAK_FP64_TFLOPS = 78.6       # dense FP64, matrix cores (= vector FP64 on this chip)
PEAK_FP32_MFMA_TFLOPS = 157.3  # dense FP32 matrix cores
PEAK_HBM_GBPS = 8000.0
PEAK_FP16_MFMA_TFLOPS = 2500.0  # dense FP16 matrix cores

# The two forms of the solve that are timed.  Both stop on the energy-stagnation
# rule and are checked against the exact minimum (stored spectrum) at 1e-10.
#   mixed: complex64 Krylov solves, FFTs and sparse direct solves (left-preconditioned
#          GMRES), complex128 Gram matrices, energy, line search and pole sum;
#   fp64:  everything complex128, GMRES at the paper's tolerance (right-preconditioned).
# Both forms use the paper's 30 poles (Section 4); the FP64 form also its GMRES tolerance.
# The mixed form stops on the left-preconditioned residual (a different quantity) at 5e-4,
# its initial filter at 1e-4.  The timed forms accept GMRES convergence on the Arnoldi
# residual estimate (gmres_verify=0: no recomputed-residual check after a converged cycle)
# and stop at the first line search that leaves the energy unchanged to 8 eps |E| (stall=1);
# every timed solve's energy is checked against the exact minimum.
# mixed_f16 is the mixed form with the sparse solve's factor blocks rounded to fp16.
LEGS = {
    "mixed": dict(precision=1, gmres_rtol=5e-4, filter_rtol=1e-4, npoles=30, gmres_verify=0, stall=1),
    "mixed_f16": dict(precision=1, gmres_rtol=5e-4, filter_rtol=1e-4, npoles=30, spp_products=2, gmres_verify=0,
                      stall=1),
    # the mixed form on a window estimated on the GPU in every step (no stored spectrum)
    "estimated": dict(precision=1, gmres_rtol=5e-4, filter_rtol=1e-4, npoles=30, gmres_verify=0, stall=1),
    "fp64": dict(precision=0, gmres_rtol=1e-5, filter_rtol=1e-5, npoles=30, gmres_verify=0, stall=1),
    # Section 3.3 (Algorithm 2): U U^H precomputed from N + 8 filtered Gaussian columns
    "precomputed": dict(precision=1, gmres_rtol=1e-6, filter_rtol=1e-5, npoles=30, stall=1),
}


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


# legs that precompute the preconditioner: oversampling columns k of the random block
PRECOMPUTE = {"precomputed": 8}
PRECOMPUTE_SEED = 1606
# legs that estimate the spectral window on the GPU inside the step (ommEstimateSpectrum on
# N + k columns) instead of taking it from the stored spectrum
ESTIMATE = {"estimated": 8}
ESTIMATE_SEED = 1607

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spp_gemm_traffic.json")


def measured_traffic(form: str):
    """HBM bytes per launch of the sparse-solve GEMM from the committed counter passes
    (FETCH_SIZE and WRITE_SIZE, calibrated on a copy kernel), or None when no record
    exists for this form, its solve settings differ from the form's (they decide the mix
    of launches), or a source it was taken with has changed since: the kernel, and the
    file that builds its launches (which blocks each launch multiplies)."""
    try:
        with open(TRAFFIC_FILE) as f:
            entry = json.load(f).get(form)
        if not entry or not entry.get("sources") or entry.get("settings") != LEGS.get(form):
            return None
        for rel, want in entry["sources"].items():
            with open(os.path.join(ROOT, rel), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != want:
                    return None
    except (OSError, KeyError, ValueError, AttributeError):
        return None
    return entry["hbm_bytes_per_launch"]


def roofline_for(profile: dict, fp32: bool, form: str, split: int):
    """Dominant kernel class -> roofline object (algorithmic work / measured time).

    The sparse-solve GEMM with split products streams each factor block once at
    128 flops (complex-equivalent) per byte, far above the fp16 matrix rate's balance
    point: it is priced against HBM, with the executed fp16 matrix rate alongside.
    `split`: fp16 products per real product (3: hi/lo factors, 2: fp16 factors, 0: none)."""
    name, rec = max(profile.items(), key=lambda kv: kv[1]["ms"])
    secs = rec["ms"] * 1e-3
    launches = max(1, rec["launches"])
    if name == "spp_solve_gemm" and split:
        achieved = rec["bytes"] / secs / 1e9
        f16 = split * rec["flops"] / secs / 1e12
        return name, {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                      "frac": achieved / PEAK_HBM_GBPS, "traffic": measured_traffic(form),
                      "algorithmic_bytes_per_launch": rec["bytes"] / launches,
                      "flops_per_launch": rec["flops"] / launches,
                      "f16_mfma_tflops": f16, "f16_mfma_frac": f16 / PEAK_FP16_MFMA_TFLOPS,
                      "kernel": name, "dtype": ("split-f16 products" if split == 3 else
                                                "f16 factors, split-f16 right-hand sides") + ", f32 accumulation",
                      "launches": rec["launches"], "avg_launch_us": 1e3 * rec["ms"] / launches}
    if name in ("spp_solve_gemm", "omm_outer", "spp_setup") and rec["flops"] > 0:
        achieved = rec["flops"] / secs / 1e12
        peak = PEAK_FP32_MFMA_TFLOPS if fp32 else PEAK_FP64_TFLOPS
        return name, {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                      "frac": achieved / peak,
                      "traffic": measured_traffic(form) if name == "spp_solve_gemm" else None,
                      "algorithmic_bytes_per_launch": rec["bytes"] / launches,
                      "flops_per_launch": rec["flops"] / launches,
                      "kernel": name, "dtype": "f32" if fp32 else "f64", "launches": rec["launches"],
                      "avg_launch_us": 1e3 * rec["ms"] / launches}
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


def cpu_baseline(inst, win, precond_calls: int, rtol: float, npoles: int, seconds_cap: float = 30.0):
    """The oracle's preconditioned solve, timed on a bounded sample and scaled to one solve.

    Sample: the oracle's preconditioner setup for every pole (stencils, sparse P_j,
    SuperLU factorization), then preconditioner applications on single columns
    until the time cap, on one host thread (BLAS pools limited to 1).
    One solve = setup + precond_calls x N x (time per column)."""
    from oracle import solve as osolve
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        return _cpu_baseline(inst, win, precond_calls, rtol, npoles, seconds_cap, osolve)


def _cpu_baseline(inst, win, precond_calls, rtol, npoles, seconds_cap, osolve):
    t0 = time.perf_counter()
    opts = osolve.SolveOptions(gmres_rtol=rtol, filter_rtol=rtol, npoles=npoles)
    P = osolve.FermiPreconditioner(2, inst.m, inst.V, *win, opts)
    t_setup = time.perf_counter() - t0
    cols = 0
    t1 = time.perf_counter()
    while True:
        P(inst.X0[:, cols:cols + 1], rtol)
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


def run_leg(pomm, torch, inst, win, lam, opts, steps: int, warmup: int, oversample: int | None = None,
            estimate: int | None = None):
    """Time `steps` complete solves (setup + solve + destroy) after `warmup` untimed ones.

    Kernel timing: the last warmup step records every kernel class (the per-class
    breakdown, and the dominant class); the timed steps record only the dominant class,
    so that the event pairs of the other classes do not load the timed region.  With no
    warmup the timed steps record every class."""
    N = inst.N
    dev = torch.device("cuda:0")
    import numpy as np
    X0 = torch.from_numpy(np.ascontiguousarray(inst.X0.T)).to(dev)
    X = torch.empty_like(X0)
    infos, times, profiles = [], [], []
    full = []
    B = None
    if oversample is not None:   # the random block is input data: drawn and uploaded once
        from paper_1603_09724_amd import inputs
        B = torch.from_numpy(np.ascontiguousarray(
            inputs.gaussian_test_block(inst.n, N + oversample, PRECOMPUTE_SEED).T)).to(dev)

    Best = None
    if estimate is not None:   # the start block of the window estimate is input data too
        from paper_1603_09724_amd import inputs
        Best = torch.from_numpy(np.ascontiguousarray(
            inputs.gaussian_test_block(inst.n, N + estimate, ESTIMATE_SEED).T)).to(dev)
    est = {}

    phases = {"estimate": [], "setup": []}   # host wall time of the synchronous calls, per step

    def step(classes):
        t = time.perf_counter()
        X.copy_(X0)
        w = win
        if Best is not None:
            t_e = time.perf_counter()
            e = pomm.estimate_spectrum(2, inst.m, inst.V, N, Best, tol=1e-6)
            phases["estimate"].append(time.perf_counter() - t_e)
            est.update(e)
            w = (e["lo"], e["homo"], e["lumo"])
        t_s = time.perf_counter()
        h = pomm.Handle(2, inst.m, inst.V, N, w, options=opts)   # ommSetup returns when the setup is done
        phases["setup"].append(time.perf_counter() - t_s)
        if classes == "all":
            h.set_profiling(True)
        elif classes:
            h.set_profiling(True, classes=classes)
        if B is not None:
            h.precompute(B)
        info = h.solve(X)
        info["gmres_steps"], info["precond_calls"] = h.counters()   # including any precompute
        info["sigma"] = h.sigma
        info["npoles"] = h.npoles
        prof = h.profile() if classes else None
        h.close()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        infos.append(info)
        return prof

    for i in range(warmup):
        prof = step("all" if i == warmup - 1 else None)
        if prof:
            full.append(prof)
    dominant = max(full[-1].items(), key=lambda kv: kv[1]["ms"])[0] if full else None
    times.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        profiles.append(step([dominant] if dominant else "all"))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    last = infos[-1]
    Estar = 0.5 * sum(l - last["sigma"] for l in lam[:N])
    e_rel = max(abs(i["energy"] - Estar) / abs(Estar) for i in infos[-steps:])

    def aggregate(profs):
        agg = {}
        for prof in profs:
            for k, v in prof.items():
                a = agg.setdefault(k, {"ms": 0.0, "bytes": 0.0, "flops": 0.0, "launches": 0})
                for f in a:
                    a[f] += v[f]
        return agg

    agg = aggregate(profiles)
    breakdown = aggregate(full[-1:]) if full else {k: {f: x / steps for f, x in v.items()} for k, v in agg.items()}
    st = sorted(times)
    med = lambda v: 1e3 * sorted(v)[len(v) // 2] if v else None
    return {"dt": dt, "last": last, "e_rel": e_rel, "agg": agg, "breakdown": breakdown, "estimate": dict(est),
            "phase_ms": {k: med(v[-steps:]) for k, v in phases.items() if v},
            "breakdown_source": "last warmup step, every kernel class recorded" if full else
                                "timed steps, every kernel class recorded",
            "latency_ms": {"p50": 1e3 * st[len(st) // 2],
                           "p99": 1e3 * st[min(len(st) - 1, math.ceil(0.99 * len(st)) - 1)]}}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lattice8_2d_m128_N64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--legs", default="mixed,fp64,precomputed,mixed_f16,estimated",
                    help="solve forms to time (first = headline)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU (the solve is not sharded); use --gpus 1", file=sys.stderr)
        return 2

    import torch

    from paper_1603_09724_amd import inputs, pomm

    gen, desc = WORKLOADS[args.workload]
    inst = getattr(inputs, gen)()
    win, lam = load_window(args.workload, inst)
    N = inst.N
    legs = [l for l in args.legs.split(",") if l]
    res = {}
    for name in legs:
        res[name] = run_leg(pomm, torch, inst, win, lam, pomm.default_options(**LEGS[name]), args.steps, args.warmup,
                            PRECOMPUTE.get(name), ESTIMATE.get(name))
        if res[name]["e_rel"] > 1e-10:
            print("bench.py: %s energy error %.3e above 1e-10" % (name, res[name]["e_rel"]), file=sys.stderr)
    head = legs[0]
    r0 = res[head]
    fp32 = LEGS[head]["precision"] == 1
    products = pomm.default_options(**LEGS[head]).spp_products
    split = 0 if not fp32 else {pomm.PRODUCTS_SPLIT16: 3, pomm.PRODUCTS_F16: 2}.get(products, 0)
    dom, roof = roofline_for(r0["agg"], fp32, head, split)
    hx = hx_leg(pomm, torch, inst, win, systems=r0["last"]["npoles"] * N)

    def leg_summary(name):
        r = res[name]
        settings = dict(LEGS[name])
        if name in PRECOMPUTE:
            settings.update(precompute="Algorithm 2", oversample=PRECOMPUTE[name], random_seed=PRECOMPUTE_SEED)
        if name in ESTIMATE:
            e = r["estimate"]
            settings.update(window="ommEstimateSpectrum in every step", block_extra=ESTIMATE[name],
                            random_seed=ESTIMATE_SEED, estimate_rounds=e.get("iters"),
                            estimate_applies=e.get("applies"), homo=e.get("homo"), lumo=e.get("lumo"))
        return {"value": 1.0 / r["dt"], "ms_per_step": 1e3 * r["dt"], "settings": settings,
                "energy_rel_err": r["e_rel"], "iters": r["last"]["iters"], "stop_rule": r["last"]["stop_rule"],
                "gmres_steps": r["last"]["gmres_steps"], "precond_calls": r["last"]["precond_calls"],
                "latency_ms": r["latency_ms"],
                "phase_ms_p50": r["phase_ms"],
                "kernel_classes_ms_per_step": {k: v["ms"] for k, v in r["breakdown"].items()},
                "kernel_classes_source": r["breakdown_source"]}

    out = {
        "metric": "preconditioned-OMM solves/s at 1e-10 relative energy error",
        "value": 1.0 / r0["dt"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r0["dt"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ({3: "f32+f64, split-f16 sparse-solve products",
                   2: "f32+f64, f16 sparse-solve factors"}.get(split, "f32+f64")) if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": inst.n, "N": N, "form": head,
                   **LEGS[head], "npoles": r0["last"]["npoles"], "inner": "sparsifying"},
        "accuracy": {"energy_rel_err": r0["e_rel"], "iters": r0["last"]["iters"],
                     "stop_rule": r0["last"]["stop_rule"], "gmres_steps": r0["last"]["gmres_steps"],
                     "precond_calls": r0["last"]["precond_calls"]},
        "latency_ms": r0["latency_ms"],
        "phase_ms_p50": r0["phase_ms"],
        "roofline": roof,
        "kernel_classes_ms_per_step": {k: v["ms"] for k, v in r0["breakdown"].items()},
        "kernel_classes_source": r0["breakdown_source"],
        "legs": {name: leg_summary(name) for name in legs},
        "hx": hx,
    }
    if not args.no_cpu:
        ref = "fp64" if "fp64" in res else head
        out["cpu_baseline"] = cpu_baseline(inst, win, int(res[ref]["last"]["precond_calls"]),
                                           LEGS[ref]["gmres_rtol"], int(res[ref]["last"]["npoles"]))
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
