"""Benchmark: one CC global step of the 16384-body Salpeter Plummer workload.

`python bench.py [--steps K] [--warmup W] [--precision fp64|mixed]` runs W
untimed and K timed steps on one GPU and prints one JSON line.  A step is one
global step evolve_cc(all, dt=1/64) (split, recursion into every component,
drift/kick/drift), started each time from the same initial conditions, which
are already resident in HBM.  `value` is algorithmic pair interactions per
second: the pair time steps the splits need (n-1 for a fully connected set,
n(n-1)/2 otherwise) plus the pairs kicked, divided by the wall time per step.

The line also carries an eta scan (`eta_scan`, skipped with --no-eta-scan):
the same workload integrated for four global steps with FP64 and with mixed
precision at several eta, its energy error |dE/E| and wall seconds per N-body
time unit, and for each precision the largest eta that keeps |dE/E| <= 1e-6.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "pair interactions/s; wall-s per N-body time, FP64 vs mixed @ same |dE/E|"
FLOP_TAU = 48      # FP64 operations of one pair time step, eq. 19 (div and sqrt counted as 1)
FLOP_KICK = 26     # FP64 operations of one symmetric pair kick, eqs. 8-9
PEAK_FP64_VECTOR = 78.6e12   # MI355X: 256 CU x 2.4 GHz x 128 FP64 FLOP/clk/CU

# HBM bytes per sweep launch on this workload (rocprofv3 FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0, the factors from a plain 256 MiB device copy; see
# profiles/hbm_traffic_plummer16k_salpeter_fp64.md), valid for the kernel
# sources with this SHA-1; any other source reports null.
SWEEP_TRAFFIC_BYTES = 11286717
SWEEP_TRAFFIC_SOURCES = ("paper_1407_7105_amd/csrc/cc_kernels.hip", "paper_1407_7105_amd/csrc/cc_device.h",
                         "paper_1407_7105_amd/csrc/cc_screen64.h")
SWEEP_TRAFFIC_SHA1 = "791c7299319d7c72a3032b4c96cffdd0f6d1db73"


def sweep_traffic():
    import hashlib
    h = hashlib.sha1()
    for f in SWEEP_TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return SWEEP_TRAFFIC_BYTES if h.hexdigest() == SWEEP_TRAFFIC_SHA1 else None


def cpu_baseline(p, dt, eta):
    """The FP64 oracle on a bounded sample of the same workload (one host
    thread): its breadth-first split of all particles at the pivot steps
    dt, dt/2, ..., dt/128 (the levels where the large component lives) and
    four kicks of every pair (the kick sweep at its full size)."""
    import oracle
    q = p.copy()
    par = oracle.Params(eta=eta)
    evals = pairs = 0
    t0 = time.perf_counter()
    for k in range(8):
        _, _, e = oracle.split_labels(q, dt / 2 ** k, par)
        evals += e
    for _ in range(4):
        pairs += oracle.kick(q, dt, p=par)
    t1 = time.perf_counter()
    return {"value": (evals + pairs) / (t1 - t0), "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle on the same 16384-body state: splits at dt/2^k, k=0..7 ({evals} tau "
                      f"evaluations) and 4 all-pair kicks ({pairs} pairs); {t1 - t0:.1f} s on one host thread"}


def eta_scan(p, wl, dev, small_max, etas=(0.01, 0.03, 0.1, 0.3), steps=4, bound=1e-6):
    """FP64 against mixed precision at equal energy error: each precision is
    run at every eta for `steps` global steps from the same initial conditions;
    |dE/E| comes from the library's compensated diagnostics (eqs. 1-3)."""
    import torch

    from paper_1407_7105_amd import CC_FP64, CC_MIXED, Context, State
    dt = wl["dt"]
    rows = []
    for name, prec in (("fp64", CC_FP64), ("mixed", CC_MIXED)):
        for eta in etas:
            ctx = Context(device=0, eta=eta, eps2=wl["eps2"], precision=prec, small_max=small_max)
            s = State.from_numpy(p, device=dev)
            e0 = ctx.diagnostics(s)["energy"]
            ctx.evolve(s, dt, dt)  # warm-up of this context's buffers, then the timed run from the start
            s = State.from_numpy(p, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.evolve(s, dt, steps * dt)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            e1 = ctx.diagnostics(s)["energy"]
            rows.append({"precision": name, "eta": eta, "dE_over_E": abs((e1 - e0) / e0),
                         "wall_s_per_nbody_time": wall / (steps * dt)})
            print(f"# eta scan {name} eta={eta}: |dE/E|={rows[-1]['dE_over_E']:.3e} "
                  f"{rows[-1]['wall_s_per_nbody_time']:.3f} s per N-body time", file=sys.stderr, flush=True)
    chosen = {}
    for name in ("fp64", "mixed"):
        ok = [r for r in rows if r["precision"] == name and r["dE_over_E"] <= bound]
        chosen[name] = max(ok, key=lambda r: r["eta"]) if ok else None
    ratio = None
    if chosen["fp64"] and chosen["mixed"]:
        ratio = chosen["fp64"]["wall_s_per_nbody_time"] / chosen["mixed"]["wall_s_per_nbody_time"]
    return {"t": steps * dt, "bound": bound, "rows": rows, "chosen": chosen,
            "mixed_speedup_at_equal_dE": ratio}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--small-max", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-eta-scan", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the launch shapes on this workload first (the library defaults are the tuner's "
                         "choice for it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see DESIGN.md for how the "
              "sweep would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1407_7105_amd import CC_FP64, CC_MIXED, Context, State

    wl = synth.WORKLOADS[2]
    dt, eta = wl["dt"], wl["eta"]
    p = synth.workload(2)
    dev = torch.device("cuda:0")
    ic = State.from_numpy(p, device=dev)
    s = ic.copy()
    prec = CC_FP64 if args.precision == "fp64" else CC_MIXED
    ctx = Context(device=0, eta=eta, eps2=wl["eps2"], precision=prec, small_max=args.small_max)

    def step():
        for f in State.FIELDS:
            getattr(s, f).copy_(getattr(ic, f))
        return ctx.evolve(s, dt, dt)

    tune = None
    if args.autotune:
        # launch shapes (on-chip size limit, sweep tiles per workgroup) from
        # the library's autotuner, on this workload, before anything is timed
        tune = ctx.autotune(ic, dt)
        print(f"# autotune: {tune}", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        t = time.perf_counter()
        step()
        print(f"# warmup step {i}: {time.perf_counter() - t:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    work = 0
    t0 = time.perf_counter()
    stats = None
    for _ in range(args.steps):
        stats = step()
        work += stats["tau_pairs_alg"] + stats["kick_pairs"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    print(f"# timed: {args.steps} steps, {ms:.2f} ms/step", file=sys.stderr, flush=True)
    value = work / (t1 - t0)

    roof = None
    fam = None
    if not args.no_roofline:
        # same steps again with every launch bracketed by HIP events on the library's stream
        ctx.timing(True)
        for _ in range(args.steps):
            step()
        fam = ctx.timing_report()
        ctx.timing(False)
        busy = {k: v for k, v in fam.items() if v["launches"]}

        def flops_of(v):
            return FLOP_TAU * v["tau_pairs"] + FLOP_KICK * v["kick_pairs"]

        # the dominant kernel is the family doing most of the step's arithmetic
        # (the sweep); the on-chip components' launches run beside it on a
        # second stream, so their event time overlaps it and is latency, not work
        dom = max(busy, key=lambda k: flops_of(busy[k]))
        d = busy[dom]
        flops = flops_of(d)
        achieved = flops / (d["ms"] * 1e-3) / 1e12 if d["ms"] > 0 else 0.0
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": achieved / (PEAK_FP64_VECTOR / 1e12),
                "traffic": sweep_traffic() if dom == "sweep" else None, "traffic_unit": "bytes per launch",
                "avg_launch_ms": d["ms"] / d["launches"], "launches_per_step": d["launches"] / args.steps}

    scan = None if args.no_eta_scan else eta_scan(p, wl, dev, args.small_max)

    out = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == CC_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "plummer16k_salpeter", "n": p.n, "imf": "salpeter 0.1-100",
                   "eta": eta, "eps": 0.0, "dt": dt, "step": "one CC global step",
                   "launch_shapes": tune},
        "wall_s_per_nbody_time": (ms / 1e3) / dt,
        "stats_per_step": stats,
        "roofline": roof,
        "kernel_ms_per_step": None if fam is None else
        {k: round(v["ms"] / args.steps, 4) for k, v in fam.items() if v["launches"]},
        "eta_scan": scan,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, dt, eta)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
