"""Benchmark: CC global steps of the 262 144-body Plummer workload with hard
binaries (Salpeter masses 0.1-100, 10% binaries with a log-uniform in
[1e-5, 1e-3]), FP64, on one GPU.

`python bench.py [--steps K] [--warmup W]` integrates W untimed and then K
timed global steps of evolve_cc(all, dt0) (split, recursion into every
component, drift/kick/drift) from the workload's initial conditions, which
are resident in HBM before the timed region starts.  The global pivot step is
dt0 = 1/512: the top of the power-of-two hierarchy is a free parameter of the
method, and with it one step of this workload is a bounded unit of work
(about 1/8 of a step at 1/64, the same levels below).  `value` is algorithmic
pair interactions per second: the pair time steps the splits need (n-1 for a
fully connected set, n(n-1)/2 otherwise) plus the pairs kicked (label_i !=
label_j), over the wall time of the K steps.

Beside the headline the line carries
  - `roofline`: the sweep (the kernel family with most of the arithmetic),
    from HIP events around each of its launches on the stream it runs on,
    recorded during the timed steps; `roofline_kick` the same for the kick;
  - `conservation`: |dE/E|, |dP| and |dL| over the integrated time;
  - `mixed_force_error`: rms and max relative error of the mixed-precision
    kick against the FP64 kick on every particle of the workload;
  - `eta_scan`: FP64 and mixed precision at several eta from the same initial
    conditions, their |dE/E| and wall seconds per N-body time, and the speed
    ratio at equal |dE/E| <= 1e-6;
  - `secondary`: the 16 384-body Salpeter Plummer workload, one global step
    at dt0 = 1/64 restarted from its initial conditions;
  - `cc_kepler`: the headline workload with two-body components advanced by
    the Kepler flow (CC_KEPLER), same work measure;
  - `batching`: on that workload, the plain FP64 path (every set through the
    grid-wide kernels) against the batched path in FP64 and in mixed
    precision, wall seconds per N-body time at equal |dE/E| <= 1e-6;
  - `paper_softened_plummer`: the paper's softened 1024-body Plummer test,
    first global step, CC against HOLD (counts and time);
  - `cpu_baseline`: the FP64 CPU oracle on a bounded sample of the same state,
    on one host thread and on all host cores of this process.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "pair interactions/s; wall-s per N-body time, FP64 vs mixed @ same |dE/E|"
FLOP_TAU = 54      # FP64 operations of one literal pair time step, eq. 19: 44 + 7 divisions + 3 roots
                   # (division and root counted as 1)
FLOP_KICK = 26     # FP64 operations of one symmetric pair kick, eqs. 8-9
PEAK_FP64_VECTOR = 78.6e12   # MI355X: 256 CU x 2.4 GHz x 128 FP64 FLOP/clk/CU

HEADLINE = 5       # workload index in synth.WORKLOADS
DT0 = 1.0 / 512

# HBM bytes per sweep launch on this workload and step (rocprofv3 FETCH_SIZE
# x 2.0 + WRITE_SIZE x 1.0, the factors from a plain 256 MiB device copy; see
# profiles/hbm_traffic_plummer262k_salpeter_bin10_fp64.md) and the sweep's
# counter-measured FP64 rate (profiles/counters_plummer262k_salpeter_bin10_fp64.md),
# valid for the kernel sources with this SHA-1 only: any other source reports null.
SWEEP_TRAFFIC_BYTES = 5.28e8
SWEEP_COUNTERS = {"fp64_flop_per_pair": 27.6, "valu_instructions_per_pair": 34.6, "valu_issue": 0.83,
                  "achieved_tflops": 25.9, "frac": 25.9 / 78.6,
                  "note": "FP64 add, mul, trans x1 and FMA x2 from SQ_INSTS_VALU_*_F64 x 64 lanes, one step"}
SWEEP_TRAFFIC_SOURCES = ("paper_1407_7105_amd/csrc/cc_kernels.hip", "paper_1407_7105_amd/csrc/cc_device.h",
                         "paper_1407_7105_amd/csrc/cc_screen64.h", "paper_1407_7105_amd/csrc/cc_screen32.h",
                         "paper_1407_7105_amd/csrc/cc_tiles.h", "paper_1407_7105_amd/csrc/cc_kepler.h")
SWEEP_TRAFFIC_SHA1 = "0964edf120be72f801a653ea9a3e36097f8512de"


def sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for f in SWEEP_TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sweep_traffic():
    if SWEEP_TRAFFIC_BYTES is None:
        return None
    return SWEEP_TRAFFIC_BYTES if sources_sha1() == SWEEP_TRAFFIC_SHA1 else None


def sweep_counters():
    return SWEEP_COUNTERS if sources_sha1() == SWEEP_TRAFFIC_SHA1 else None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))   # a GPU's share of the host


# ---------------------------------------------------------------------------
# CPU baseline (the only part of this file that runs the oracle)
# ---------------------------------------------------------------------------
_SAMPLE = {}


def _oracle_share(task):
    """One share of the baseline sample: oracle BFS splits of a random
    subsample of the state at the pivot steps dt0/2^k, and the oracle's pair
    kick sums of a slice of sampled particles against all n."""
    import oracle
    p, dt0, eta = _SAMPLE["p"], _SAMPLE["dt0"], _SAMPLE["eta"]
    seed, nsub, levels, idx = task
    from synth import Particles
    par = oracle.Params(eta=eta)
    rng = np.random.default_rng(seed)
    sub = np.sort(rng.choice(p.n, nsub, replace=False))
    q = Particles(*(np.ascontiguousarray(a[sub]) for a in p.arrays()))   # the subsample, contiguous
    evals = 0
    for k in levels:
        _, e = oracle.split_bfs(q, dt0 / 2 ** k, p=par)
        evals += e
    pairs = 0
    if len(idx):
        oracle.accel(p, np.asarray(idx, np.int64), par)
        pairs = len(idx) * (p.n - 1)
    return evals, pairs


def cpu_baseline(p, dt0, eta, seed=7105):
    """The oracle, as it stands, on a bounded sample of the headline state:
    BFS splits (Sec. 2.3) of 14 000-particle subsamples at dt0/2^k, k = 0..5,
    and all-partner kick sums (eqs. 8-9) of 1024 sampled particles.  Timed on
    one host thread, then the same amount of work split over the host cores
    (one process per core)."""
    import multiprocessing as mp

    _SAMPLE.update(p=p, dt0=dt0, eta=eta)
    rng = np.random.default_rng(seed)
    acc_idx = rng.choice(p.n, 1024, replace=False)
    nsub = 14000
    t0 = time.perf_counter()
    e1, k1 = _oracle_share((seed, nsub, list(range(6)), acc_idx))
    t1 = time.perf_counter()
    single = (e1 + k1) / (t1 - t0)
    out = {"value": single, "unit": "pairs/s", "cores": 1, "kind": "oracle", "cpu": cpu_model(),
           "sample": f"oracle on the headline state (n = {p.n}): BFS splits of a {nsub}-particle random subsample at "
                     f"dt0/2^k, k = 0..5 ({e1} tau evaluations), and all-partner kick sums of 1024 sampled "
                     f"particles ({k1} pairs); {t1 - t0:.1f} s on one host thread"}
    nproc = host_threads()
    if nproc > 1:
        # about the same total work in nproc equal shares: every process splits
        # a subsample of nsub / sqrt(nproc) particles at the six levels (a
        # split costs the square of the set size) and takes 1/nproc of the
        # sampled kick rows
        nsub_w = int(round(nsub / np.sqrt(nproc)))
        tasks = [(seed + 1 + w, nsub_w, list(range(6)), acc_idx[w::nproc]) for w in range(nproc)]
        ctx = mp.get_context("fork")   # no GPU state exists yet in this process
        t0 = time.perf_counter()
        with ctx.Pool(nproc) as pool:
            res = pool.map(_oracle_share, tasks)
        t1 = time.perf_counter()
        e = sum(r[0] for r in res)
        k = sum(r[1] for r in res)
        out["all_cores"] = {"value": (e + k) / (t1 - t0), "unit": "pairs/s", "cores": nproc,
                            "sample": f"{nproc} processes, each splitting a {nsub_w}-particle subsample at the "
                                      f"same six levels and taking 1/{nproc} of the kick rows ({e} tau "
                                      f"evaluations, {k} pairs); {t1 - t0:.1f} s"}
    return out


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------
def roofline_of(fam, name, flop_per_tau, flop_per_kick, traffic=None):
    v = fam.get(name)
    if not v or not v["launches"] or v["ms"] <= 0:
        return None
    flops = flop_per_tau * v["tau_pairs"] + flop_per_kick * v["kick_pairs"]
    achieved = flops / (v["ms"] * 1e-3) / 1e12
    return {"kernel": name, "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR / 1e12,
            "unit": "TFLOP/s", "frac": achieved / (PEAK_FP64_VECTOR / 1e12), "traffic": traffic,
            "traffic_unit": "bytes per launch", "launches": v["launches"], "avg_launch_ms": v["ms"] / v["launches"],
            "flop_per_unit": {"tau_pair": flop_per_tau, "kick_pair": flop_per_kick},
            "units": {"tau_pairs": v["tau_pairs"], "kick_pairs": v["kick_pairs"]}}


def conservation(d0, d1, p):
    ms = p.m
    pscale = float(np.sum(ms * np.sqrt(p.vx ** 2 + p.vy ** 2 + p.vz ** 2)))
    r = np.stack([p.x, p.y, p.z], 1)
    v = np.stack([p.vx, p.vy, p.vz], 1)
    lscale = float(np.sum(ms * np.linalg.norm(np.cross(r, v), axis=1)))
    dP = float(np.linalg.norm(np.asarray(d1["P"]) - np.asarray(d0["P"])))
    dL = float(np.linalg.norm(np.asarray(d1["L"]) - np.asarray(d0["L"])))
    return {"dE_over_E": abs((d1["energy"] - d0["energy"]) / d0["energy"]), "dP": dP, "dP_rel": dP / pscale,
            "dL": dL, "dL_rel": dL / lscale, "E0": d0["energy"], "E1": d1["energy"]}


def mixed_force_error(p, wl, dev):
    """rms and max over all particles of |a_mixed - a_fp64| / |a_fp64|, from
    the library's kick (velocities start at zero, h = 1) in both precisions."""
    import torch

    from paper_1407_7105_amd import CC_FP64, CC_MIXED, Context, State
    acc = {}
    for name, prec in (("fp64", CC_FP64), ("mixed", CC_MIXED)):
        ctx = Context(device=0, eta=wl["eta"], eps2=wl["eps2"], precision=prec)
        s = State.from_numpy(p, device=dev)
        for f in ("vx", "vy", "vz"):
            getattr(s, f).zero_()
        ctx.kick(s, 1.0)
        torch.cuda.synchronize()
        acc[name] = torch.stack([s.vx, s.vy, s.vz], 1)
        ctx.close()
    num = torch.linalg.norm(acc["mixed"] - acc["fp64"], dim=1)
    den = torch.linalg.norm(acc["fp64"], dim=1)
    rel = (num / den).cpu().numpy()
    return {"rms": float(np.sqrt(np.mean(rel ** 2))), "max": float(rel.max()), "median": float(np.median(rel)),
            "particles": int(rel.size), "reference": "the library's FP64 kick (bit-identical to the oracle's sums)"}


def eta_scan(p, wl, dev, dt0, etas=(0.01, 0.03, 0.1), steps=2, bound=1e-6):
    """FP64 against mixed precision at equal energy error: each precision runs
    `steps` global steps at every eta from the same initial conditions;
    |dE/E| from the library's compensated diagnostics (eqs. 1-3)."""
    import torch

    from paper_1407_7105_amd import CC_FP64, CC_MIXED, Context, State
    rows = []
    for name, prec in (("fp64", CC_FP64), ("mixed", CC_MIXED)):
        for eta in etas:
            ctx = Context(device=0, eta=eta, eps2=wl["eps2"], precision=prec)
            s = State.from_numpy(p, device=dev)
            e0 = ctx.diagnostics(s)["energy"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.evolve(s, dt0, steps * dt0)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            e1 = ctx.diagnostics(s)["energy"]
            rows.append({"precision": name, "eta": eta, "dE_over_E": abs((e1 - e0) / e0),
                         "wall_s_per_nbody_time": wall / (steps * dt0), "kick_pairs": st["kick_pairs"],
                         "tau_pairs_alg": st["tau_pairs_alg"]})
            ctx.close()
            print(f"# eta scan {name} eta={eta}: |dE/E|={rows[-1]['dE_over_E']:.3e} "
                  f"{rows[-1]['wall_s_per_nbody_time']:.3f} s per N-body time", file=sys.stderr, flush=True)
    chosen = {}
    for name in ("fp64", "mixed"):
        ok = [r for r in rows if r["precision"] == name and r["dE_over_E"] <= bound]
        chosen[name] = max(ok, key=lambda r: r["eta"]) if ok else None
    ratio = None
    if chosen["fp64"] and chosen["mixed"]:
        ratio = chosen["fp64"]["wall_s_per_nbody_time"] / chosen["mixed"]["wall_s_per_nbody_time"]
    return {"t": steps * dt0, "dt0": dt0, "bound": bound, "rows": rows, "chosen": chosen,
            "mixed_speedup_at_equal_dE": ratio}


def secondary(dev, steps=3):
    """The 16 384-body Salpeter Plummer workload: one global step at dt0 = 1/64,
    restarted from its initial conditions each time."""
    import torch

    import synth
    from paper_1407_7105_amd import Context, State
    wl = synth.WORKLOADS[2]
    p = synth.workload(2)
    ic = State.from_numpy(p, device=dev)
    s = ic.copy()
    ctx = Context(device=0, eta=wl["eta"], eps2=wl["eps2"])

    def step():
        for f in State.FIELDS:
            getattr(s, f).copy_(getattr(ic, f))
        return ctx.evolve(s, wl["dt"], wl["dt"])

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    work = 0
    for _ in range(steps):
        st = step()
        work += st["tau_pairs_alg"] + st["kick_pairs"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.close()
    return {"workload": wl["name"], "n": p.n, "dt0": wl["dt"], "steps": steps,
            "ms_per_step": (t1 - t0) * 1e3 / steps, "value": work / (t1 - t0), "unit": "pairs/s"}


def kepler_leg(p, wl, dev, dt0, steps=3):
    """CC_KEPLER (two-body components by the Kepler flow) on the headline
    workload: one warm-up and `steps` timed global steps from the initial
    conditions, the same work measure as the headline."""
    import torch

    from paper_1407_7105_amd import Context, State
    ctx = Context(device=0, eta=wl["eta"], eps2=wl["eps2"], kepler=1)
    s = State.from_numpy(p, device=dev)
    d0 = ctx.diagnostics(s)
    ctx.evolve(s, dt0, dt0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    work = solves = 0
    for _ in range(steps):
        st = ctx.evolve(s, dt0, dt0)
        work += st["tau_pairs_alg"] + st["kick_pairs"]
        solves += st["kepler_solves"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    d1 = ctx.diagnostics(s)
    ctx.close()
    cons = conservation(d0, d1, p)
    cons["t"] = (steps + 1) * dt0
    print(f"# cc_kepler: {wall * 1e3 / steps:.1f} ms per step, |dE/E| {cons['dE_over_E']:.3e}", file=sys.stderr,
          flush=True)
    return {"ms_per_step": wall * 1e3 / steps, "value": work / wall, "unit": "pairs/s",
            "kepler_solves_per_step": solves / steps, "conservation": cons}


def batching(dev, etas=(0.01, 0.03, 0.1, 0.3), steps=4, bound=1e-6):
    """The batched path against the plain one on the 16 384-body Salpeter
    Plummer workload (dt0 = 1/64, `steps` global steps from its initial
    conditions at each eta): plain FP64 (every set through the grid-wide
    kernels, one level visit at a time), FP64 batched (two-body and small
    components in persistent on-chip launches beside the recursion) and
    mixed precision batched.  Each form's wall seconds per N-body time at the
    largest eta whose |dE/E| <= bound, and the ratios."""
    import torch

    import synth
    from paper_1407_7105_amd import CC_FP64, CC_MIXED, Context, State
    wl = synth.WORKLOADS[2]
    p = synth.workload(2)
    dt0 = wl["dt"]
    forms = (("plain_fp64", dict(plain=1, precision=CC_FP64)), ("batched_fp64", dict(precision=CC_FP64)),
             ("batched_mixed", dict(precision=CC_MIXED)))
    rows = []
    for name, kw in forms:
        for eta in etas:
            ctx = Context(device=0, eta=eta, eps2=wl["eps2"], **kw)
            s = State.from_numpy(p, device=dev)
            e0 = ctx.diagnostics(s)["energy"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.evolve(s, dt0, steps * dt0)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            e1 = ctx.diagnostics(s)["energy"]
            ctx.close()
            rows.append({"form": name, "eta": eta, "dE_over_E": abs((e1 - e0) / e0),
                         "wall_s_per_nbody_time": wall / (steps * dt0), "splits": st["splits"],
                         "max_depth_seen": st["max_depth_seen"]})
            print(f"# batching {name} eta={eta}: |dE/E|={rows[-1]['dE_over_E']:.3e} "
                  f"{rows[-1]['wall_s_per_nbody_time']:.3f} s per N-body time", file=sys.stderr, flush=True)
    chosen = {}
    for name, _ in forms:
        ok = [r for r in rows if r["form"] == name and r["dE_over_E"] <= bound]
        chosen[name] = max(ok, key=lambda r: r["eta"]) if ok else None

    def ratio(a, b):
        if chosen[a] and chosen[b]:
            return chosen[a]["wall_s_per_nbody_time"] / chosen[b]["wall_s_per_nbody_time"]
        return None
    return {"workload": wl["name"], "n": p.n, "dt0": dt0, "t": steps * dt0, "bound": bound, "rows": rows,
            "chosen": chosen, "mixed_batched_speedup_vs_plain_fp64": ratio("plain_fp64", "batched_mixed"),
            "batched_fp64_speedup_vs_plain_fp64": ratio("plain_fp64", "batched_fp64")}


def paper_splits(dev):
    """The paper's softened Plummer test (Sec. 3.1): 1024 equal masses,
    softening 1/256, eta = 0.01, the first global step of 700/512, under the
    CC and HOLD splits: operation counts and GPU wall time of the step."""
    import torch

    import synth
    from paper_1407_7105_amd import Context, State
    p = synth.plummer(1024, 1)
    dt = 700 / 512
    out = {"n": 1024, "eps": 1 / 256, "eta": 0.01, "dt": dt,
           "paper_cc_counts": {"kicks": 1.1e9, "tau_evals": 6.6e8, "drifts": 5.0e6}}
    for name, hold in (("cc", 0), ("hold", 1)):
        best = None
        for _ in range(3):
            ctx = Context(device=0, eta=0.01, eps2=(1 / 256) ** 2, hold=hold)
            s = State.from_numpy(p, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.evolve(s, dt, dt)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ctx.close()
            best = wall if best is None else min(best, wall)
        out[name] = {"ms": best * 1e3, "tau_pairs_alg": st["tau_pairs_alg"], "kick_pairs": st["kick_pairs"],
                     "kicks_both_sides": 2 * st["kick_pairs"], "drifts": st["drifts"],
                     "max_depth_seen": st["max_depth_seen"]}
        print(f"# paper softened Plummer first step, {name}: {best * 1e3:.1f} ms, {st['tau_pairs_alg']} tau, "
              f"{2 * st['kick_pairs']} kicks, {st['drifts']} drifts", file=sys.stderr, flush=True)
    out["hold_over_cc_time"] = out["hold"]["ms"] / out["cc"]["ms"]
    out["hold_over_cc_tau"] = out["hold"]["tau_pairs_alg"] / out["cc"]["tau_pairs_alg"]
    return out


def _run(dev, p, dt0, t_end, **kw):
    """One integration from p's state: (|dE/E|, wall s, stats)."""
    import torch

    from paper_1407_7105_amd import Context, State
    ctx = Context(device=0, **kw)
    s = State.from_numpy(p, device=dev)
    e0 = ctx.diagnostics(s)["energy"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ctx.evolve(s, dt0, t_end)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e1 = ctx.diagnostics(s)["energy"]
    ctx.close()
    return abs((e1 - e0) / e0), wall, st


def repro_eta_scan(dev, etas=(0.003, 0.01, 0.03, 0.1), dt0=1 / 64, t_end=1.0):
    """The paper's second-order test (Sec. 3.1): the softened 1024-body
    Plummer sphere (softening 1/256) for one N-body time at several eta under
    the CC and HOLD splits: |dE/E| (second order in eta) and GPU wall time."""
    import synth
    p = synth.plummer(1024, 1)
    rows = []
    for name, hold in (("cc", 0), ("hold", 1)):
        for eta in etas:
            de, wall, st = _run(dev, p, dt0, t_end, eta=eta, eps2=(1 / 256) ** 2, hold=hold)
            rows.append({"split": name, "eta": eta, "dE_over_E": de, "wall_s": wall,
                         "tau_pairs_alg": st["tau_pairs_alg"], "kick_pairs": st["kick_pairs"]})
            print(f"# repro eta scan {name} eta={eta}: |dE/E|={de:.3e} {wall:.3f} s", file=sys.stderr, flush=True)
    slopes = {}
    for name in ("cc", "hold"):
        r = [x for x in rows if x["split"] == name]
        slopes[name] = [float(np.log(r[k + 1]["dE_over_E"] / r[k]["dE_over_E"]) / np.log(r[k + 1]["eta"] / r[k]["eta"]))
                        for k in range(len(r) - 1)]
    return {"n": 1024, "eps": 1 / 256, "dt0": dt0, "t": t_end, "rows": rows, "slopes": slopes}


def repro_fractal(dev, dims=(1.6, 2.0, 2.6, 3.0), seeds=(1, 2, 3, 4), dt0=1 / 64, t_end=0.25, eta=0.03):
    """The paper's fractal test (Sec. 3.3): 1024 equal-mass bodies in
    Goodwin-Whitworth box fractals of dimension D, virial ratio 1/2, no
    softening, eta = 0.03, integrated for 1/4 N-body time under CC, CC_KEPLER
    and HOLD: mean |dE/E|, GPU wall time and pair steps over the seeds."""
    import synth
    rows = []
    for dim in dims:
        ps = [synth.fractal(1024, 100 * int(10 * dim) + sd, dim=dim) for sd in seeds]
        for name, kw in (("cc", {}), ("cc_kepler", {"kepler": 1}), ("hold", {"hold": 1})):
            des, walls, taus = [], [], []
            for p in ps:
                de, wall, st = _run(dev, p, dt0, t_end, eta=eta, **kw)
                des.append(de)
                walls.append(wall)
                taus.append(st["tau_pairs_alg"])
            rows.append({"dim": dim, "method": name, "dE_over_E_mean": float(np.mean(des)),
                         "wall_s_mean": float(np.mean(walls)), "tau_pairs_alg_mean": float(np.mean(taus))})
            print(f"# repro fractal D={dim} {name}: |dE/E|={rows[-1]['dE_over_E_mean']:.3e} "
                  f"{rows[-1]['wall_s_mean']:.3f} s {rows[-1]['tau_pairs_alg_mean']:.3e} tau", file=sys.stderr,
                  flush=True)
    return {"n": 1024, "eta": eta, "dt0": dt0, "t": t_end, "seeds": list(seeds), "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--dt0", type=float, default=DT0, help="global pivot step (power of two)")
    ap.add_argument("--small-max", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-eta-scan", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-force-error", action="store_true")
    ap.add_argument("--no-batching", action="store_true")
    ap.add_argument("--no-kepler", action="store_true")
    ap.add_argument("--no-paper-splits", action="store_true")
    ap.add_argument("--repro", action="store_true",
                    help="also run the paper's eta scan (Sec. 3.1) and fractal-dimension scan (Sec. 3.3) on the GPU")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the launch shapes on this workload first (the library defaults are the tuner's "
                         "choice on the 16 384-body workload)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import synth
    wl = synth.WORKLOADS[HEADLINE]
    eta = wl["eta"]
    dt0 = args.dt0
    t_gen = time.perf_counter()
    p = synth.workload(HEADLINE)
    print(f"# workload {wl['name']}: n = {p.n}, generated in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)

    base = None
    if not args.no_cpu_baseline:
        # before anything touches the GPU (the all-cores leg forks workers)
        base = cpu_baseline(p, dt0, eta)
        print(f"# cpu baseline: {base['value']:.3e} pairs/s on one thread"
              + (f", {base['all_cores']['value']:.3e} on {base['all_cores']['cores']}" if "all_cores" in base else ""),
              file=sys.stderr, flush=True)

    import torch

    from paper_1407_7105_amd import CC_FP64, CC_MIXED, Context, State

    dev = torch.device("cuda:0")
    prec = CC_FP64 if args.precision == "fp64" else CC_MIXED
    ctx = Context(device=0, eta=eta, eps2=wl["eps2"], precision=prec, small_max=args.small_max)
    s = State.from_numpy(p, device=dev)
    d0 = ctx.diagnostics(s)

    tune = None
    if args.autotune:
        tune = ctx.autotune(s, dt0)
        print(f"# autotune: {tune}", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        t = time.perf_counter()
        ctx.evolve(s, dt0, dt0)
        torch.cuda.synchronize()
        print(f"# warmup step {i}: {time.perf_counter() - t:.3f} s", file=sys.stderr, flush=True)

    # timed steps, with every launch bracketed by HIP events on its own stream
    ctx.timing(True)
    torch.cuda.synchronize()
    work = tau_alg = kick = 0
    totals = {}
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = ctx.evolve(s, dt0, dt0)
        work += st["tau_pairs_alg"] + st["kick_pairs"]
        for k, v in st.items():
            if k not in ("t_reached", "max_depth_seen"):
                totals[k] = totals.get(k, 0) + v
        totals["max_depth_seen"] = max(totals.get("max_depth_seen", 0), st["max_depth_seen"])
        print(f"# timed step {i}: {time.perf_counter() - t0:.3f} s cumulative", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fam = ctx.timing_report()
    ctx.timing(False)
    ms = (t1 - t0) * 1e3 / args.steps
    value = work / (t1 - t0)
    print(f"# timed: {args.steps} steps, {ms:.2f} ms/step, {value:.3e} pairs/s", file=sys.stderr, flush=True)

    d1 = ctx.diagnostics(s)
    cons = conservation(d0, d1, p)
    cons["t"] = (args.warmup + args.steps) * dt0

    roof = roofline_of(fam, "sweep", FLOP_TAU, 0, sweep_traffic())
    if roof is not None:
        roof["counter_measured"] = sweep_counters()
    roof_kick = roofline_of(fam, "kick", 0, FLOP_KICK)
    ctx.close()

    ferr = None if args.no_force_error else mixed_force_error(p, wl, dev)
    scan = None if args.no_eta_scan else eta_scan(p, wl, dev, dt0)
    sec = None if args.no_secondary else secondary(dev)
    kep = None if args.no_kepler else kepler_leg(p, wl, dev, dt0)
    bat = None if args.no_batching else batching(dev)
    pap = None if args.no_paper_splits else paper_splits(dev)
    rep = {"eta_scan": repro_eta_scan(dev), "fractal": repro_fractal(dev)} if args.repro else None

    out = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == CC_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "n": p.n, "imf": "salpeter 0.1-100", "binaries": "10%, a in [1e-5, 1e-3]",
                   "eta": eta, "eps": 0.0, "dt0": dt0, "step": "one CC global step (continuing integration)",
                   "kick_order": "fast", "launch_shapes": tune},
        "wall_s_per_nbody_time": (ms / 1e3) / dt0,
        "stats_timed_steps": totals,
        "roofline": roof,
        "roofline_kick": roof_kick,
        "kernel_ms_per_step": {k: round(v["ms"] / args.steps, 3) for k, v in fam.items() if v["launches"]},
        "conservation": cons,
        "mixed_force_error": ferr,
        "eta_scan": scan,
        "secondary": sec,
        "cc_kepler": kep,
        "batching": bat,
        "paper_softened_plummer": pap,
    }
    if rep is not None:
        out["repro"] = rep
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
