"""Benchmark of the SPH neighbour-interaction sweep on one MI355X.

Workload: 128^3 = 2 097 152 particles in the periodic unit cube, jittered cubic
lattice, Wendland C4 kernel with 200 neighbours, ideal gas (the 2M-particle
configuration the pair-rate metric is quoted on).  A timed step is one full
sph_step: kick, drift, tree build, density with the smoothing-length
iteration, EOS, forces, closing kick and FP64 reductions.

value  = pair interactions per second of the whole step for the mixed path:
         (sum_i |G_i| + sum_i |F_i|) counted by the kernels, divided by the
         wall time of the timed steps (tree build and kick included).
Also reported: the same for the FP64 path, the density+force-only rate of
the metric's definition (kernel times from HIP events inside the library),
the roofline of the dominant kernel, the per-field errors of each precision
against the stored FP64 oracle trajectory of the workload (a fresh run of
init + its steps, sampled particles), and the FP64 CPU oracle on a sample
(all threads and one thread).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--small]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Useful (algorithmic) floating-point operations per interaction, counted from
# the formulas of the sweep for the Wendland C4 kernel (FMA counted as 2):
#   density, per gather pair and smoothing-length iteration:
#     x_j - x_i (3), r^2 (5), r (1), q (1), f(q) (10), q f'(q) (6), two sums (5) = 31
#   force, per force-set pair:
#     x_j - x_i (3), r^2 (5), r (1), two kernel gradients 2 x (q 1, g 8, G 2) = 22,
#     v_ij (3), v.x (5), hbar (2), mu (6), viscosity Pi (10), Wbar gradient (2),
#     pair scalar (6), acceleration (6), PdV and heating sums (7), signal speed (1) = 84
FLOP_DENSITY_PAIR = 31
FLOP_FORCE_PAIR = 84
PEAK = {"f64": 78.6e12, "f32": 157.3e12}   # MI355X vector peaks (FP32 figure is the packed one)
PEAK_F32_UNPACKED = 78.6e12   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, without packed FP32
KERNEL_INDEX = {"m4": 0, "wc2": 1, "wc4": 2, "wc6": 3}


def _ngroups(sizes):
    return int(sum((int(k) + 63) // 64 for k in sizes))


def make_workload(name, small=False):
    """Synthetic workloads (sph_inputs); `large` is the one the metric is quoted on."""
    import sph_inputs as si
    if name == "large":
        ns = 64 if small else 128
        c = si.config_large(n_side=ns)
        c["desc"] = f"{ns}^3 jittered lattice, periodic unit cube, Wendland C4, 200 neighbours"
    elif name == "two_phase":
        ns = 64 if small else 128
        c = si.config_two_phase(n_side=ns)
        c["desc"] = f"{ns}^3 two-phase slab (density 10 in 1, shear 0.1), Wendland C4, 200 neighbours"
    elif name == "batch":
        b = si.config_batch(nsets=32 if small else 256)
        keys = b["sets"][0].keys()
        st = {k: np.concatenate([x[k] for x in b["sets"]]) for k in keys}
        offs = np.concatenate([[0], np.cumsum([len(x["x"]) for x in b["sets"]])]).tolist()
        c = {"state": st, "params": b["params"], "set_offsets": offs, "graph": True,
             "desc": f"{len(b['sets'])} independent periodic boxes of 4096-65536 particles, "
                     f"cubic spline, 64 neighbours"}
    elif name == "spheres":
        if small:
            c = si.config_spheres(n1=1_200_000, n2=480_000)
        else:
            c = si.config_spheres()
        c["desc"] = (f"two spheres of {len(c['state']['x'])} particles in vacuum, stiffened gas, "
                     f"Wendland C4, 200 neighbours")
    else:
        raise ValueError(name)
    c["workload"] = name
    c["autotune"] = True   # (the bucket size the library's autotuner picks)
    c["n"] = len(c["state"]["x"])
    offs = c.get("set_offsets") or [0, c["n"]]
    c["ngroups"] = _ngroups(np.diff(offs))
    return c


WORKLOADS = ("large", "two_phase", "batch", "spheres")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


SCHEMES = ("dynamic", "entropy", "evolved", "interface")


def with_scheme(case, schemes):
    """Switch on the optional schemes; the interface correction takes the
    material ids the workload defines (the slab, the second sphere)."""
    if not schemes:
        return case
    case = dict(case, params=dict(case["params"], **{k: True for k in schemes}))
    if "interface" in schemes and "mat" not in case["state"]:
        st = case["state"]
        if case.get("workload") == "two_phase":
            mat = (st["u"] < 0.5).astype(np.float64)
        elif case.get("workload") == "spheres":
            mat = (st["vx"] < 0.0).astype(np.float64)
        else:
            mat = np.zeros(len(st["x"]))
        case["state"] = dict(st, mat=mat)
    return case


def run_gpu(case, precision, steps, warmup, graph=False):
    """Warm up, then time `steps` full steps.  Kernel durations come from HIP
    events the library records on its stream around each sweep kernel, read
    after every timed step (the read synchronises, which the wall time of the
    timed region includes).  With `graph`, one captured step is replayed and
    timed by wall clock; kernel durations then come from the last three eager
    warm-up steps."""
    import torch
    import paper_2511_11425_amd as sph
    p = dict(case["params"], precision=precision)
    P = sph.ParticleArrays.from_state(case["state"], device="cuda:0")
    ctx = sph.Context(p, set_offsets=case.get("set_offsets"))
    ctx.init(P)
    bucket = p.get("bucket", 32)
    if case.get("autotune"):
        bucket = ctx.autotune(P)
    tden, tfor, ttree, ttot, twalk, tdwalk = [], [], [], [], [], []
    for w in range(warmup):
        if graph and w >= warmup - 3:
            # the replayed graph runs the same kernels: their durations are
            # taken from the last eager warm-up steps
            ctx.set_timing(True)
        ctx.step(P)
        if graph and w >= warmup - 3:
            st = ctx.stats()
            tden.append(st["t_density_ms"]); tfor.append(st["t_forces_ms"])
            ttree.append(st["t_tree_ms"]); ttot.append(st["t_total_ms"])
            twalk.append(st["t_force_walk_ms"]); tdwalk.append(st["t_density_walk_ms"])
    ctx.set_timing(False)
    torch.cuda.synchronize()
    if graph:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            ctx.graph_capture_step(P, 0.0, stream=stream)
        torch.cuda.synchronize()
        s0 = ctx.stats()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for _ in range(steps):
                ctx.graph_launch(stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = ctx.stats()
    else:
        ctx.set_timing(True)
        s0 = ctx.stats()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.step(P)
            st = ctx.stats()
            tden.append(st["t_density_ms"]); tfor.append(st["t_forces_ms"])
            ttree.append(st["t_tree_ms"]); ttot.append(st["t_total_ms"])
            twalk.append(st["t_force_walk_ms"]); tdwalk.append(st["t_density_walk_ms"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.set_timing(False)
    pairs = (st["pairs_density_total"] - s0["pairs_density_total"]) + \
            (st["pairs_force_total"] - s0["pairs_force_total"])
    wall = t1 - t0
    res = {
        "precision": precision, "bucket": bucket, "graph": graph,
        "pairs_per_s": pairs / wall,
        "ms_per_step": 1e3 * wall / steps,
        "pairs_density": st["pairs_density"], "pairs_force": st["pairs_force"],
        "cand_density": st["cand_density"], "cand_force": st["cand_force"],
        "nr_scans_mean": st["nr_scans"] / max(1, case["ngroups"]),
        "nr_iter_max": st["nr_iter_max"], "n_noconv": st["n_noconv"],
        "n_overflow": st["n_overflow"],
        "slots_density": st["slots_density"], "slots_force": st["slots_force"],
        "groups_by_level": list(st["groups_by_level"]),
        "launch": {sph.LAUNCH_GROUPS: "groups", sph.LAUNCH_PERSISTENT: "persistent",
                   sph.LAUNCH_WALK: "walk"}[st["launch"]],
        "workgroups_force": st["workgroups_force"],
        "groups_walked": st["groups_walked"],
    }
    if tden:
        res.update({"t_density_ms": float(np.mean(tden)), "t_forces_ms": float(np.mean(tfor)),
                    "t_tree_ms": float(np.mean(ttree)), "t_step_ms": float(np.mean(ttot)),
                    "t_force_walk_ms": float(np.mean(twalk)),
                    "t_density_walk_ms": float(np.mean(tdwalk))})
        # (the sweeps: the walk kernels and the density and force kernels)
        res["metric_rate"] = (st["pairs_density"] + st["pairs_force"]) / \
            (1e-3 * (max(res["t_density_walk_ms"], 0.0) + res["t_density_ms"] +
                     max(res["t_force_walk_ms"], 0.0) + res["t_forces_ms"]))
    ctx.close()
    del P
    torch.cuda.empty_cache()
    return res


GOLDEN = {"large": ("large_fp64_10steps.json", 10), "two_phase": ("two_phase_fp64_3steps.json", 3),
          "spheres": ("spheres_1step.json", 1)}


def errors_vs_oracle(case, precision, bucket, launch):
    """Per-field errors of a fresh run (init + the stored number of global
    steps, this precision) against the FP64 oracle trajectory stored under
    tests/golden for this workload, on its sampled particles: x absolute, v
    relative to max |v|, u rho H relative, a relative to the rms of |a| over
    all particles, du/dt relative to its rms, dt of the last step relative."""
    import torch
    import paper_2511_11425_amd as sph
    if case["workload"] not in GOLDEN or case.get("schemes"):
        return None
    name, steps = GOLDEN[case["workload"]]
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    if g["n"] != case["n"]:
        return None
    rows = np.asarray(g["rows"])
    P = sph.ParticleArrays.from_state(case["state"], device="cuda:0")
    ctx = sph.Context(dict(case["params"], precision=precision, bucket=bucket, launch=launch))
    ctx.init(P)
    for _ in range(steps):
        ctx.step(P)
    st = ctx.stats()
    got = P.numpy()
    ctx.close()
    del P
    torch.cuda.empty_cache()
    fin, rec = g["final"], g["records"][-1]
    out = {"x": max(float(np.max(np.abs(got[k][rows] - np.asarray(fin[k])))) for k in "xyz")}
    vmax = max(float(np.max(np.abs(fin[k]))) for k in ("vx", "vy", "vz"))
    out["v"] = max(float(np.max(np.abs(got[k][rows] - np.asarray(fin[k])))) for k in
                   ("vx", "vy", "vz")) / vmax
    for k in ("u", "rho", "H"):
        ref = np.asarray(fin[k])
        out[k] = float(np.max(np.abs(got[k][rows] - ref) / np.abs(ref)))
    out["a"] = max(float(np.max(np.abs(got[k][rows] - np.asarray(fin[k])))) for k in
                   ("ax", "ay", "az")) / rec["rms_a"]
    out["dudt"] = float(np.max(np.abs(got["dudt"][rows] - np.asarray(fin["dudt"])))) / \
        rec["rms_dudt"]
    out["dt"] = abs(st["dt_used"] - rec["dt"]) / rec["dt"]
    out["reference"] = (f"FP64 oracle, {len(rows)} sampled particles after init and "
                        f"{steps} global step(s) ({name})")
    return out


def traffic_of(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when that summary was taken on a different kernel source or workload."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("workload") != workload:
        return None
    src = os.path.join(ROOT, "paper_2511_11425_amd", "csrc", "sph_sweep.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def cpu_baseline(case, seconds=15.0):
    """The FP64 oracle (as it stands) on a bounded sample of the same workload:
    density (smoothing-length solve) and forces for a random subset of rows,
    sized from a pilot run to take about `seconds` (a batch: its first set)."""
    if case.get("set_offsets"):
        o = case["set_offsets"]
        case = dict(case, state={k: v[o[0]:o[1]] for k, v in case["state"].items()},
                    desc=case["desc"] + " (first set)")
    s = case["state"]
    n = len(s["x"])
    # two pilots separate the fixed cost (the cell list over every particle)
    # from the cost per row; three runs of about seconds / 3 each follow and
    # the median is reported
    r1, r2 = min(n, 20000), min(n, 80000)
    p1 = _oracle_sample(case, r1)
    p2 = _oracle_sample(case, r2) if r2 > r1 else p1
    per_row = max((p2["secs"] - p1["secs"]) / max(r2 - r1, 1), p1["secs"] / r1 * 0.05, 1e-9)
    fixed = max(p1["secs"] - per_row * r1, 0.0)
    rows = int(min(n, max(r1, (seconds / 3 - fixed) / per_row)))
    runs = [_oracle_sample(case, rows, final=True) for _ in range(3)]
    out = sorted(runs, key=lambda r: r["value"])[1]
    # one thread: the same per-row cost on fewer rows (median of 3)
    import oracle
    cores = oracle.num_threads()
    oracle.set_threads(1)
    try:
        rows1 = max(2000, rows // max(cores, 1))
        one = sorted((_oracle_sample(case, rows1, final=True) for _ in range(3)),
                     key=lambda r: r["value"])[1]
    finally:
        oracle.set_threads(cores)
    out["single_thread"] = {"value": one["value"], "cores": 1, "sample": one["sample"]}
    return out


def _oracle_sample(case, nrows, final=False):
    import oracle
    s, p = case["state"], case["params"]
    n = len(s["x"])
    rng = np.random.default_rng(123)
    rows = np.sort(rng.choice(n, size=nrows, replace=False))
    t0 = time.perf_counter()
    d = oracle.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"], rows=rows)
    t1 = time.perf_counter()
    # full-size H/rho/Omega for the force sample: the oracle needs every particle's
    # H; use the initial guess for the others (the force pass cost is the same)
    H = s["H"].copy(); H[rows] = d["H"]
    rho = np.full(n, 1.0); rho[rows] = d["rho"]
    om = np.ones(n); om[rows] = d["omega"]
    Pp, cs = oracle.eos(p, rho, s["u"])
    t2 = time.perf_counter()
    f = oracle.forces(p, s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"], H, rho, om,
                      Pp, cs, rows=rows)
    t3 = time.perf_counter()
    pairs = int(d["count"].sum() + f["count"].sum())
    secs = (t1 - t0) + (t3 - t2)
    if not final:
        return {"rows": rows.size, "secs": secs}
    who = (f"all {n} particles" if rows.size == n else f"{rows.size} random particles of {n}")
    return {"value": pairs / secs, "unit": "pair interactions/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{who} of the workload ({case['desc']}): smoothing-length solve + "
                      f"forces, {pairs} pairs in {secs:.1f} s (cell-list build included), "
                      f"median of 3 runs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-verify", action="store_true",
                    help="skip the per-field errors against the stored oracle trajectory")
    ap.add_argument("--small", action="store_true", help="64^3 instead of 128^3 (quick check)")
    ap.add_argument("--precisions", default="mixed,fp64")
    ap.add_argument("--workload", default="large", choices=list(WORKLOADS))
    ap.add_argument("--graph", action="store_true", help="replay one captured step as a HIP graph")
    ap.add_argument("--bucket", type=int, default=0,
                    help="bucket size 8, 16, 32 or 64 (default: the workload's)")
    ap.add_argument("--launch", default="", choices=["", "groups", "persistent", "walk"],
                    help="sweep launch shape (default: the autotuner's choice)")
    ap.add_argument("--scheme", default="",
                    help="comma list of optional schemes: " + ",".join(SCHEMES))
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device 5 times (calibrates the HBM "
                         "FETCH_SIZE/WRITE_SIZE counters against a known byte count)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        nbytes = args.copy_probe << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the sweep runs on one GPU per process; --gpus must be 1"}))
        sys.exit(2)
    log(f"generating workload {args.workload}")
    schemes = [k for k in args.scheme.split(",") if k]
    for k in schemes:
        if k not in SCHEMES:
            ap.error(f"unknown scheme {k}")
    case = with_scheme(make_workload(args.workload, args.small), schemes)
    case["schemes"] = schemes
    if args.bucket:
        case = dict(case, params=dict(case["params"], bucket=args.bucket), autotune=False)
    if args.launch:
        case = dict(case, params=dict(case["params"], launch=args.launch), autotune=False)
    graph = args.graph or case.get("graph", False)
    results = {}
    for prec in args.precisions.split(","):
        log(f"timing {prec}")
        results[prec] = run_gpu(case, prec, args.steps, args.warmup, graph=graph)
        log(json.dumps(results[prec]))
    head = results.get("mixed") or results[next(iter(results))]
    mixed = head["precision"] == "mixed"
    dtype = "f32" if mixed else "f64"
    roof = None
    if "t_forces_ms" in head:
        # roofline of the dominant kernel of the headline path: algorithmic flops
        # of one launch over its mean duration in the timed steps
        dom = "forces" if head["t_forces_ms"] >= head["t_density_ms"] else "density"
        if dom == "forces":
            flops = head["pairs_force"] * FLOP_FORCE_PAIR
            t = head["t_forces_ms"] * 1e-3
        else:
            flops = head["pairs_density"] * FLOP_DENSITY_PAIR * head["nr_scans_mean"]
            t = head["t_density_ms"] * 1e-3
        kidx = KERNEL_INDEX[case["params"].get("kernel", "m4")]
        # (kernel template: ..., launch mode 0 walking, 1 listed, 2 listed persistent)
        lm = {"walk": 0, "groups": 1, "persistent": 2}[head["launch"]]
        # (forces: no rung maximum; the fifth accumulator unless FP64 without the
        # evolved density in a listed shape)
        ev = "true" if (mixed or lm == 0 or "evolved" in case.get("schemes", [])) else "false"
        kname = f"k_{dom}<{kidx}, {'true' if mixed else 'false'}" + \
            (f", false, {lm}, {ev}>" if dom == "forces" else f", {lm}>")
        achieved = flops / t
        roof = {"bound": "alu", "kernel": kname, "achieved": achieved / 1e12,
                "peak": PEAK[dtype] / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK[dtype],
                "traffic": traffic_of(kname, args.workload if not args.small else None),
                "launch_ms": t * 1e3, "flops_per_launch": flops}
        if mixed:
            roof["peak_unpacked"] = PEAK_F32_UNPACKED / 1e12
            roof["frac_unpacked"] = achieved / PEAK_F32_UNPACKED
    errs = {}
    if not args.no_verify:
        for prec in results:
            log(f"errors against the oracle, {prec}")
            errs[prec] = errors_vs_oracle(case, prec, results[prec]["bucket"],
                                          results[prec]["launch"])
    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(case)
    out = {
        "metric": "pair interactions/sec (density+force) at 2M particles; FP32-mixed vs FP64",
        "workload": args.workload,
        "value": head["pairs_per_s"],
        "unit": "pair interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": case["desc"] + ", full KDK step" +
                   (", mixed precision" if mixed else ", FP64") +
                   (", replayed HIP graph" if graph else ""),
                   "particles": case["n"], "bucket": head["bucket"], "launch": head["launch"],
                   "schemes": schemes,
                   "parallelism": "single GPU"},
        "fp64": {k: results["fp64"].get(k) for k in ("pairs_per_s", "ms_per_step", "metric_rate",
                                                     "t_density_ms", "t_forces_ms")}
        if "fp64" in results else None,
        "mixed_vs_fp64": (results["mixed"]["pairs_per_s"] / results["fp64"]["pairs_per_s"])
        if "mixed" in results and "fp64" in results else None,
        "metric_rate_density_force_only": head.get("metric_rate"),
        "phases_ms": {k: head.get(k) for k in ("t_tree_ms", "t_density_walk_ms", "t_density_ms",
                                               "t_force_walk_ms", "t_forces_ms", "t_step_ms")},
        "pairs": {k: head[k] for k in ("pairs_density", "pairs_force", "cand_density",
                                       "cand_force", "nr_scans_mean", "n_overflow",
                                       "slots_density", "slots_force", "groups_by_level",
                                       "groups_walked")},
        "roofline": roof,
        "errors_vs_oracle": errs or None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
