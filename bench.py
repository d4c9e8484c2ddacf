"""Benchmark: SSA reaction events per second on one MI355X, with the VALU roofline and the
CPU oracle as a reported baseline.

One step is the whole hot path over one batch of synthetic input: the forward pass
(trajectories, grid alignment, cross-trajectory mean and variance) followed by the
likelihood-ratio backward pass of a squared-error loss on the grid means (re-simulating
the same trajectories).  Both run through the library's persistent work-stealing kernels.
value = forward events per step / step time: the backward's re-simulated events are
reported beside it, never added.

Beside the step, the line reports the batched form against plain launches: the 64 random
networks of the batched workload (5-40 species, 10-120 reactions, 256-16384 trajectories
each, 200-point grids) as one graph-replayed persistent launch, against one plain launch
per network through the same table-driven kernel; the results are checked bit-identical.

Default workload: the 4-species viral network, 10^4 trajectories, t_end = 50, 1000-point
grid; the loss target is the mean of the same network with log rates perturbed by
N(0, 0.1^2) (computed once, outside the timed region).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload viral|differentiated|large]
       [--no-cpu-baseline] [--no-batched] [--copy-calibration]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1007_1768_amd import inputs  # noqa: E402

PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9     # full-rate VALU lane operations per second (MI355X)
HBM_PEAK = 8.0e12

# Algorithmic VALU work per SSA event, in full-rate lane operations (a 32x32->64-bit
# multiply and a reciprocal count 4, as quarter-rate instructions).
W_PHILOX = 10 * (2 * 4 + 2)        # per round: two 32x32->64 products, two 3-way xors
W_UNIFORMS = 2 * 7                 # two 53-bit conversions
W_NEGLOG = 37                      # exponent split, (m-1)/(m+1), 10-term Horner, recombination
W_DIV = 13                         # one IEEE binary64 division (reciprocal + refinement + fixup)
W_ALIGN = 4                        # grid bin of an event time on a uniform grid: scale, ceil, test, convert


def propensity_ops(model):
    reac = np.asarray(model["reac"])
    ops = 0
    for row in reac:
        order = int(row.sum())
        if order == 0:
            ops += 1
        elif order == 1:
            ops += 2
        elif (row == 2).any():
            ops += 5
        else:
            ops += 4
    return ops


def mean_changes(model, n_fired_share=None):
    nu = np.asarray(model["prod"]) - np.asarray(model["reac"])
    per = (nu != 0).sum(axis=1)
    if n_fired_share is None:
        return float(per.mean())
    return float((per * n_fired_share).sum())


def w_forward(model, crossing_frac, changes):
    M = model["reac"].shape[0]
    return (W_PHILOX + W_UNIFORMS + W_NEGLOG + W_DIV + 1 + propensity_ops(model) + (M - 1) + 2 * M
            + changes * 6 + crossing_frac * W_ALIGN)


def w_backward(model, crossings_per_event):
    M, S = model["reac"].shape
    return (W_PHILOX + W_UNIFORMS + W_NEGLOG + W_DIV + 1 + propensity_ops(model) + (M - 1) + 2 * M
            + 4 * M + min(1.0, crossings_per_event) * W_ALIGN + crossings_per_event * (2 * S + 4 * M))


def kernel_sources_hash():
    """FNV-1a 64 over the sources of the network-specialised kernels (the headers they are
    compiled from at run time), to tie stored counter readings of those kernels to the code
    they came from."""
    h = 0xcbf29ce484222325
    d = os.path.join(ROOT, "paper_1007_1768_amd", "csrc")
    for f in ("ssa_device.hpp", "ssa_jit.hpp", "ssa_sim.hpp"):
        for byte in open(os.path.join(d, f), "rb").read():
            h = ((h ^ byte) * 0x100000001b3) & 0xffffffffffffffff
    return "%016x" % h


def stored_traffic(kernel, workload_name):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE summary in profiles/, or None
    when there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.txt" % (kernel, workload_name))
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources_fnv64") != kernel_sources_hash():
        return None
    try:
        return int(float(kv["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def batched_vs_plain(ssa, torch, dev):
    """The batched workload as one graph-replayed launch and as one plain launch per network."""
    nets = inputs.random_networks()
    models = [ssa.Model.from_dict(n) for n in nets]
    grids = [torch.tensor(n["grid"], device=dev) for n in nets]
    means = [torch.empty((len(n["grid"]), n["reac"].shape[1]), dtype=torch.float64, device=dev) for n in nets]
    vars_ = [torch.empty_like(v) for v in means]
    batch = ssa.Batch(models, [n["n_traj"] for n in nets], [n["t_end"] for n in nets], [n["grid"] for n in nets],
                      [n["seed"] for n in nets])
    batch.run(dev, outs=(means, vars_))                       # capture + warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, st = batch.run(dev, outs=(means, vars_), with_stats=True)
    torch.cuda.synchronize()
    batched_s = time.perf_counter() - t0
    # the batch's own autotuner (window sizes timed on this batch), then the tuned replay
    tune = batch.autotune()
    batch.run(dev, outs=(means, vars_))                       # re-capture with the chosen window
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, st_t = batch.run(dev, outs=(means, vars_), with_stats=True)
    torch.cuda.synchronize()
    tuned_s = time.perf_counter() - t0
    saved = os.environ.get("SSA_KERNEL")
    os.environ["SSA_KERNEL"] = "generic"                      # the batched kernel's code path
    identical = True
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain = [ssa.run_device(models[b], n["n_traj"], n["t_end"], grids[b], n["seed"])[:2]
                 for b, n in enumerate(nets)]
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - t0
        for b, (pm, pv) in enumerate(plain):
            identical &= bool(torch.equal(pm, means[b]) and torch.equal(pv, vars_[b]))
    finally:
        if saved is None:
            os.environ.pop("SSA_KERNEL", None)
        else:
            os.environ["SSA_KERNEL"] = saved
    batch.close()
    for mo in models:
        mo.close()
    return {"workload": "64 random networks, 5-40 species, 10-120 reactions, %d trajectories, 200-point grids"
                        % sum(n["n_traj"] for n in nets),
            "events": st["events"], "batched_ms": round(batched_s * 1e3, 3), "plain_ms": round(plain_s * 1e3, 3),
            "batched_events_per_s": round(st["events"] / batched_s, 1),
            "speedup": round(plain_s / batched_s, 3), "identical": identical,
            "tuned": {"win_bytes": tune["win_bytes"], "batched_ms": round(tuned_s * 1e3, 3),
                      "events": st_t["events"], "speedup": round(plain_s / tuned_s, 3)}}


def wide_sweep(ssa, torch, dev):
    """Networks with many reactions: the sequential order (one trajectory per lane) against
    the 64-chunk order (one trajectory per wave), and above 512 reactions the 64-chunk
    kernel with its dependency-graph update against full re-evaluation.  Forward
    (mean/variance) kernel time, best of two launches, t_end 0.5, 50-point grid, seed 9."""
    def run(m, N):
        grid = torch.tensor(inputs.uniform_grid(0.5, 50), dtype=torch.float64, device=dev)
        model = ssa.Model.from_dict(m)
        best = None
        try:
            for _ in range(2):
                _, _, _, st = ssa.run_device(model, N, 0.5, grid, 9, with_stats=True)
                torch.cuda.synchronize()
                if best is None or st["kernel_ms"] < best["kernel_ms"]:
                    best = st
        except ssa.SSAError as e:
            return {"error": str(e).split(":")[0]}
        finally:
            model.close()
        return {"events": best["events"], "kernel_ms": round(best["kernel_ms"], 3),
                "events_per_s": round(best["events"] / best["kernel_ms"] * 1e3, 1)}

    old = os.environ.get("SSA_WIDE_DEPG")
    rows = []
    try:
        for M in (32, 64, 128, 256, 512, 1024, 2048, 4096):
            S = min(48, M // 2)
            base = inputs.wide_network(M, S=S)
            for N in (1024, 16384, 131072):
                if M >= 2048 and N > 16384:
                    continue
                for order in ("seq", "block64"):
                    m = dict(base)
                    m["sum_order"] = order
                    variants = [("-", None)] if (order == "seq" or M <= 512) else [("depg", "1"), ("full", "0")]
                    for vname, env in variants:
                        if env is not None:
                            os.environ["SSA_WIDE_DEPG"] = env
                        rows.append(dict(set="few_species", M=M, S=S, N=N, order=order, update=vname, **run(m, N)))
        for M in (600, 1024, 2048, 4096):
            m = inputs.wide_network(M)
            for N in (1024, 16384, 65536):
                for vname, env in (("depg", "1"), ("full", "0")):
                    os.environ["SSA_WIDE_DEPG"] = env
                    rows.append(dict(set="sparse", M=M, S=int(m["reac"].shape[1]), N=N, order="block64",
                                     update=vname, **run(m, N)))
    finally:
        if old is None:
            os.environ.pop("SSA_WIDE_DEPG", None)
        else:
            os.environ["SSA_WIDE_DEPG"] = old
    return rows


def adaptive_measure(ssa, torch, dev, reps=3, workload="viral"):
    """Adaptive selective memory on a workload's network (viral: 10^4 trajectories; large:
    10^6, taken in epochs of bounded memory), t_end 50, groups of k = N Avg-Y points:
    whole-call device time (event-log passes, sorts, moments, group averages), best of
    reps, and the sizes."""
    w = inputs.WORKLOADS[workload]
    m = w["model"]()
    N, t_end, seed = w["n_traj"], w["t_end"], w["seed"]
    model = ssa.Model.from_dict(m)
    best, best_wall = None, float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        out = ssa.adaptive_device(model, N, t_end, seed, N, with_stats=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - a0
        best_wall = min(best_wall, wall)        # the first call also compiles the network's kernels
        st = out["stats"]
        if best is None or st["kernel_ms"] < best["kernel_ms"]:
            best = dict(st, P=int(out["xy_time"].shape[0]))
    best["wall_ms"] = 1e3 * best_wall
    model.close()
    return {"workload": "%s: %d trajectories, t_end %g, Avg-XY groups of %d points" % (workload, N, t_end, N),
            "events": best["events"], "avg_xy_points": best["P"], "device_ms": round(best["kernel_ms"], 3),
            "wall_ms_with_size_query": round(best["wall_ms"], 3),
            "events_per_s": round(best["events"] / best["kernel_ms"] * 1e3, 1)}


def hiv_stress(ssa, torch, dev, N=16384, t_end=5.0, G=101, seed=7, reps=2):
    """The HIV network of Table 1 (27 reactions, bursts of 200 virions, F-dependent
    infectivities) as a long-trajectory stress case: forward mean/variance of N
    trajectories over t_end days on a G-point grid; kernel time, best of reps."""
    m = inputs.hiv()
    model = ssa.Model.from_dict(m)
    grid = torch.tensor(inputs.uniform_grid(t_end, G), dtype=torch.float64, device=dev)
    best = None
    for _ in range(reps):
        _, _, _, st = ssa.run_device(model, N, t_end, grid, seed, with_stats=True)
        torch.cuda.synchronize()
        if best is None or st["kernel_ms"] < best["kernel_ms"]:
            best = st
    model.close()
    return {"workload": "hiv: %d trajectories, t_end %g days, %d-point grid" % (N, t_end, G),
            "events": best["events"], "max_steps": best["max_steps"], "kernel_ms": round(best["kernel_ms"], 3),
            "events_per_s": round(best["events"] / best["kernel_ms"] * 1e3, 1)}


def throughput_case(ssa, torch, dev, name="large", steps=3, warmup=1):
    """The same step (forward mean/var + LR backward) on a workload that fills the chip
    (large: 10^6 trajectories, 10^4-point grid, histogram): kernel times and the
    roofline fraction of both kernels, for comparison with the latency-bound default."""
    m, w = workload(name)
    N, t_end, G, seed = w["n_traj"], w["t_end"], w["G"], w["seed"]
    grid = torch.tensor(inputs.uniform_grid(t_end, G), dtype=torch.float64, device=dev)
    model = ssa.Model.from_dict(m)
    hist = w.get("hist")
    prates = torch.tensor(inputs.perturbed_rates(m, w.get("perturb_seed", 404)), device=dev)
    target, _, _, _ = ssa.run_device(model, N, t_end, grid, w.get("target_seed", 44), rates=prates)
    fw, bw = [], []
    for i in range(warmup + steps):
        mean, var, _, sf = ssa.run_device(model, N, t_end, grid, seed, hist=hist, with_stats=True)
        _, sb = ssa.backward_device(model, N, t_end, grid, seed, 2.0 * (mean - target), mean, with_stats=True)
        if i >= warmup:
            fw.append(sf["kernel_ms"])
            bw.append(sb["kernel_ms"])
    torch.cuda.synchronize()
    model.close()
    S = m["reac"].shape[1]
    crossings = G * N / max(sf["events"], 1)
    f_ms, b_ms = float(np.mean(fw)), float(np.mean(bw))
    f_ops = w_forward(m, min(1.0, crossings), mean_changes(m)) * sf["events"] / (f_ms * 1e-3)
    b_ops = w_backward(m, crossings) * sf["events"] / (b_ms * 1e-3)
    return {"workload": "%s: %d trajectories, t_end %g, %d-point grid%s, forward mean/var + LR backward"
                        % (name, N, t_end, G, ", histogram" if hist else ""),
            "events": sf["events"], "fwd_kernel_ms": round(f_ms, 3), "bwd_kernel_ms": round(b_ms, 3),
            "events_per_s": round(sf["events"] / ((f_ms + b_ms) * 1e-3), 1),
            "fwd_valu_frac": round(f_ops / PEAK_LANE_OPS, 4), "bwd_valu_frac": round(b_ops / PEAK_LANE_OPS, 4)}


def workload(name):
    w = dict(inputs.WORKLOADS[name])
    m = w["model"]()
    return m, w


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="viral", choices=["viral", "differentiated", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched / plain comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for HBM counter calibration)")
    ap.add_argument("--wide-sweep", action="store_true",
                    help="only run the many-reaction sweep (sum orders, dependency graph) and print it")
    ap.add_argument("--adaptive", action="store_true",
                    help="only time the adaptive selective memory on the viral workload and print it")
    ap.add_argument("--adaptive-large", action="store_true",
                    help="only time the adaptive selective memory at 10^6 trajectories (epochs) and print it")
    ap.add_argument("--hiv", action="store_true",
                    help="only run the HIV network stress case (forward) and print it")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path; trajectory "
              "ranges would shard across GPUs with one all-reduce of the exact integer sums",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1007_1768_amd import ssa

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        n = (1 << 30) // 8
        x = torch.ones(n, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}))
        return
    if args.adaptive_large:
        print(json.dumps({"adaptive": adaptive_measure(ssa, torch, dev, reps=1, workload="large")}), flush=True)
        return
    if args.hiv:
        print(json.dumps({"hiv": hiv_stress(ssa, torch, dev)}), flush=True)
        return
    if args.adaptive:
        print(json.dumps({"adaptive": adaptive_measure(ssa, torch, dev)}), flush=True)
        return
    if args.wide_sweep:
        print(json.dumps({"sweep": "wide networks, forward events/s", "rows": wide_sweep(ssa, torch, dev)}),
              flush=True)
        return

    m, w = workload(args.workload)
    N, t_end, G, seed = w["n_traj"], w["t_end"], w["G"], w["seed"]
    grid_np = inputs.uniform_grid(t_end, G)
    grid = torch.tensor(grid_np, dtype=torch.float64, device=dev)
    model = ssa.Model.from_dict(m)
    hist = w.get("hist")
    stream = torch.cuda.current_stream()

    # target of the loss: the same network with perturbed log rates (untimed)
    prates = torch.tensor(inputs.perturbed_rates(m, w.get("perturb_seed", 404)), device=dev)
    target, _, _, _ = ssa.run_device(model, N, t_end, grid, w.get("target_seed", 44), rates=prates)
    torch.cuda.synchronize()

    S, M = m["reac"].shape[1], m["reac"].shape[0]
    mean = torch.empty((G, S), dtype=torch.float64, device=dev)
    var = torch.empty_like(mean)
    hbuf = torch.empty((G, hist[3]), dtype=torch.int32, device=dev) if hist else None
    gbuf = torch.empty(M, dtype=torch.float64, device=dev)

    def step(with_stats):
        _, _, _, sf = ssa.run_device(model, N, t_end, grid, seed, hist=hist, out=(mean, var, hbuf),
                                     with_stats=with_stats)
        wts = 2.0 * (mean - target)
        _, sb = ssa.backward_device(model, N, t_end, grid, seed, wts, mean, out=gbuf, with_stats=with_stats)
        return sf, sb

    # warm-up with statistics: event counts (the same every step), status checks and the
    # kernels' own times
    fwd_ms, bwd_ms = [], []
    stats_f = stats_b = None
    for _ in range(max(args.warmup, 3)):
        stats_f, stats_b = step(True)
        assert stats_f["flags"] == 0 and stats_b["flags"] == 0, (stats_f, stats_b)
        fwd_ms.append(stats_f["kernel_ms"])
        bwd_ms.append(stats_b["kernel_ms"])
    fwd_ms, bwd_ms = fwd_ms[-3:], bwd_ms[-3:]
    torch.cuda.synchronize()

    # timed steps: the calls are asynchronous on the stream (no statistics, so no host wait
    # inside a step), as a training loop issues them
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step(False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = e0.elapsed_time(e1) / args.steps
    events = args.steps * (stats_f["events"] + stats_b["events"])
    value = stats_f["events"] / (step_ms * 1e-3)

    # forward-only timing (same kernels, no backward, issued like the steps), for the
    # grad / plain ratio
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    f0.record(stream)
    for _ in range(args.steps):
        ssa.run_device(model, N, t_end, grid, seed, hist=hist, out=(mean, var, hbuf))
    f1.record(stream)
    torch.cuda.synchronize()
    fwd_only_ms = f0.elapsed_time(f1) / args.steps

    # roofline of the dominant kernel (algorithmic lane-ops per launch / mean launch time)
    crossings = G * N / max(stats_f["events"], 1)                 # grid points passed per event
    cross_frac = min(1.0, crossings)
    changes = mean_changes(m)
    fwd_avg = float(np.mean(fwd_ms))
    bwd_avg = float(np.mean(bwd_ms))
    jit = os.environ.get("SSA_KERNEL") != "generic" and M <= 32 and S <= 64
    # the kernels the library picks by work items (64 trajectories each) per CU: up to 2,
    # two-wave blocks (a drawing wave beside each simulating one); up to 8, the backward in
    # generations; beyond, the refilling backward
    items_per_cu = ((N + 63) // 64) / torch.cuda.get_device_properties(0).multi_processor_count
    if bwd_avg >= fwd_avg:
        kname = (("ssa_jit_bwd_pc" if items_per_cu <= 2 else "ssa_jit_bwd_gen" if items_per_cu <= 8
                  else "ssa_jit_bwd") if jit else "sim_kernel_bwd")
        kms, wop = bwd_avg, w_backward(m, crossings)
    else:
        kname = ((("ssa_jit_fwd_hist_pc" if hist else "ssa_jit_fwd_pc") if items_per_cu <= 2
                  else "ssa_jit_fwd_atomic") if jit else "fwd_kernel")
        kms, wop = fwd_avg, w_forward(m, cross_frac, changes)
    achieved = wop * stats_f["events"] / (kms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(PEAK_LANE_OPS / 1e12, 3),
                "unit": "Tlane-op/s", "frac": round(achieved * 1e12 / PEAK_LANE_OPS, 5),
                "traffic": stored_traffic(kname, args.workload),
                "kernel": kname, "kernel_ms": round(kms, 4), "ops_per_event": round(wop, 1)}

    out = {
        "metric": "SSA reaction events/sec on 1 MI355X (+ % VALU roofline); batched & grad vs plain",
        "value": round(value, 1),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+i32",
        "data": "synthetic",
        "config": {"workload": "%s: %d trajectories, t_end %g, %d-point grid, forward mean/var + LR backward"
                               % (args.workload, N, t_end, G),
                   "n_traj": N, "grid_points": G, "t_end": t_end, "species": S, "reactions": M,
                   "histogram": list(hist) if hist else None},
        "fwd_events_per_step": stats_f["events"],
        "bwd_events_per_step": stats_b["events"],
        "fwd_kernel_ms": round(fwd_avg, 4),
        "bwd_kernel_ms": round(bwd_avg, 4),
        "fwd_only_ms": round(fwd_only_ms, 4),
        "grad_vs_plain": round(step_ms / fwd_only_ms, 3),
        "wall_s": round(wall, 3),
        "roofline": roofline,
    }

    if not args.no_batched:
        out["batched_vs_plain"] = batched_vs_plain(ssa, torch, dev)
        # the other forms, each timed on its own workload (see --adaptive, --hiv)
        out["throughput_case"] = throughput_case(ssa, torch, dev)
        out["adaptive_memory"] = adaptive_measure(ssa, torch, dev)
        out["hiv_stress"] = hiv_stress(ssa, torch, dev)

    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        thr = orc.default_threads()
        # bounded sample of the same workload: a slice of its trajectories (forward + gradient,
        # as in a step), repeated until at least 10 s of oracle time have passed
        n_cpu = min(N, int(os.environ.get("BENCH_CPU_TRAJ", str(min(N, 20000)))))
        tw = target.cpu().numpy()
        cpu_events, reps = 0, 0
        a0 = time.perf_counter()
        while True:
            st, ref = orc.run(m, n_cpu, t_end, grid_np, seed, hist=hist, threads=thr)
            st2, g, _ = orc.grad(m, n_cpu, t_end, grid_np, seed, 2.0 * (ref["mean"] - tw), ref["mean"],
                                 threads=thr)
            cpu_events += ref["events"]
            reps += 1
            if time.perf_counter() - a0 >= 10.0:
                break
        cpu_s = time.perf_counter() - a0
        out["cpu_baseline"] = {"value": round(cpu_events / cpu_s, 1), "unit": "events/s", "cores": thr,
                               "kind": "oracle",
                               "sample": "%d x (trajectories 0..%d of %d, forward + gradient), %.1f s"
                                         % (reps, n_cpu - 1, N, cpu_s)}
    print(json.dumps(out), flush=True)
    model.close()


if __name__ == "__main__":
    main()
