"""Benchmark: SSA reaction events per second on one MI355X, with the VALU roofline and the
CPU oracle as a reported baseline.

One step is the whole hot path over one batch of synthetic input: the forward pass
(trajectories, grid alignment, cross-trajectory mean, variance and histogram) followed by
the likelihood-ratio backward pass of a squared-error loss on the grid means
(re-simulating the same trajectories).  value = forward events per step / step time, the
step (everything both calls launch and the loss weights between them) captured once as a
HIP graph and replayed K times, timed with HIP events on the replay stream; the replays
must equal the eager step bit for bit.  K eager steps with statistics, timed in the same
run, give the kernel times, launch forms and the roofline.  The backward's re-simulated
events are reported beside the value, never added.

Default workload (large): the 4-species viral network, 10^6 trajectories, t_end = 50,
10^4-point grid, 64-bin histogram of I at every grid point, gradient enabled; the loss
target is the mean of the same network with log rates perturbed by N(0, 0.1^2) (computed
once, outside the timed region).  The line also carries the same step on the viral
workload (10^4 trajectories, 1000-point grid: a launch too small to fill the chip), the
batched form against each network's plain launch, the adaptive selective memory, the HIV
network stress case and the oracle on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large|viral|differentiated]
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
    """The forward event's work, the score update of every reaction (4 per reaction:
    compare, select, product, add) and, per grid point the interval crosses, the
    contraction of the S centred states with the M scores (S x M lane operations)."""
    M, S = model["reac"].shape
    return (W_PHILOX + W_UNIFORMS + W_NEGLOG + W_DIV + 1 + propensity_ops(model) + (M - 1) + 2 * M
            + 4 * M + min(1.0, crossings_per_event) * W_ALIGN + crossings_per_event * S * M)


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


def _median_ms(torch, stream, fn, reps):
    """Median over reps of fn()'s device time, HIP events on stream around each call."""
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def batched_vs_plain(ssa, torch, dev, replays=20, plain_passes=3):
    """The batched workload as one graph-replayed launch (median of `replays` replays)
    against one plain launch per network, each through that network's default kernel
    (median of `plain_passes` passes over the 64 networks); the results must be equal bit
    for bit."""
    nets = inputs.random_networks()
    models = [ssa.Model.from_dict(n) for n in nets]
    grids = [torch.tensor(n["grid"], device=dev) for n in nets]
    means = [torch.empty((len(n["grid"]), n["reac"].shape[1]), dtype=torch.float64, device=dev) for n in nets]
    vars_ = [torch.empty_like(v) for v in means]
    stream = torch.cuda.current_stream()
    batch = ssa.Batch(models, [n["n_traj"] for n in nets], [n["t_end"] for n in nets], [n["grid"] for n in nets],
                      [n["seed"] for n in nets])
    _, _, st = batch.run(dev, outs=(means, vars_), with_stats=True)   # capture, warm-up, event count
    for _ in range(2):
        batch.run(dev, outs=(means, vars_))
    batched_ms = _median_ms(torch, stream, lambda: batch.run(dev, outs=(means, vars_)), replays)
    # the batch's own autotuner (window sizes timed on this batch), then the tuned replays
    tune = batch.autotune()
    batch.run(dev, outs=(means, vars_))                       # re-capture with the chosen window
    tuned_ms = _median_ms(torch, stream, lambda: batch.run(dev, outs=(means, vars_)), replays)
    torch.cuda.synchronize()
    outs = [(torch.empty_like(means[b]), torch.empty_like(vars_[b])) for b in range(len(nets))]

    def plain_pass():
        for b, n in enumerate(nets):
            ssa.run_device(models[b], n["n_traj"], n["t_end"], grids[b], n["seed"], out=(outs[b][0], outs[b][1], None))

    plain_pass()                                              # compiles the specialised kernels
    plain_ms = _median_ms(torch, stream, plain_pass, plain_passes)
    identical = all(bool(torch.equal(outs[b][0], means[b]) and torch.equal(outs[b][1], vars_[b]))
                    for b in range(len(nets)))
    batch.close()
    for mo in models:
        mo.close()
    return {"workload": "64 random networks, 5-40 species, 10-120 reactions, %d trajectories, 200-point grids"
                        % sum(n["n_traj"] for n in nets),
            "events": st["events"], "batched_ms": round(batched_ms, 3), "plain_ms": round(plain_ms, 3),
            "timing": "median of %d graph replays / of %d passes of 64 plain launches (each network's default "
                      "kernel), HIP events" % (replays, plain_passes),
            "batched_events_per_s": round(st["events"] / (batched_ms * 1e-3), 1),
            "speedup": round(plain_ms / batched_ms, 3), "identical": identical,
            "tuned": {"win_bytes": tune["win_bytes"], "batched_ms": round(tuned_ms, 3),
                      "speedup": round(plain_ms / tuned_ms, 3)}}


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


def hiv_long(ssa, torch, dev, N=2048, t_end=4000.0, G=101, seed=7, epoch_days=40.0):
    """The HIV network of Table 1 over the paper's horizon of 4000 days (about 1.5e8 events per
    trajectory), taken in epochs of simulation time (ssa_run_begin / advance / finish); one
    progress line per epoch; mean and variance on a 101-point grid at the end."""
    m = inputs.hiv()
    model = ssa.Model.from_dict(m)
    grid = inputs.uniform_grid(t_end, G)
    run = ssa.Run(model, N, t_end, grid, seed)
    t, events, kms = 0.0, 0, 0.0
    forms = set()
    a0 = time.perf_counter()
    while t < t_end:
        t = min(t_end, t + epoch_days)
        st = run.advance(t)
        events += st["events"]
        kms += st["kernel_ms"]
        forms.add((st["form"], st["blocks"]))
        print(json.dumps({"hiv_long_epoch_to_day": t, "events": events, "kernel_ms": round(kms, 1),
                          "max_steps": st["max_steps"], "wall_s": round(time.perf_counter() - a0, 1)}), flush=True)
    mean, var, _, st = run.finish()
    torch.cuda.synchronize()
    wall = time.perf_counter() - a0
    run.close()
    model.close()
    mv = mean.cpu().numpy()
    return {"workload": "hiv: %d trajectories, t_end %g days, %d-point grid, epochs of %g days"
                        % (N, t_end, G, epoch_days),
            "launch_forms": sorted(forms),
            "events": st["events"], "max_steps": st["max_steps"], "kernel_ms": round(st["kernel_ms"], 1),
            "wall_s": round(wall, 1), "events_per_s": round(st["events"] / (st["kernel_ms"] * 1e-3), 1),
            "mean_at_end": [round(float(v), 3) for v in mv[-1]]}


def workload(name):
    w = dict(inputs.WORKLOADS[name])
    m = w["model"]()
    return m, w


KERNEL_NAMES = {
    # (direction, launch form) -> name of the specialised kernel in the trace
    ("fwd", "two_wave"): "ssa_jit_fwd_pc", ("fwd", "generations"): "ssa_jit_fwd_atomic",
    ("bwd", "two_wave"): "ssa_jit_bwd_pc", ("bwd", "generations"): "ssa_jit_bwd_gen", ("bwd", "refill"): "ssa_jit_bwd",
    ("fwd", "table"): "fwd_kernel", ("bwd", "table"): "sim_kernel_bwd",
}


def kernel_name(direction, form, hist):
    k = KERNEL_NAMES.get((direction, form), "%s_%s" % (direction, form))
    if hist and direction == "fwd" and k.startswith("ssa_jit_fwd"):
        k = {"ssa_jit_fwd_pc": "ssa_jit_fwd_hist_pc", "ssa_jit_fwd_atomic": "ssa_jit_fwd_hist"}[k]
    return k


def measure_step(ssa, torch, dev, name, steps, warmup, graph_steps=True):
    """The step (forward mean/var[/histogram] + loss weights + LR backward) on a named
    workload: K steps timed with HIP events on the launch stream, each step's own time
    too, every launch's statistics (events, launch form, simulation-kernel time by HIP
    events around it) from the timed steps themselves; forward-only steps for the
    grad / plain ratio; the roofline of the dominant simulation kernel."""
    m, w = workload(name)
    N, t_end, G, seed = w["n_traj"], w["t_end"], w["G"], w["seed"]
    grid = torch.tensor(inputs.uniform_grid(t_end, G), dtype=torch.float64, device=dev)
    model = ssa.Model.from_dict(m)
    hist = w.get("hist")
    stream = torch.cuda.current_stream()
    # target of the loss: the same network with perturbed log rates (untimed)
    prates = torch.tensor(inputs.perturbed_rates(m, w.get("perturb_seed", 404)), device=dev)
    target, _, _, _ = ssa.run_device(model, N, t_end, grid, w.get("target_seed", 44), rates=prates)
    S, M = m["reac"].shape[1], m["reac"].shape[0]
    mean = torch.empty((G, S), dtype=torch.float64, device=dev)
    var = torch.empty_like(mean)
    hbuf = torch.empty((G, hist[3]), dtype=torch.int32, device=dev) if hist else None
    gbuf = torch.empty(M, dtype=torch.float64, device=dev)
    wts = torch.empty_like(mean)

    def step():
        _, _, _, sf = ssa.run_device(model, N, t_end, grid, seed, hist=hist, out=(mean, var, hbuf), with_stats=True)
        torch.sub(mean, target, out=wts)
        wts.mul_(2.0)
        _, sb = ssa.backward_device(model, N, t_end, grid, seed, wts, mean, out=gbuf, with_stats=True)
        return sf, sb

    for _ in range(warmup):
        sf, sb = step()
        assert sf["flags"] == 0 and sb["flags"] == 0, (sf, sb)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    fs, bs = [], []
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        sf, sb = step()
        ev[i + 1].record(stream)
        fs.append(sf)
        bs.append(sb)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = ev[0].elapsed_time(ev[-1]) / steps
    per_step = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    assert all(f["events"] == fs[0]["events"] and f["flags"] == 0 for f in fs)
    assert all(b["events"] == fs[0]["events"] and b["flags"] == 0 for b in bs)
    events = fs[0]["events"]

    # forward-only steps (same calls, no backward), for the grad / plain ratio
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    f0.record(stream)
    for _ in range(steps):
        ssa.run_device(model, N, t_end, grid, seed, hist=hist, out=(mean, var, hbuf))
    f1.record(stream)
    torch.cuda.synchronize()
    fwd_only_ms = f0.elapsed_time(f1) / steps

    # the same step without statistics, captured once as a HIP graph (torch.cuda.graph) and
    # replayed K times; every replay must give the eager step's results bit for bit
    def step_graph():
        ssa.run_device(model, N, t_end, grid, seed, hist=hist, out=(mean, var, hbuf))
        torch.sub(mean, target, out=wts)
        wts.mul_(2.0)
        ssa.backward_device(model, N, t_end, grid, seed, wts, mean, out=gbuf)

    graph_ms, graph_per, g_wall = step_ms, per_step, wall
    if graph_steps:
        outs = [mean, var, gbuf] + ([hbuf] if hist else [])
        want = [x.clone() for x in outs]
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step_graph()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step_graph()
        torch.cuda.synchronize()
        for _ in range(warmup):
            graph.replay()
        torch.cuda.synchronize()
        gev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        g_t0 = time.perf_counter()
        gev[0].record(stream)
        for i in range(steps):
            graph.replay()
            gev[i + 1].record(stream)
        torch.cuda.synchronize()
        g_wall = time.perf_counter() - g_t0
        graph_ms = gev[0].elapsed_time(gev[-1]) / steps
        graph_per = [gev[i].elapsed_time(gev[i + 1]) for i in range(steps)]
        assert all(torch.equal(a, b) for a, b in zip(outs, want)), "graph replay differs from the eager step"
        del graph
    torch.cuda.synchronize()
    model.close()

    # the forward's trajectory order.  The step above runs with SSA_FWD_ORDER=0: it repeats
    # one run, and a forward of a run the model has recorded before takes its trajectories
    # longest first by those counts -- exact for the same run again (another statistic of the
    # same trajectories), a hint for other rates.  Here, with the order on: a run's first
    # forward (no record), the same run again, and a run ordered by the counts of the same
    # trajectories under rates 1 % and 10 % away (log-normal), each the best of two kernel
    # times; eager steps of the same run again; and eager steps that draw new trajectories
    # every step (a new seed each: no record for the forward, the backward takes its
    # forward's)
    def fwd_stats(mdl, rates=None, sd=seed):
        return ssa.run_device(mdl, N, t_end, grid, sd, hist=hist, rates=rates, with_stats=True)[3]

    def eager_steps(mdl, seeds, want_fwd_ordered):
        def one(sd, check=True):
            _, _, _, sf = ssa.run_device(mdl, N, t_end, grid, sd, hist=hist, out=(mean, var, hbuf),
                                         with_stats=True)
            torch.sub(mean, target, out=wts)
            wts.mul_(2.0)
            _, sb = ssa.backward_device(mdl, N, t_end, grid, sd, wts, mean, out=gbuf, with_stats=True)
            assert not check or (sf["ordered"] == want_fwd_ordered and sb["ordered"]), (sf, sb)
            assert sf["flags"] == 0 and sb["flags"] == 0, (sf, sb)
            return sf
        one(seeds[0] if want_fwd_ordered else seeds[0] - 1, check=False)   # untimed: the model's record
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sfs = [one(sd) for sd in seeds]
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / len(seeds)
        ev = sum(f["events"] for f in sfs) / len(seeds)
        return {"steps": len(seeds), "eager_ms_per_step": round(ms, 4),
                "events_per_s": round(ev / (ms * 1e-3), 1),
                "fwd_kernel_ms": round(float(np.mean([f["kernel_ms"] for f in sfs])), 4)}

    order = None
    if fs[0]["form"] == "generations":
        near = {"1%": torch.tensor(inputs.perturbed_rates(m, 405, sigma=0.01), device=dev), "10%": prates}
        saved = os.environ.pop("SSA_FWD_ORDER", None)
        try:
            cold, again, stale = [], [], {k: [] for k in near}
            for _ in range(2):
                fresh = ssa.Model.from_dict(m)
                s = fwd_stats(fresh)
                assert not s["ordered"] and s["events"] == events, s
                cold.append(s["kernel_ms"])
                s = fwd_stats(fresh)
                fresh.close()
                assert s["ordered"] and s["events"] == events, s
                again.append(s["kernel_ms"])
                for k, r in near.items():
                    other = ssa.Model.from_dict(m)
                    fwd_stats(other, r)
                    s = fwd_stats(other)
                    other.close()
                    assert s["ordered"] and s["events"] == events, s
                    stale[k].append(s["kernel_ms"])
            model2 = ssa.Model.from_dict(m)
            same = eager_steps(model2, [seed] * 5, True)
            new_seed = eager_steps(model2, [seed + 1000 + i for i in range(5)], False)
            model2.close()
        finally:
            if saved is not None:
                os.environ["SSA_FWD_ORDER"] = saved
        order = {"timed_steps_forward_ordered": any(f["ordered"] for f in fs),
                 "no_record_fwd_kernel_ms": round(min(cold), 4),
                 "same_run_again_fwd_kernel_ms": round(min(again), 4),
                 "record_rates_1pct_away_fwd_kernel_ms": round(min(stale["1%"]), 4),
                 "record_rates_10pct_away_fwd_kernel_ms": round(min(stale["10%"]), 4),
                 "same_run_again_steps": same, "new_seed_every_step": new_seed}

    # roofline of the dominant simulation kernel: algorithmic lane-ops per launch / its mean
    # launch time over the timed steps
    crossings = G * N / max(events, 1)                 # grid points passed per event
    fwd_avg = float(np.mean([f["kernel_ms"] for f in fs]))
    bwd_avg = float(np.mean([b["kernel_ms"] for b in bs]))
    wf = w_forward(m, min(1.0, crossings), mean_changes(m))
    wb = w_backward(m, crossings)
    kf = kernel_name("fwd", fs[0]["form"], hist)
    kb = kernel_name("bwd", bs[0]["form"], hist)
    if bwd_avg >= fwd_avg:
        kname, kms, wop, blocks = kb, bwd_avg, wb, bs[0]["blocks"]
    else:
        kname, kms, wop, blocks = kf, fwd_avg, wf, fs[0]["blocks"]
    achieved = wop * events / (kms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(PEAK_LANE_OPS / 1e12, 3),
                "unit": "Tlane-op/s", "frac": round(achieved * 1e12 / PEAK_LANE_OPS, 5),
                "traffic": stored_traffic(kname, name),
                "kernel": kname, "kernel_ms": round(kms, 4), "ops_per_event": round(wop, 1),
                "events_per_launch": events, "blocks": blocks,
                "other_kernel": {"kernel": kf if kname == kb else kb, "kernel_ms": round(fwd_avg if kname == kb
                                                                                        else bwd_avg, 4),
                                 "ops_per_event": round(wf if kname == kb else wb, 1),
                                 "frac": round((wf * events / (fwd_avg * 1e-3) if kname == kb
                                                else wb * events / (bwd_avg * 1e-3)) / PEAK_LANE_OPS, 5)}}
    cfg = {"workload": "%s: %d trajectories, t_end %g, %d-point grid%s, forward mean/var%s + LR backward"
                       % (name, N, t_end, G, ", histogram of I (%d bins)" % hist[3] if hist else "",
                          "/histogram" if hist else ""),
           "n_traj": N, "grid_points": G, "t_end": t_end, "species": S, "reactions": M,
           "histogram": list(hist) if hist else None}
    return dict(cfg=cfg, events=events, step_ms=step_ms, median_step_ms=float(np.median(per_step)),
                graph_ms=graph_ms, graph_median_ms=float(np.median(graph_per)), graph_wall=g_wall,
                fwd_ms=fwd_avg, bwd_ms=bwd_avg, fwd_only_ms=fwd_only_ms, wall=wall, roofline=roofline,
                fwd_form=fs[0]["form"], bwd_form=bs[0]["form"], fwd_blocks=fs[0]["blocks"],
                bwd_blocks=bs[0]["blocks"], target=target.cpu().numpy(), model=m, w=w, order=order)


def cpu_baseline(m, w, target):
    """The oracle on the host cores over a bounded sample of the workload (trajectories
    0..n-1, forward with the workload's histogram + gradient, as in a step), repeated for
    at least 10 s on all threads and 5 s on one; forward events per second."""
    from oracle import oracle as orc
    N, t_end, G, seed, hist = w["n_traj"], w["t_end"], w["G"], w["seed"], w.get("hist")
    grid_np = inputs.uniform_grid(t_end, G)

    def rate(threads, n_cpu, min_s):
        ev, reps = 0, 0
        a0 = time.perf_counter()
        while True:
            st, ref = orc.run(m, n_cpu, t_end, grid_np, seed, hist=hist, threads=threads)
            st2, _, _ = orc.grad(m, n_cpu, t_end, grid_np, seed, 2.0 * (ref["mean"] - target), ref["mean"],
                                 threads=threads)
            assert st == 0 and st2 == 0
            ev += ref["events"]
            reps += 1
            if time.perf_counter() - a0 >= min_s:
                break
        return ev / (time.perf_counter() - a0), reps, time.perf_counter() - a0

    thr = orc.default_threads()
    scale = 1.0 if G <= 1000 else 0.2          # a 10^4-point grid makes the gradient ~10x dearer
    n_all = min(N, max(256, int(20000 * scale)))
    n_one = min(N, max(64, int(2000 * scale)))
    v_all, r_all, s_all = rate(thr, n_all, 10.0)
    v_one, r_one, s_one = rate(1, n_one, 5.0)
    model_name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model_name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(v_all, 1), "unit": "events/s", "cores": thr, "kind": "oracle",
            "sample": "%d x (trajectories 0..%d of %d, forward + gradient), %.1f s on %d threads"
                      % (r_all, n_all - 1, N, s_all, thr),
            "cpu_model": model_name,
            "single_thread": {"value": round(v_one, 1), "unit": "events/s",
                              "sample": "%d x (trajectories 0..%d), %.1f s" % (r_one, n_one - 1, s_one)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["large", "viral", "differentiated"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched / plain comparison")
    ap.add_argument("--eager", action="store_true",
                    help="time the K eager steps only, without the graph capture (for counter-collection runs)")
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
    ap.add_argument("--hiv-long", action="store_true",
                    help="only run the HIV network over 4000 days (2048 trajectories, epochs of 40 days) and print it")
    ap.add_argument("--autotune", action="store_true",
                    help="only run the forward and backward autotuners on the viral, differentiated and large "
                         "workloads and print what they chose")
    args = ap.parse_args()
    # the timed steps repeat one run: forwards in index order, as a run's first forward
    # (the forward's order by a recorded run is measured on its own, see measure_step)
    os.environ["SSA_FWD_ORDER"] = "0"

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
    if args.hiv_long:
        print(json.dumps({"hiv_long": hiv_long(ssa, torch, dev)}), flush=True)
        return
    if args.adaptive:
        print(json.dumps({"adaptive": adaptive_measure(ssa, torch, dev)}), flush=True)
        return
    if args.autotune:
        for name in ("viral", "differentiated", "large"):
            m, w = workload(name)
            grid = torch.tensor(inputs.uniform_grid(w["t_end"], w["G"]), dtype=torch.float64, device=dev)
            model = ssa.Model.from_dict(m)
            f = ssa.autotune_forward(model, w["n_traj"], w["t_end"], grid, w["seed"])
            b = ssa.autotune_backward(model, w["n_traj"], w["t_end"], grid, w["seed"])
            model.close()
            print(json.dumps({"autotune": name, "n_traj": w["n_traj"], "grid_points": w["G"],
                              "forward": f, "backward": b}), flush=True)
        return
    if args.wide_sweep:
        print(json.dumps({"sweep": "wide networks, forward events/s", "rows": wide_sweep(ssa, torch, dev)}),
              flush=True)
        return

    r = measure_step(ssa, torch, dev, args.workload, args.steps, args.warmup, graph_steps=not args.eager)
    out = {
        "metric": "SSA reaction events/sec on 1 MI355X (+ % VALU roofline); batched & grad vs plain",
        "value": round(r["events"] / (r["graph_ms"] * 1e-3), 1),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["graph_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+i32",
        "data": "synthetic",
        "config": r["cfg"],
        "timing": ("K eager steps with statistics, HIP events on the launch stream" if args.eager else
                   "K replays of the step captured as one HIP graph (forward, loss weights, backward), HIP "
                   "events on the replay stream; kernel times and launch forms from K eager steps with "
                   "statistics timed in the same run"),
        "median_step_ms": round(r["graph_median_ms"], 4),
        "eager_ms_per_step": round(r["step_ms"], 4),
        "eager_median_step_ms": round(r["median_step_ms"], 4),
        "fwd_events_per_step": r["events"],
        "bwd_events_per_step": r["events"],
        "fwd_kernel_ms": round(r["fwd_ms"], 4),
        "bwd_kernel_ms": round(r["bwd_ms"], 4),
        "launch_forms": {"forward": r["fwd_form"], "backward": r["bwd_form"], "forward_blocks": r["fwd_blocks"],
                         "backward_blocks": r["bwd_blocks"]},
        "fwd_only_ms": round(r["fwd_only_ms"], 4),
        "forward_order": r["order"],
        "grad_vs_plain": round(r["step_ms"] / r["fwd_only_ms"], 3),
        "wall_s": round(r["graph_wall"], 3),
        "eager_wall_s": round(r["wall"], 3),
        "roofline": r["roofline"],
    }

    if not args.no_batched:
        # the other forms, each timed on its own workload (see --adaptive, --hiv)
        other = "viral" if args.workload != "viral" else "large"
        o = measure_step(ssa, torch, dev, other, args.steps, args.warmup, graph_steps=not args.eager)
        out["%s_case" % other] = {"workload": o["cfg"]["workload"], "events": o["events"],
                                  "ms_per_step": round(o["graph_ms"], 4),
                                  "events_per_s": round(o["events"] / (o["graph_ms"] * 1e-3), 1),
                                  "eager_ms_per_step": round(o["step_ms"], 4),
                                  "fwd_kernel_ms": round(o["fwd_ms"], 4), "bwd_kernel_ms": round(o["bwd_ms"], 4),
                                  "grad_vs_plain": round(o["step_ms"] / o["fwd_only_ms"], 3),
                                  "launch_forms": {"forward": o["fwd_form"], "backward": o["bwd_form"]},
                                  "roofline_frac": o["roofline"]["frac"], "roofline_kernel": o["roofline"]["kernel"]}
        out["batched_vs_plain"] = batched_vs_plain(ssa, torch, dev)
        out["adaptive_memory"] = adaptive_measure(ssa, torch, dev)
        out["hiv_stress"] = hiv_stress(ssa, torch, dev)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(r["model"], r["w"], r["target"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
