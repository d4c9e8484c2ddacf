"""Parity at the workloads' full sizes, in the launch configuration the benchmark times.

* large: 10^6 trajectories, 10^4-point grid, histogram of I: mean, variance and the
  histogram at every grid point equal to the oracle's (the oracle runs all 10^6
  trajectories on the host cores, about half a minute), and every histogram row sums to N;
* differentiated: 10^5 trajectories, 1000-point grid: the backward gradient against the
  oracle's within 1e-12 of its L1 scale;
* batched: the 64-network workload in one graph-replayed launch; four networks of
  different sizes (including ones above 32 and 64 reactions) checked against the oracle
  at their full trajectory counts.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1007_1768_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1007_1768_amd import ssa as s
    s.load()
    return s


def test_large_workload_full_parity(ssa):
    w = inputs.WORKLOADS["large"]
    m = w["model"]()
    N, t_end, G, seed, hist = w["n_traj"], w["t_end"], w["G"], w["seed"], w["hist"]
    grid = inputs.uniform_grid(t_end, G)
    model = ssa.Model.from_dict(m)
    mean, var, h, st = ssa.run_device(model, N, t_end, torch.tensor(grid, device=DEV), seed, hist=hist,
                                      with_stats=True)
    torch.cuda.synchronize()
    model.close()
    h = h.cpu().numpy().astype(np.int64)
    assert np.all(h.sum(axis=1) == N)
    s, ref = orc.run(m, N, t_end, grid, seed, hist=hist)
    assert s == 0
    assert st["events"] == ref["events"]
    assert np.array_equal(mean.cpu().numpy(), ref["mean"])
    assert np.array_equal(var.cpu().numpy(), ref["var"])
    assert np.array_equal(h, ref["hist"].astype(np.int64))


def test_differentiated_workload_full_gradient(ssa):
    w = inputs.WORKLOADS["differentiated"]
    m = w["model"]()
    N, t_end, G, seed = w["n_traj"], w["t_end"], w["G"], w["seed"]
    grid = inputs.uniform_grid(t_end, G)
    model = ssa.Model.from_dict(m)
    gd = torch.tensor(grid, device=DEV)
    # the loss target and the centring mean come from the oracle, so no input of the
    # comparison is a GPU result
    s, tgt = orc.run(m, N, t_end, grid, w["target_seed"], rates=inputs.perturbed_rates(m, w["perturb_seed"]))
    assert s == 0
    s, ref = orc.run(m, N, t_end, grid, seed)
    assert s == 0
    wts = 2.0 * (ref["mean"] - tgt["mean"])
    grad, st = ssa.backward_device(model, N, t_end, gd, seed, torch.tensor(wts, device=DEV),
                                   torch.tensor(ref["mean"], device=DEV), with_stats=True)
    torch.cuda.synchronize()
    model.close()
    assert st["form"] == "generations" and st["events"] == ref["events"], st
    s, gref, l1 = orc.grad(m, N, t_end, grid, seed, wts, ref["mean"])
    assert s == 0
    g = grad.cpu().numpy()
    assert np.all(np.abs(g - gref) <= 1e-12 * l1), np.max(np.abs(g - gref) / l1)


def test_batched_workload_full_size_sampled_networks(ssa):
    nets = inputs.random_networks()
    models = [ssa.Model.from_dict(n) for n in nets]
    batch = ssa.Batch(models, [n["n_traj"] for n in nets], [n["t_end"] for n in nets], [n["grid"] for n in nets],
                      [n["seed"] for n in nets])
    means, vars_, st = batch.run(DEV, with_stats=True)
    torch.cuda.synchronize()
    sizes = [n["reac"].shape[0] for n in nets]
    picks = [int(np.argmin(sizes)), next(i for i, M in enumerate(sizes) if 32 < M <= 64),
             next(i for i, M in enumerate(sizes) if M > 100), int(np.argmin([n["n_traj"] for n in nets]))]
    for b in picks:
        n = nets[b]
        s, ref = orc.run(n, n["n_traj"], n["t_end"], n["grid"], n["seed"])
        assert s == 0
        assert np.array_equal(means[b].cpu().numpy(), ref["mean"]), b
        assert np.array_equal(vars_[b].cpu().numpy(), ref["var"]), b
    batch.close()
    for mo in models:
        mo.close()


@pytest.mark.parametrize("budget", [None, "3000000"])
def test_adaptive_viral_full_size(ssa, monkeypatch, budget):
    """Adaptive selective memory on the viral workload (10^4 trajectories, t_end 50, groups
    of k = 10^4 points), in one pass and in epochs of at most 3·10^6 records: every Avg-Y
    point time equal to the oracle's union of event times, and the Avg-XY points of the
    first, a middle and the last group bit-identical to the oracle's evaluation of those
    groups."""
    if budget:
        monkeypatch.setenv("SSA_ADAPTIVE_RECORDS", budget)
    w = inputs.WORKLOADS["viral"]
    m = w["model"]()
    N, t_end, seed, k = w["n_traj"], w["t_end"], w["seed"], w["n_traj"]
    model = ssa.Model.from_dict(m)
    out = ssa.adaptive_device(model, N, t_end, seed, k, with_y=True, with_stats=True)
    torch.cuda.synchronize()
    model.close()
    P = out["xy_time"].shape[0]
    groups = [0, P // 2, P - 1]
    st, ref = orc.adaptive_groups(m, N, t_end, seed, k, groups)
    assert st == 0
    assert out["stats"]["events"] == ref["events"]
    assert np.array_equal(out["y_time"].cpu().numpy(), ref["y_time"])
    assert P == -(-ref["y_time"].shape[0] // k)
    assert np.array_equal(out["xy_time"].cpu().numpy()[groups], ref["xy_time"])
    assert np.array_equal(out["xy_mean"].cpu().numpy()[groups], ref["xy_mean"])
    assert np.array_equal(out["xy_var"].cpu().numpy()[groups], ref["xy_var"])
