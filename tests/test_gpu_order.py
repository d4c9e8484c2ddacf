"""GPU checks of the trajectory order of the backward and the forward.

A forward in generations records every trajectory's event count; a backward of the same
run (trajectory count, horizon, seed, event cap, grid and rate arrays) then takes its
trajectories longest first, and so does a later forward with the same trajectory count,
horizon, seed and event cap (its rates may differ).  The order must never change a bit:
each trajectory keeps its index, its Philox stream and its row of the fixed-order
reduction, and the forward's sums are exact integers.
Cases: without and with a recorded order (mean and variance weights, generations and
refilled lanes); a backward of another run (other seed, other grid array, other trajectory
count) ignores the record; a record gone stale (rates changed in place after the forward)
is still used and still gives the exact gradient; two models keep their own records; the
forward in recorded order gives the moments and histogram of an unordered one, also under
other rates, and matches the CPU oracle; the statistics say which order ran.
"""
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1007_1768_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
# 3907 work items: beyond two-wave launches, so the lane kernels run
N, T_END, G, SEED = 250_000, 6.0, 300, 91


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1007_1768_amd import ssa as s
    s.load()
    return s


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.fixture
def form(request, monkeypatch):
    if request.param:
        monkeypatch.setenv("SSA_LAUNCH_FORM", request.param)
    else:
        monkeypatch.delenv("SSA_LAUNCH_FORM", raising=False)
    return request.param or "generations"


@pytest.mark.parametrize("form", [None, "refill"], indirect=True)
@pytest.mark.parametrize("quad", [False, True])
def test_recorded_order_gives_the_same_gradient(ssa, form, quad):
    m = inputs.viral()
    grid = _t(inputs.uniform_grid(T_END, G))
    rng = np.random.default_rng(3)
    w = _t(rng.normal(size=(G, 4)))
    wv = _t(rng.normal(size=(G, 4)) * 1e-3) if quad else None
    model = ssa.Model.from_dict(m)
    print("order form %s quad %s" % (form, quad), flush=True)
    other = ssa.Model.from_dict(m)                    # the moments, from a model whose record stays apart
    mean, var, _, _ = ssa.run_device(other, N, T_END, grid, SEED)
    vh = var if quad else None
    g0, s0 = ssa.backward_device(model, N, T_END, grid, SEED, w, mean, wv=wv, vhat=vh, with_stats=True)
    _, _, _, sf = ssa.run_device(model, N, T_END, grid, SEED, with_stats=True)
    g1, s1 = ssa.backward_device(model, N, T_END, grid, SEED, w, mean, wv=wv, vhat=vh, with_stats=True)
    torch.cuda.synchronize()
    assert sf["form"] == "generations" and s0["form"] == form and s1["form"] == form, (sf, s0, s1)
    assert not s0["ordered"] and s1["ordered"], (s0, s1)
    assert s0["events"] == s1["events"] == sf["events"]
    assert torch.equal(g0, g1), (g0, g1)
    model.close()
    other.close()


def test_other_runs_ignore_the_record(ssa):
    m = inputs.viral()
    grid = _t(inputs.uniform_grid(T_END, G))
    w = _t(np.random.default_rng(4).normal(size=(G, 4)))
    model = ssa.Model.from_dict(m)
    mean, _, _, _ = ssa.run_device(model, N, T_END, grid, SEED)
    grid2 = grid.clone()                              # same values, another array
    for args in [(N, T_END, grid, SEED + 1), (N, T_END, grid2, SEED), (N - 64, T_END, grid, SEED),
                 (N, T_END + 1.0, _t(inputs.uniform_grid(T_END + 1.0, G)), SEED)]:
        g, st = ssa.backward_device(model, *args, w, mean, with_stats=True)
        ref = ssa.Model.from_dict(m)                  # a model with no record
        g_ref, st_ref = ssa.backward_device(ref, *args, w, mean, with_stats=True)
        torch.cuda.synchronize()
        ref.close()
        assert not st["ordered"] and not st_ref["ordered"], (args[0], args[1], args[3], st)
        assert torch.equal(g, g_ref)
    model.close()


def test_stale_record_still_exact(ssa):
    m = inputs.viral()
    grid = _t(inputs.uniform_grid(T_END, G))
    w = _t(np.random.default_rng(5).normal(size=(G, 4)))
    rates = _t(m["rates"])
    model = ssa.Model.from_dict(m)
    mean, _, _, _ = ssa.run_device(model, N, T_END, grid, SEED, rates=rates)
    rates.mul_(_t(np.exp(np.random.default_rng(6).normal(0.0, 0.3, 9))))   # in place: same array
    g, st = ssa.backward_device(model, N, T_END, grid, SEED, w, mean, rates=rates, with_stats=True)
    ref = ssa.Model.from_dict(m)
    g_ref, st_ref = ssa.backward_device(ref, N, T_END, grid, SEED, w, mean, rates=rates, with_stats=True)
    torch.cuda.synchronize()
    ref.close()
    model.close()
    assert st["ordered"] and not st_ref["ordered"]
    assert st["events"] == st_ref["events"]
    assert torch.equal(g, g_ref)


def test_models_keep_their_own_records(ssa):
    m = inputs.viral()
    grid = _t(inputs.uniform_grid(T_END, G))
    w = _t(np.random.default_rng(7).normal(size=(G, 4)))
    a, b = ssa.Model.from_dict(m), ssa.Model.from_dict(m)
    mean, _, _, _ = ssa.run_device(a, N, T_END, grid, SEED)
    _, _, _, _ = ssa.run_device(b, N, T_END, grid, SEED + 5)
    ga, sa = ssa.backward_device(a, N, T_END, grid, SEED, w, mean, with_stats=True)
    gb, sb = ssa.backward_device(b, N, T_END, grid, SEED, w, mean, with_stats=True)
    torch.cuda.synchronize()
    assert sa["ordered"] and not sb["ordered"]
    assert torch.equal(ga, gb)
    a.close()
    b.close()


def test_forward_in_recorded_order_gives_the_same_outputs(ssa):
    m = inputs.viral()
    grid = _t(inputs.uniform_grid(T_END, G))
    hist = (1, 0, 1, 64)
    model = ssa.Model.from_dict(m)
    print("forward order: record, ordered, other rates, other seed", flush=True)
    a = ssa.run_device(model, N, T_END, grid, SEED, hist=hist, with_stats=True)
    b = ssa.run_device(model, N, T_END, grid, SEED, hist=hist, with_stats=True)
    torch.cuda.synchronize()
    assert a[3]["form"] == b[3]["form"] == "generations", (a[3], b[3])
    assert not a[3]["ordered"] and b[3]["ordered"], (a[3], b[3])
    assert a[3]["events"] == b[3]["events"]
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)
    # a fit's next step: the same trajectories under other rates, ordered by the old counts
    rates = _t(np.asarray(m["rates"]) * np.exp(np.random.default_rng(8).normal(0.0, 0.3, 9)))
    c = ssa.run_device(model, N, T_END, grid, SEED, hist=hist, rates=rates, with_stats=True)
    ref = ssa.Model.from_dict(m)                      # a model with no record
    r = ssa.run_device(ref, N, T_END, grid, SEED, hist=hist, rates=rates, with_stats=True)
    # another seed: other trajectories, the record is not used
    d = ssa.run_device(model, N, T_END, grid, SEED + 1, hist=hist, with_stats=True)
    e = ssa.run_device(ref, N, T_END, grid, SEED + 1, hist=hist, with_stats=True)
    torch.cuda.synchronize()
    ref.close()
    model.close()
    assert c[3]["ordered"] and not r[3]["ordered"], (c[3], r[3])
    assert not d[3]["ordered"] and not e[3]["ordered"], (d[3], e[3])
    assert c[3]["events"] == r[3]["events"] and d[3]["events"] == e[3]["events"]
    for x, y in list(zip(c[:3], r[:3])) + list(zip(d[:3], e[:3])):
        assert torch.equal(x, y)


def test_forward_in_recorded_order_matches_the_oracle(ssa, monkeypatch):
    monkeypatch.setenv("SSA_LAUNCH_FORM", "generations")
    m = inputs.viral()
    n, t_end, g, seed, hist = 3001, 6.0, 41, 12, (1, 0, 1, 16)
    grid_np = inputs.uniform_grid(t_end, g)
    grid = _t(grid_np)
    model = ssa.Model.from_dict(m)
    print("forward order vs oracle: N %d" % n, flush=True)
    ssa.run_device(model, n, t_end, grid, seed, hist=hist)
    mean, var, h, st = ssa.run_device(model, n, t_end, grid, seed, hist=hist, with_stats=True)
    torch.cuda.synchronize()
    model.close()
    assert st["ordered"] and st["form"] == "generations", st
    s, ref = orc.run(m, n, t_end, grid_np, seed, hist=hist)
    assert s == 0
    assert np.array_equal(mean.cpu().numpy(), ref["mean"]) and np.array_equal(var.cpu().numpy(), ref["var"])
    assert np.array_equal(h.cpu().numpy().astype(np.int64), ref["hist"].astype(np.int64))
    assert st["events"] == ref["events"]


def test_forward_order_switch(ssa, monkeypatch):
    """SSA_FWD_ORDER=0: a forward of a recorded run stays in index order, with the same outputs."""
    m = inputs.viral()
    grid = _t(inputs.uniform_grid(T_END, G))
    model = ssa.Model.from_dict(m)
    print("forward order switch", flush=True)
    a = ssa.run_device(model, N, T_END, grid, SEED, with_stats=True)
    monkeypatch.setenv("SSA_FWD_ORDER", "0")
    b = ssa.run_device(model, N, T_END, grid, SEED, with_stats=True)
    monkeypatch.delenv("SSA_FWD_ORDER")
    c = ssa.run_device(model, N, T_END, grid, SEED, with_stats=True)
    torch.cuda.synchronize()
    model.close()
    assert not a[3]["ordered"] and not b[3]["ordered"] and c[3]["ordered"], (a[3], b[3], c[3])
    for x, y, z in zip(a[:2], b[:2], c[:2]):
        assert torch.equal(x, y) and torch.equal(x, z)
