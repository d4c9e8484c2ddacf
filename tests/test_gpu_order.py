"""GPU checks of the backward's trajectory order.

A forward in generations records every trajectory's event count; a backward of the same
run (trajectory count, horizon, seed, event cap, grid and rate arrays) then takes its
trajectories longest first.  The order must never change a bit of the gradient: each
trajectory keeps its index, its Philox stream and its row of the fixed-order reduction.
Cases: without and with a recorded order (mean and variance weights, generations and
refilled lanes); a backward of another run (other seed, other grid array, other trajectory
count) ignores the record; a record gone stale (rates changed in place after the forward)
is still used and still gives the exact gradient; two models keep their own records; the
statistics say which order ran.
"""
import os

import numpy as np
import pytest

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
