"""GPU parity of the likelihood-ratio backward in each of its launch forms.

The specialised backward runs in one of three forms, chosen by the launch size: blocks of
a simulating and a drawing wave (up to two work items of 64 trajectories per CU), persistent
blocks that refill a wave by generations (beyond: the form the large workload's gradient
runs), and persistent blocks that refill each lane as its trajectory ends (by request or a
tuned launch).  Every form must give the oracle's gradient within 1e-12 of its L1 scale, with mean
weights and with mean and variance weights, and the call must report the form it ran.

* forced forms (SSA_LAUNCH_FORM) at small sizes: a ragged count on a fine grid, grid points
  at, just below and duplicated on event times, and a network whose trajectories reach an
  absorbing state long before t_end;
* the persistent forms (generations, the default beyond two-wave launches and the large
  workload's own; refilled lanes) at the large workload's grid (10^4 points, t_end 50) with
  more than 2048 work items, after a forward of the same run (so their trajectories run
  longest first, in the order of the lengths that forward recorded).
"""
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1007_1768_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1007_1768_amd import ssa as s
    s.load()
    return s


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _event_grid():
    """Grid points at the last event times of a few viral trajectories, one ulp below them
    and duplicated, plus 0 and t_end (non-uniform)."""
    m = inputs.viral()
    t_end = 3.0
    pts = [0.0, 0.0, t_end]
    for i in range(6):
        st, r = orc.trajectory(m, 2, i, t_end, np.array([t_end]))
        assert st == 0
        tl = float(r["t_last"])
        pts += [tl, tl, float(np.nextafter(tl, -np.inf))]
    return np.array(sorted(pts))


CASES = {
    "viral_ragged_fine_grid": (inputs.viral, 700, 20.0, lambda: inputs.uniform_grid(20.0, 400), 21),
    "viral_event_time_grid": (inputs.viral, 300, 3.0, _event_grid, 2),
    "pure_death_absorbing": (lambda: inputs._model("death", ["X"], [({"X": 1}, {}, 1.0)], [5]), 200, 50.0,
                             lambda: inputs.uniform_grid(50.0, 60), 5),
}


@pytest.fixture(params=["two_wave", "generations", "refill"])
def form(request):
    old = os.environ.get("SSA_LAUNCH_FORM")
    os.environ["SSA_LAUNCH_FORM"] = request.param
    yield request.param
    if old is None:
        os.environ.pop("SSA_LAUNCH_FORM", None)
    else:
        os.environ["SSA_LAUNCH_FORM"] = old


@pytest.mark.parametrize("case", sorted(CASES))
def test_backward_form_matches_oracle(ssa, form, case):
    make, N, t_end, make_grid, seed = CASES[case]
    m = make()
    grid = make_grid()
    st, ref = orc.run(m, N, t_end, grid, seed)
    assert st == 0
    rng = np.random.default_rng(seed)
    w = rng.normal(size=ref["mean"].shape)
    wv = rng.normal(size=ref["mean"].shape) / (1.0 + ref["var"])
    model = ssa.Model.from_dict(m)
    print("case %s form %s N %d G %d" % (case, form, N, grid.shape[0]), flush=True)
    g, sb = ssa.backward_device(model, N, t_end, _t(grid), seed, _t(w), _t(ref["mean"]), with_stats=True)
    gq, sq = ssa.backward_device(model, N, t_end, _t(grid), seed, _t(w), _t(ref["mean"]), wv=_t(wv),
                                 vhat=_t(ref["var"]), with_stats=True)
    torch.cuda.synchronize()
    model.close()
    assert sb["form"] == form and sq["form"] == form, (sb, sq)
    assert sb["events"] == ref["events"] and sq["events"] == ref["events"]
    st, gref, l1 = orc.grad(m, N, t_end, grid, seed, w, ref["mean"])
    assert st == 0
    assert np.all(np.abs(g.cpu().numpy() - gref) <= 1e-12 * l1), (g.cpu().numpy(), gref, l1)
    st, gref, l1 = orc.grad(m, N, t_end, grid, seed, w, ref["mean"], wv=wv, vhat=ref["var"])
    assert st == 0
    assert np.all(np.abs(gq.cpu().numpy() - gref) <= 1e-12 * l1), (gq.cpu().numpy(), gref, l1)


# The large workload's network, horizon and grid with just over 2048 work items: the
# persistent forms at the large workload's grid (generations by default, refilled lanes when
# asked for), against the oracle's gradients computed once.
N_BIG, T_BIG, G_BIG, SEED_BIG = 135000, 50.0, 10000, 55


@pytest.fixture(scope="module")
def big_ref():
    m = inputs.viral()
    grid = inputs.uniform_grid(T_BIG, G_BIG)
    st, ref = orc.run(m, N_BIG, T_BIG, grid, SEED_BIG)
    assert st == 0
    rng = np.random.default_rng(SEED_BIG)
    w = rng.normal(size=ref["mean"].shape)
    wv = rng.normal(size=ref["mean"].shape) / (1.0 + ref["var"])
    grads = {}
    st, grads["mean"], l1m = orc.grad(m, N_BIG, T_BIG, grid, SEED_BIG, w, ref["mean"])
    assert st == 0
    st, grads["mean_and_variance"], l1q = orc.grad(m, N_BIG, T_BIG, grid, SEED_BIG, w, ref["mean"], wv=wv,
                                                   vhat=ref["var"])
    assert st == 0
    return m, grid, ref, w, wv, grads, {"mean": l1m, "mean_and_variance": l1q}


@pytest.mark.parametrize("weights", ["mean", "mean_and_variance"])
@pytest.mark.parametrize("asked", [None, "refill"])
def test_persistent_backward_at_large_grid(ssa, big_ref, monkeypatch, weights, asked):
    m, grid, ref, w, wv, grads, l1 = big_ref
    if asked:
        monkeypatch.setenv("SSA_LAUNCH_FORM", asked)
    else:
        monkeypatch.delenv("SSA_LAUNCH_FORM", raising=False)
    model = ssa.Model.from_dict(m)
    gd = _t(grid)
    print("persistent backward N %d G %d weights %s form %s" % (N_BIG, G_BIG, weights, asked), flush=True)
    mean, var, _, sf = ssa.run_device(model, N_BIG, T_BIG, gd, SEED_BIG, with_stats=True)
    quad = weights == "mean_and_variance"
    g, sb = ssa.backward_device(model, N_BIG, T_BIG, gd, SEED_BIG, _t(w), _t(ref["mean"]),
                                wv=_t(wv) if quad else None, vhat=_t(ref["var"]) if quad else None,
                                with_stats=True)
    torch.cuda.synchronize()
    model.close()
    assert sb["form"] == (asked or "generations"), sb
    assert sb["ordered"], sb        # longest first, from the lengths the forward above recorded
    assert sb["events"] == ref["events"] == sf["events"]
    assert np.array_equal(mean.cpu().numpy(), ref["mean"]) and np.array_equal(var.cpu().numpy(), ref["var"])
    assert np.all(np.abs(g.cpu().numpy() - grads[weights]) <= 1e-12 * l1[weights]), (g.cpu().numpy(), grads[weights])
