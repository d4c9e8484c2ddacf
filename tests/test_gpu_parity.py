"""GPU parity: the HIP path through the C ABI against the CPU oracle.

* record mode: every trajectory's grid states, event count, draws, time of the last event,
  firing counts and integrated propensities are bit-identical to the oracle's;
* forward: per-grid-point mean and variance equal to the oracle's (both sides form exact
  integer sums and round each moment once; the contract's 1e-12 relative bound is also
  reported), histograms exactly equal, event totals equal;
* sizes span several work chunks with a ragged tail; edge cases as in the oracle suite.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1007_1768_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1007_1768_amd import ssa as s
    s.load()
    return s


DEV = "cuda:0"


def _close(a, b, rel=1e-12):
    a = np.asarray(a)
    b = np.asarray(b)
    both_zero = (a == 0) & (b == 0)
    ok = both_zero | (np.abs(a - b) <= rel * np.abs(b))
    return bool(ok.all()), float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def _record_parity(ssa, m, seed, t_end, grid, trajs, rates=None, max_events=0):
    model = ssa.Model.from_dict(m)
    lo, hi = min(trajs), max(trajs) + 1
    st, rec = ssa.record(model, lo, hi - lo, t_end, grid, seed, rates=rates, max_events=max_events)
    model.close()
    for i in trajs:
        s2, r = orc.trajectory(m, seed, i, t_end, grid, rates=rates, max_events=max_events or 2**62)
        assert st == s2 == 0, (st, s2)
        k = i - lo
        assert np.array_equal(rec["states"][k], r["states"]), ("states", i)
        assert int(rec["events"][k]) == r["events"], ("events", i)
        assert int(rec["draws"][k]) == r["draws"], ("draws", i)
        assert rec["t_last"][k] == r["t_last"], ("t_last", i)
        assert np.array_equal(rec["n_fired"][k], r["n_fired"]), ("n_fired", i)
        assert np.array_equal(rec["a_int"][k], r["a_int"]), ("a_int", i)


RECORD_CASES = {
    "immigration_death": (inputs.immigration_death(), 1, 100.0, 101, range(0, 200)),
    "viral": (inputs.viral(), 2, 50.0, 1000, range(0, 150)),
    "viral_far_ids": (inputs.viral(), 2, 50.0, 1000, range(10**6 - 70, 10**6)),
    # trajectory indices across 2^32 and near 2^40: the high word of the Philox counter's
    # trajectory half is non-zero
    "viral_ids_across_2_32": (inputs.viral(), 2, 50.0, 1000, range(2**32 - 40, 2**32 + 30)),
    "viral_ids_2_40": (inputs.viral(), 7, 20.0, 200, range(2**40 + 3, 2**40 + 70)),
    "burst_200": (inputs._model("burst", ["I", "V"], [({"I": 1}, {"I": 1, "V": 200}, 2.0), ({"V": 1}, {}, 0.5),
                                                      ({"I": 1}, {}, 0.3)], [5, 0]), 3, 10.0, 41, range(0, 130)),
    "homodimer": (inputs._model("dimer", ["A", "B"], [({"A": 2}, {"B": 1}, 0.1), ({"B": 1}, {"A": 2}, 1.0)],
                                [20, 0]), 4, 3.0, 7, range(0, 100)),
    "pure_death_absorbing": (inputs._model("death", ["X"], [({"X": 1}, {}, 1.0)], [5]), 5, 1000.0, 5, range(0, 70)),
}


@pytest.mark.parametrize("case", sorted(RECORD_CASES))
def test_record_bit_exact(ssa, case):
    m, seed, t_end, G, trajs = RECORD_CASES[case]
    _record_parity(ssa, m, seed, t_end, inputs.uniform_grid(t_end, G), list(trajs))


def test_record_random_networks(ssa):
    nets = [n for n in inputs.random_networks(count=24) if n["reac"].shape[0] <= 32][:4]
    assert nets
    for n in nets:
        t_end = min(n["t_end"], 1.0)
        _record_parity(ssa, n, n["seed"], t_end, inputs.uniform_grid(t_end, 9), list(range(0, 70)))


def test_record_edge_grids(ssa):
    m = inputs.viral()
    t_end = 3.0
    st, base = orc.trajectory(m, 2, 5, t_end, np.array([t_end]))
    tl = base["t_last"]
    below = np.nextafter(tl, -np.inf)
    # grid points at an event time, just below it, duplicated, and at t_end
    _record_parity(ssa, m, 2, t_end, np.array([0.0, 0.0, below, tl, tl, t_end]), list(range(0, 10)))
    # event exactly at t_end is applied
    _record_parity(ssa, m, 2, tl, np.array([tl]), [5])
    # t_end = 0, a single grid point
    _record_parity(ssa, m, 2, 0.0, np.array([0.0]), list(range(0, 65)))
    # zero rates: nothing ever fires, no draw is made
    _record_parity(ssa, inputs.viral(rates=np.zeros(9)), 2, 50.0, inputs.uniform_grid(50.0, 4), list(range(3)))
    # rates override through the ABI
    rates = inputs.perturbed_rates(m, 11)
    _record_parity(ssa, m, 2, 5.0, inputs.uniform_grid(5.0, 11), list(range(0, 66)), rates=rates)


def _fwd(ssa, m, N, t_end, grid, seed, hist=None):
    model = ssa.Model.from_dict(m)
    g = torch.tensor(grid, dtype=torch.float64, device=DEV)
    mean, var, h, stats = ssa.run_device(model, N, t_end, g, seed, hist=hist, with_stats=True)
    torch.cuda.synchronize()
    out = (mean.cpu().numpy(), var.cpu().numpy(), None if h is None else h.cpu().numpy(), stats)
    model.close()
    return out


FWD_CASES = {
    "immigration_death_full": (inputs.immigration_death(), 1000, 100.0, 101, 1, (0, 0, 1, 200)),
    "viral_ragged": (inputs.viral(), 2083, 50.0, 1000, 2, (1, 0, 1, 64)),
    "viral_N1": (inputs.viral(), 1, 50.0, 1000, 2, None),
    "viral_N7": (inputs.viral(), 7, 20.0, 333, 3, None),
    "viral_G1": (inputs.viral(), 300, 20.0, 1, 3, None),
    "homodimer": (inputs._model("dimer", ["A", "B"], [({"A": 2}, {"B": 1}, 0.1), ({"B": 1}, {"A": 2}, 1.0)],
                                [20, 0]), 5000, 3.0, 31, 4, (0, 0, 2, 7)),
}


@pytest.mark.parametrize("case", sorted(FWD_CASES))
def test_forward_moments(ssa, case):
    m, N, t_end, G, seed, hist = FWD_CASES[case]
    grid = inputs.uniform_grid(t_end, G)
    mean, var, h, stats = _fwd(ssa, m, N, t_end, grid, seed, hist=hist)
    st, ref = orc.run(m, N, t_end, grid, seed, hist=hist)
    assert st == 0
    ok, worst = _close(mean, ref["mean"])
    assert ok, ("mean", worst)
    ok, worst = _close(var, ref["var"])
    assert ok, ("var", worst)
    assert np.array_equal(mean, ref["mean"]) and np.array_equal(var, ref["var"])
    assert stats["events"] == ref["events"]
    if hist is not None:
        assert np.array_equal(h.astype(np.int64), ref["hist"].astype(np.int64))


def test_forward_viral_full_workload(ssa):
    """The 4-species network at its full size: 10^4 trajectories, 1000-point grid."""
    w = inputs.WORKLOADS["viral"]
    m = w["model"]()
    grid = inputs.uniform_grid(w["t_end"], w["G"])
    mean, var, _, stats = _fwd(ssa, m, w["n_traj"], w["t_end"], grid, w["seed"])
    st, ref = orc.run(m, w["n_traj"], w["t_end"], grid, w["seed"])
    assert st == 0
    assert np.array_equal(mean, ref["mean"]) and np.array_equal(var, ref["var"])
    assert stats["events"] == ref["events"]


def test_forward_nonuniform_grid_with_duplicates(ssa):
    m = inputs.viral()
    rng = np.random.default_rng(3)
    grid = np.sort(np.concatenate([rng.uniform(0, 10.0, 300), [0.0, 0.0, 5.0, 5.0, 10.0]]))
    mean, var, _, _ = _fwd(ssa, m, 700, 10.0, grid, 9)
    st, ref = orc.run(m, 700, 10.0, grid, 9)
    assert _close(mean, ref["mean"])[0] and _close(var, ref["var"])[0]


def test_overflow_and_event_limit_reported(ssa):
    m = inputs._model("grow", ["X"], [({}, {"X": 1}, 1.0)], [2**31 - 10])
    model = ssa.Model.from_dict(m)
    g = torch.tensor([1000.0], dtype=torch.float64, device=DEV)
    with pytest.raises(ssa.SSAError) as e:
        ssa.run_device(model, 64, 1000.0, g, 1, with_stats=True)
    assert e.value.status == ssa.E_OVERFLOW
    model.close()
    model = ssa.Model.from_dict(inputs.viral())
    g = torch.tensor([50.0], dtype=torch.float64, device=DEV)
    with pytest.raises(ssa.SSAError) as e:
        ssa.run_device(model, 64, 50.0, g, 1, max_events=100, with_stats=True)
    assert e.value.status == ssa.E_EVENT_LIMIT
    # and the next call on the same model is clean again
    ssa.run_device(model, 64, 50.0, g, 1, with_stats=True)
    model.close()


def test_results_do_not_depend_on_launch_history(ssa):
    m = inputs.viral()
    grid = inputs.uniform_grid(20.0, 200)
    a = _fwd(ssa, m, 3000, 20.0, grid, 5)
    b = _fwd(ssa, m, 3000, 20.0, grid, 5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_forward_many_reactions(ssa):
    """Networks above 32 reactions run the table-driven kernel whose selection uses block
    checkpoints of the partial sums; their moments equal the oracle's."""
    nets = [n for n in inputs.random_networks(count=20) if n["reac"].shape[0] > 32][:4]
    assert any(n["reac"].shape[0] > 64 for n in nets)
    for n in nets:
        t_end = min(n["t_end"], 0.3)
        grid = inputs.uniform_grid(t_end, 37)
        mean, var, _, stats = _fwd(ssa, n, 333, t_end, grid, n["seed"])
        st, ref = orc.run(n, 333, t_end, grid, n["seed"])
        assert st == 0
        assert np.array_equal(mean, ref["mean"]) and np.array_equal(var, ref["var"]), n["name"]
        assert stats["events"] == ref["events"]
