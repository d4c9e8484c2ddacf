"""GPU parity of the adaptive selective memory (event log sorted by time on the device).

Avg-Y (points, means, variances) and Avg-XY must equal the oracle's bit for bit: the same
trajectories, exact integer moments at every distinct event time, and the same left-to-
right sums per group.  Cases: the viral network, immigration-death, a closed network, a
random network with bimolecular reactions, one trajectory, k = 1, k beyond the number of
points, an absorbing network (no event at all), rates given at run time, and both the
network-specialised and the table-driven kernels.
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


@pytest.fixture(params=["jit", "generic"])
def kernel(request):
    old = os.environ.get("SSA_KERNEL")
    if request.param == "generic":
        os.environ["SSA_KERNEL"] = "generic"
    elif old is not None:
        del os.environ["SSA_KERNEL"]
    yield request.param
    if old is None:
        os.environ.pop("SSA_KERNEL", None)
    else:
        os.environ["SSA_KERNEL"] = old


def _iso():
    return inputs._model("iso", ["A", "B"], [({"A": 1}, {"B": 1}, 0.7), ({"B": 1}, {"A": 1}, 0.3)], [30, 10])


def _random_small():
    # the first random network with at most 32 reactions and an event changing 3 species
    for n in inputs.random_networks(count=24):
        if n["reac"].shape[0] <= 32 and ((n["prod"] - n["reac"]) != 0).sum(axis=1).max() >= 3:
            return n
    raise AssertionError("no such network")


CASES = {
    # name: (model factory, N, t_end, seed, k)
    "viral": (inputs.viral, 200, 5.0, 3, 50),
    "immigration_death": (lambda: inputs.immigration_death(10.0, 0.1, 0), 300, 30.0, 21, 300),
    "closed": (_iso, 150, 4.0, 9, 64),
    "random": (_random_small, 64, 0.2, 5, 17),
    "one_trajectory": (inputs.viral, 1, 3.0, 11, 4),
    "k1": (inputs.viral, 20, 1.0, 2, 1),
    "k_beyond": (inputs.viral, 10, 0.5, 2, 10 ** 9),
}


def _compare(out, ref):
    for a, b in (("xy_time", "xy_time"), ("xy_mean", "xy_mean"), ("xy_var", "xy_var"),
                 ("y_time", "y_time"), ("y_mean", "y_mean"), ("y_var", "y_var")):
        got = out[a].cpu().numpy()
        assert got.shape == ref[b].shape, (a, got.shape, ref[b].shape)
        assert np.array_equal(got, ref[b]), (a, np.argwhere(got != ref[b])[:5])


@pytest.mark.parametrize("case", sorted(CASES))
def test_adaptive_matches_oracle(ssa, kernel, case):
    make, N, t_end, seed, k = CASES[case]
    m = make()
    model = ssa.Model.from_dict(m)
    out = ssa.adaptive_device(model, N, t_end, seed, k, with_y=True, with_stats=True)
    torch.cuda.synchronize()
    model.close()
    st, ref = orc.adaptive(m, N, t_end, seed, k)
    assert st == 0
    _compare(out, ref)
    assert out["stats"]["events"] == ref["events"]


def test_adaptive_absorbing(ssa):
    m = inputs._model("still", ["X", "Y"], [({"X": 1}, {"Y": 1}, 0.0)], [5, 7])
    model = ssa.Model.from_dict(m)
    out = ssa.adaptive_device(model, 33, 2.0, 1, 4, with_y=True)
    torch.cuda.synchronize()
    model.close()
    assert out["y_time"].cpu().tolist() == [0.0]
    assert out["y_mean"].cpu().tolist() == [[5.0, 7.0]]
    assert out["xy_mean"].cpu().tolist() == [[5.0, 7.0]] and out["xy_var"].cpu().tolist() == [[0.0, 0.0]]


def test_adaptive_rates_override(ssa):
    m = inputs.viral()
    rates = inputs.perturbed_rates(m, 7, 0.2)
    m2 = dict(m)
    m2["rates"] = rates
    model = ssa.Model.from_dict(m)
    out = ssa.adaptive_device(model, 80, 2.0, 4, 25, rates=torch.tensor(rates, device=DEV), with_y=True)
    torch.cuda.synchronize()
    model.close()
    st, ref = orc.adaptive(m2, 80, 2.0, 4, 25)
    assert st == 0
    _compare(out, ref)


def test_adaptive_capacity_error(ssa):
    import ctypes
    m = inputs.viral()
    model = ssa.Model.from_dict(m)
    L = ssa.load()
    npts = (ctypes.c_int64 * 2)()
    buf = torch.empty(4, dtype=torch.float64, device=DEV)
    st = L.ssa_adaptive_device(model.handle, None, 50, 1.0, 3, 0, 10, ctypes.c_void_p(buf.data_ptr()),
                               ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(buf.data_ptr()), 0, None, None, None,
                               0, npts, None, None)
    torch.cuda.synchronize()
    model.close()
    assert st == ssa.E_INVALID
    assert npts[0] > 1 and npts[1] == -(-npts[0] // 10)


@pytest.fixture()
def small_epochs(monkeypatch):
    # a record budget far below the run's: the event log is taken in many epochs
    monkeypatch.setenv("SSA_ADAPTIVE_RECORDS", "4096")
    yield


@pytest.mark.parametrize("case,k", [("viral", 50), ("viral", 1000), ("random", 17), ("k1", 1)])
def test_adaptive_in_epochs_matches_oracle(ssa, small_epochs, case, k):
    """Bounded memory: trajectories pause at each epoch's end and resume with the same draw,
    the exact sums carry over and groups continue across epochs -- the same bits as one
    pass."""
    make, N, t_end, seed, _ = CASES[case]
    m = make()
    model = ssa.Model.from_dict(m)
    out = ssa.adaptive_device(model, N, t_end, seed, k, with_y=True, with_stats=True)
    torch.cuda.synchronize()
    model.close()
    st, ref = orc.adaptive(m, N, t_end, seed, k)
    assert st == 0
    _compare(out, ref)
    assert out["stats"]["events"] == ref["events"]


def test_adaptive_epochs_hiv(ssa, small_epochs):
    m = inputs.hiv()
    model = ssa.Model.from_dict(m)
    out = ssa.adaptive_device(model, 16, 0.3, 2, 16, with_y=True)
    torch.cuda.synchronize()
    model.close()
    st, ref = orc.adaptive(m, 16, 0.3, 2, 16)
    assert st == 0
    _compare(out, ref)


def _viral_b64():
    m = dict(inputs.viral())
    m["sum_order"] = "block64"
    return m


@pytest.mark.parametrize("make,N,t_end,seed,k", [(_viral_b64, 100, 3.0, 3, 40),
                                                  (lambda: inputs.wide_network(600), 32, 0.3, 5, 64),
                                                  (lambda: inputs.wide_network(1500), 16, 0.2, 7, 100)])
@pytest.mark.parametrize("epochs", [False, True])
def test_adaptive_64_chunk_order(ssa, monkeypatch, make, N, t_end, seed, k, epochs):
    """The event log of the one-trajectory-per-wave kernels (registers, and LDS rows with the
    dependency graph) in one pass and in epochs."""
    if epochs:
        monkeypatch.setenv("SSA_ADAPTIVE_RECORDS", "4096")
    m = make()
    model = ssa.Model.from_dict(m)
    out = ssa.adaptive_device(model, N, t_end, seed, k, with_y=True, with_stats=True)
    torch.cuda.synchronize()
    model.close()
    st, ref = orc.adaptive(m, N, t_end, seed, k)
    assert st == 0
    _compare(out, ref)
    assert out["stats"]["events"] == ref["events"]


@pytest.mark.parametrize("bins", ["1", "5", "300"])
@pytest.mark.parametrize("case", ["viral", "immigration_death", "closed"])
def test_adaptive_time_order_paths(ssa, monkeypatch, bins, case):
    """The time order of the event log with forced bin counts, so every path runs: one bin
    for the whole log (one radix pass; a block-wide network in global memory, beyond 2048
    records), a few bins (networks in LDS), many bins (wave-sized bins; 300 bins take three
    radix passes of 3 bits, an odd count so the result lands in the output buffers)."""
    monkeypatch.setenv("SSA_SORT_BINS", bins)
    make, N, t_end, seed, k = CASES[case]
    m = make()
    model = ssa.Model.from_dict(m)
    out = ssa.adaptive_device(model, N, t_end, seed, k, with_y=True, with_stats=True)
    torch.cuda.synchronize()
    model.close()
    st, ref = orc.adaptive(m, N, t_end, seed, k)
    assert st == 0
    _compare(out, ref)
