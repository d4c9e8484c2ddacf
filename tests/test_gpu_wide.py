"""GPU parity of the 64-chunk kernel for networks with more than 8 reactions per lane.

Networks of 600 (10 per lane), 1500 (24, ragged last chunk) and 4096 reactions (64 per
lane, the limit).  Both the dependency-graph update (default) and the full re-evaluation
(SSA_WIDE_DEPG=0) must reproduce the oracle's 64-chunk trajectories bit for bit: record
mode (grid states, events, draws, last event time, n_j, A_j) and forward moments with a
histogram; rates passed at run time override the model's in both.  The backward keeps the
scores and accumulators in LDS and matches the oracle's gradient within 1e-12 of its scale.
"""
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1007_1768_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# name: (M, seed, t_end, G, trajectories recorded, trajectories in the forward run)
CASES = {
    "wide600_q10": (600, 3, 1.0, 41, 64, 515),
    "wide1500_q24": (1500, 5, 0.5, 33, 48, 300),
    "wide4096_q64": (4096, 7, 0.2, 21, 20, 150),
}


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1007_1768_amd import ssa as s
    s.load()
    return s


@pytest.fixture(params=["depg", "full"])
def update(request):
    old = os.environ.get("SSA_WIDE_DEPG")
    os.environ["SSA_WIDE_DEPG"] = "1" if request.param == "depg" else "0"
    yield request.param
    if old is None:
        del os.environ["SSA_WIDE_DEPG"]
    else:
        os.environ["SSA_WIDE_DEPG"] = old


@pytest.mark.parametrize("case", sorted(CASES))
def test_wide_record_bit_exact(ssa, update, case):
    M, seed, t_end, G, n_rec, _ = CASES[case]
    m = inputs.wide_network(M)
    grid = inputs.uniform_grid(t_end, G)
    model = ssa.Model.from_dict(m)
    st, rec = ssa.record(model, 0, n_rec, t_end, grid, seed)
    model.close()
    assert st == 0
    for i in range(n_rec):
        s2, r = orc.trajectory(m, seed, i, t_end, grid)
        assert s2 == 0
        assert np.array_equal(rec["states"][i], r["states"]), ("states", i)
        assert int(rec["events"][i]) == r["events"], ("events", i)
        assert int(rec["draws"][i]) == r["draws"], ("draws", i)
        assert rec["t_last"][i] == r["t_last"], ("t_last", i)
        assert np.array_equal(rec["n_fired"][i], r["n_fired"]), ("n_fired", i)
        assert np.array_equal(rec["a_int"][i], r["a_int"]), ("a_int", i)


@pytest.mark.parametrize("case", sorted(CASES))
def test_wide_forward_exact(ssa, update, case):
    M, seed, t_end, G, _, N = CASES[case]
    m = inputs.wide_network(M)
    grid = inputs.uniform_grid(t_end, G)
    hist = (2, 0, 2, 24)
    model = ssa.Model.from_dict(m)
    mean, var, h, stats = ssa.run_device(model, N, t_end, torch.tensor(grid, device=DEV), seed, hist=hist,
                                         with_stats=True)
    torch.cuda.synchronize()
    model.close()
    st, ref = orc.run(m, N, t_end, grid, seed, hist=hist)
    assert st == 0
    assert np.array_equal(mean.cpu().numpy(), ref["mean"])
    assert np.array_equal(var.cpu().numpy(), ref["var"])
    assert np.array_equal(h.cpu().numpy().astype(np.int64), ref["hist"].astype(np.int64))
    assert stats["events"] == ref["events"]


def test_wide_rates_override(ssa, update):
    """Rates given at run time reach the dependency-graph re-evaluation too."""
    M, seed, t_end, G = 1500, 11, 0.5, 17
    m = inputs.wide_network(M)
    rates = m["rates"] * np.exp(np.random.default_rng(1).normal(0.0, 0.3, size=M))
    m2 = dict(m)
    m2["rates"] = rates
    grid = inputs.uniform_grid(t_end, G)
    model = ssa.Model.from_dict(m)
    N = 200
    mean, var, _, _ = ssa.run_device(model, N, t_end, torch.tensor(grid, device=DEV), seed,
                               rates=torch.tensor(rates, device=DEV))
    torch.cuda.synchronize()
    st, rec = ssa.record(model, 0, 8, t_end, grid, seed, rates=rates)
    model.close()
    st2, ref = orc.run(m2, N, t_end, grid, seed)
    assert st2 == 0
    assert np.array_equal(mean.cpu().numpy(), ref["mean"])
    assert np.array_equal(var.cpu().numpy(), ref["var"])
    for i in range(8):
        _, r = orc.trajectory(m2, seed, i, t_end, grid)
        assert np.array_equal(rec["a_int"][i], r["a_int"]), i


_WIDE_GRAD_REF = {}


@pytest.mark.parametrize("M", [600, 1500, 4096])
def test_wide_backward_matches_oracle(ssa, update, M):
    """The backward of the LDS-resident kernel (scores and accumulators in LDS rows: 96 KB
    per wave at 4096 reactions, one wave per CU) against the oracle's gradient in the same
    sum order, within 1e-12 of its L1 scale."""
    m = inputs.wide_network(M)
    N, t_end, G, seed = 96, 0.5, 11, 13
    grid = inputs.uniform_grid(t_end, G)
    if M not in _WIDE_GRAD_REF:          # the oracle once per size (both update variants use it)
        st, ref = orc.run(m, N, t_end, grid, seed)
        assert st == 0
        w = np.random.default_rng(M).normal(size=ref["mean"].shape)
        st, gref, l1 = orc.grad(m, N, t_end, grid, seed, w, ref["mean"])
        assert st == 0
        _WIDE_GRAD_REF[M] = (ref, w, gref, l1)
    ref, w, gref, l1 = _WIDE_GRAD_REF[M]
    model = ssa.Model.from_dict(m)
    print("wide backward M %d" % M, flush=True)
    g, stats = ssa.backward_device(model, N, t_end, torch.tensor(grid, device=DEV), seed,
                                   torch.tensor(w, device=DEV), torch.tensor(ref["mean"], device=DEV),
                                   with_stats=True)
    torch.cuda.synchronize()
    model.close()
    d = np.abs(g.cpu().numpy() - gref)
    assert np.all(d <= 1e-12 * l1 + 1e-300), (d / np.maximum(l1, 1e-300)).max()
    assert stats["events"] == ref["events"]
