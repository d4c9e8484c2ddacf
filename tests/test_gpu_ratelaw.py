"""GPU parity of networks with rate laws (species-dependent rate constants) and of the HIV
network of Table 1 built on them.

Record mode bit-identical to the oracle (grid states, events, draws, last event time, n_j,
A_j); forward mean, variance and histogram equal to the oracle's; the adaptive memory on
the HIV network equal to the oracle's; laws are refused where the library does not
support them (backward, batches, the 64-chunk order) and force the specialised kernels.
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


def _birth_law():
    m = inputs._model("bd", ["X"], [({}, {"X": 1}, 2.0), ({"X": 1}, {}, 0.4)], [0])
    m["laws"] = dict(species=np.array([0, -1], np.int32), slope=np.array([0.5, 0.0]), lo=np.zeros(2),
                     hi=np.array([6.0, np.inf]))
    return m


CASES = {
    "hiv": (inputs.hiv, 1.0, 11, 5),
    "birth_law": (_birth_law, 6.0, 25, 3),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_ratelaw_record_bit_exact(ssa, case):
    make, t_end, G, seed = CASES[case]
    m = make()
    grid = inputs.uniform_grid(t_end, G)
    model = ssa.Model.from_dict(m)
    n = 24
    st, rec = ssa.record(model, 0, n, t_end, grid, seed)
    model.close()
    assert st == 0
    for i in range(n):
        s2, r = orc.trajectory(m, seed, i, t_end, grid)
        assert s2 == 0
        assert np.array_equal(rec["states"][i], r["states"]), ("states", i)
        assert int(rec["events"][i]) == r["events"], ("events", i)
        assert int(rec["draws"][i]) == r["draws"], ("draws", i)
        assert rec["t_last"][i] == r["t_last"], ("t_last", i)
        assert np.array_equal(rec["n_fired"][i], r["n_fired"]), ("n_fired", i)
        assert np.array_equal(rec["a_int"][i], r["a_int"]), ("a_int", i)


def test_hiv_forward_exact(ssa):
    m = inputs.hiv()
    N, t_end, G, seed = 256, 0.5, 51, 8
    hist = (2, 0, 40, 40)                       # T cells in bins of 40
    grid = inputs.uniform_grid(t_end, G)
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


def test_hiv_adaptive_exact(ssa):
    m = inputs.hiv()
    model = ssa.Model.from_dict(m)
    out = ssa.adaptive_device(model, 16, 0.3, 2, 16, with_y=True)
    torch.cuda.synchronize()
    model.close()
    st, ref = orc.adaptive(m, 16, 0.3, 2, 16)
    assert st == 0
    for key in ("y_time", "y_mean", "y_var", "xy_time", "xy_mean", "xy_var"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key


def test_ratelaw_forces_specialised_kernels(ssa):
    old = os.environ.get("SSA_KERNEL")
    os.environ["SSA_KERNEL"] = "generic"
    try:
        m = inputs.hiv()
        grid = inputs.uniform_grid(0.2, 5)
        model = ssa.Model.from_dict(m)
        mean, var, _, _ = ssa.run_device(model, 64, 0.2, torch.tensor(grid, device=DEV), 1)
        torch.cuda.synchronize()
        model.close()
        st, ref = orc.run(m, 64, 0.2, grid, 1)
        assert np.array_equal(mean.cpu().numpy(), ref["mean"])
    finally:
        if old is None:
            del os.environ["SSA_KERNEL"]
        else:
            os.environ["SSA_KERNEL"] = old


def test_ratelaw_refusals(ssa):
    m = inputs.hiv()
    model = ssa.Model.from_dict(m)
    grid = torch.tensor(inputs.uniform_grid(1.0, 4), device=DEV)
    w = torch.zeros((4, 10), dtype=torch.float64, device=DEV)
    with pytest.raises(ssa.SSAError) as e:
        ssa.backward_device(model, 64, 1.0, grid, 1, w, w)
    assert e.value.status == ssa.E_UNSUPPORTED
    with pytest.raises(ssa.SSAError) as e:
        ssa.Batch([model], [64], [1.0], [np.array([0.0, 1.0])], [1])
    assert e.value.status == ssa.E_UNSUPPORTED
    model.close()
    b = dict(m)
    b["sum_order"] = "block64"
    with pytest.raises(ssa.SSAError) as e:
        ssa.Model.from_dict(b)
    assert e.value.status == ssa.E_UNSUPPORTED
    bad = dict(m)
    bad["laws"] = dict(m["laws"])
    bad["laws"]["lo"] = m["laws"]["lo"].copy()
    bad["laws"]["lo"][7] = -1.0
    with pytest.raises(ssa.SSAError) as e:
        ssa.Model.from_dict(bad)
    assert e.value.status == ssa.E_INVALID
