"""GPU parity of the species covariance pass: means and covariance matrices equal to the
oracle's exact-sum values at every grid point, including a network whose cross products
need the high-part path (|nu x_r| >= 2^24) and a conserved pair whose covariance is minus
the variance."""
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


CASES = {
    "viral_ragged": (inputs.viral(), 2083, 20.0, 101, 2),
    "isomerisation": (inputs._model("iso", ["A", "B"], [({"A": 1}, {"B": 1}, 1.0), ({"B": 1}, {"A": 1}, 0.5)],
                                    [20, 0]), 3000, 4.0, 9, 5),
    "large_counts": (inputs._model("big", ["A", "B", "C"], [({"A": 1}, {"A": 1, "B": 50}, 2e-6),
                                                            ({"B": 1}, {}, 1e-3), ({"B": 1}, {"C": 1}, 1e-3)],
                                   [1_000_000, 500_000, 0]), 130, 0.2, 5, 7),
    "N1": (inputs.viral(), 1, 10.0, 11, 3),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_covariance_matches_oracle(ssa, case):
    m, N, t_end, G, seed = CASES[case]
    grid = inputs.uniform_grid(t_end, G)
    model = ssa.Model.from_dict(m)
    mean, cov, st = ssa.run_cov_device(model, N, t_end, torch.tensor(grid, device=DEV), seed, with_stats=True)
    torch.cuda.synchronize()
    model.close()
    s, rmean, rcov = orc.covariance(m, N, t_end, grid, seed)
    assert s == 0
    assert np.array_equal(mean.cpu().numpy(), rmean)
    assert np.array_equal(cov.cpu().numpy(), rcov)
    if case == "isomerisation":
        c = cov.cpu().numpy()
        assert np.array_equal(c[:, 0, 1], -c[:, 0, 0])


def test_quantiles_are_order_statistics(ssa):
    """With width 1 and a top bin above every count, the q-quantile of the histogram is the
    k-th smallest count, k = max(1, ceil(q N)): compared with the sorted grid states of the
    oracle's own trajectories and with the cumulative oracle histogram."""
    m = inputs.immigration_death()
    N, t_end, G, seed = 700, 30.0, 7, 9
    spec = (0, 0, 1, 400)
    grid = inputs.uniform_grid(t_end, G)
    model = ssa.Model.from_dict(m)
    mean, var, h, _ = ssa.run_device(model, N, t_end, torch.tensor(grid, device=DEV), seed, hist=spec)
    qs = np.array([1e-9, 0.1, 0.25, 0.5, 0.75, 0.9, 1.0])
    out = ssa.hist_quantiles(h, spec, N, torch.tensor(qs, device=DEV)).cpu().numpy()
    torch.cuda.synchronize()
    model.close()
    states = np.zeros((N, G), dtype=np.int64)
    for i in range(N):
        st, r = orc.trajectory(m, seed, i, t_end, grid)
        assert st == 0
        states[i] = r["states"][:, 0]
    assert states.max() < 399
    srt = np.sort(states, axis=0)
    for iq, q in enumerate(qs):
        k = max(1, int(np.ceil(q * N)))
        assert np.array_equal(out[:, iq], srt[k - 1]), q
