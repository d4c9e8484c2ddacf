"""The likelihood-ratio gradient against central finite differences with common random
numbers (h = 1e-3 on the log rate constants), on the differentiated workload's network and
loss at 10^4 trajectories per batch.

With w = dL/dmean = 2 (m - y) from the batch's own forward pass, both estimate
sum_{g,s} w_gs d m_gs / d ln c_j: the LR backward (one re-simulation) and
sum w (m(ln c + h e_j) - m(ln c - h e_j)) / 2h with the same seed.  Sixteen independent
batches (seeds) give the mean and standard error of their difference per reaction; it must
be within 4 standard errors of zero (plus 1e-3 of the gradient's size for the O(h^2) bias).
"""
import numpy as np
import pytest

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


def test_lr_gradient_matches_central_differences(ssa):
    w_ = inputs.WORKLOADS["differentiated"]
    m = w_["model"]()
    N, t_end, G = 10_000, w_["t_end"], 200
    grid = torch.tensor(inputs.uniform_grid(t_end, G), dtype=torch.float64, device=DEV)
    model = ssa.Model.from_dict(m)
    lr0 = np.log(m["rates"])
    prates = torch.tensor(inputs.perturbed_rates(m, w_["perturb_seed"]), device=DEV)
    target, _, _, _ = ssa.run_device(model, N, t_end, grid, w_["target_seed"], rates=prates)
    h = 1e-3
    M = len(lr0)
    diffs, grads = [], []
    for b in range(16):
        seed = 1000 + b
        rates = torch.tensor(np.exp(lr0), device=DEV)
        mean, _, _, _ = ssa.run_device(model, N, t_end, grid, seed, rates=rates)
        w = 2.0 * (mean - target)
        g, _ = ssa.backward_device(model, N, t_end, grid, seed, w, mean, rates=rates)
        fd = np.zeros(M)
        for j in range(M):
            lp, lm = lr0.copy(), lr0.copy()
            lp[j] += h
            lm[j] -= h
            mp, _, _, _ = ssa.run_device(model, N, t_end, grid, seed, rates=torch.tensor(np.exp(lp), device=DEV))
            mm, _, _, _ = ssa.run_device(model, N, t_end, grid, seed, rates=torch.tensor(np.exp(lm), device=DEV))
            fd[j] = float((w * (mp - mm)).sum()) / (2 * h)
        gg = g.cpu().numpy()
        grads.append(gg)
        diffs.append(gg - fd)
    model.close()
    diffs, grads = np.array(diffs), np.array(grads)
    mean_d = diffs.mean(axis=0)
    se = diffs.std(axis=0, ddof=1) / np.sqrt(len(diffs))
    scale = np.abs(grads.mean(axis=0))
    assert np.all(np.abs(mean_d) <= 4 * se + 1e-3 * scale), (mean_d, se, scale)
