"""GPU parity of the likelihood-ratio gradient of a loss on the grid variances (and means).

The re-simulating backward with variance weights (prefix table with the quadratic columns)
must match the oracle's long-double estimator within 1e-12 of its scale (the size of the
terms as the kernel evaluates them: |w (X - m)| and |wv| (X^2 + 2|X m| + m^2 + |v|), times
|z_j|), with the specialised and the table-driven kernels; with wv = 0 it reproduces the
mean-only backward bit for bit; the autograd function returns both gradients.
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


CASES = {
    "viral": (inputs.viral, 300, 5.0, 21, 6),
    "immigration_death": (lambda: inputs.immigration_death(10.0, 0.1, 0), 500, 30.0, 16, 9),
}


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("case", sorted(CASES))
def test_variance_gradient_matches_oracle(ssa, kernel, case):
    make, N, t_end, G, seed = CASES[case]
    m = make()
    grid = inputs.uniform_grid(t_end, G)
    st, ref = orc.run(m, N, t_end, grid, seed)
    assert st == 0
    rng = np.random.default_rng(seed)
    w = rng.normal(size=ref["mean"].shape)
    wv = rng.normal(size=ref["mean"].shape) / (1.0 + ref["var"])
    model = ssa.Model.from_dict(m)
    g, _ = ssa.backward_device(model, N, t_end, _t(grid), seed, _t(w), _t(ref["mean"]), wv=_t(wv),
                               vhat=_t(ref["var"]))
    torch.cuda.synchronize()
    model.close()
    st, gref, l1 = orc.grad(m, N, t_end, grid, seed, w, ref["mean"], wv=wv, vhat=ref["var"])
    assert st == 0
    d = np.abs(g.cpu().numpy() - gref)
    assert np.all(d <= 1e-12 * l1), (d / np.maximum(l1, 1e-300)).max()


def test_zero_variance_weights_are_the_mean_backward(ssa):
    m = inputs.viral()
    N, t_end, G, seed = 200, 4.0, 17, 3
    grid = inputs.uniform_grid(t_end, G)
    model = ssa.Model.from_dict(m)
    mean, var, _, _ = ssa.run_device(model, N, t_end, _t(grid), seed)
    w = _t(np.random.default_rng(1).normal(size=(G, 4)))
    g0, _ = ssa.backward_device(model, N, t_end, _t(grid), seed, w, mean)
    g1, _ = ssa.backward_device(model, N, t_end, _t(grid), seed, w, mean, wv=torch.zeros_like(var), vhat=var)
    torch.cuda.synchronize()
    model.close()
    assert torch.equal(g0, g1)


def test_moments_autograd(ssa):
    m = inputs.viral()
    N, t_end, G, seed = 200, 4.0, 9, 5
    grid = _t(inputs.uniform_grid(t_end, G))
    model = ssa.Model.from_dict(m)
    lr = torch.tensor(np.log(m["rates"]), dtype=torch.float64, device=DEV, requires_grad=True)
    mean, var = ssa.ssa_moments(lr, model, N, t_end, grid, seed)
    cm = torch.linspace(0.1, 1.0, G * 4, dtype=torch.float64, device=DEV).reshape(G, 4)
    cv = torch.linspace(-0.01, 0.02, G * 4, dtype=torch.float64, device=DEV).reshape(G, 4)
    (mean * cm).sum().add((var * cv).sum()).backward()
    g, _ = ssa.backward_device(model, N, t_end, grid, seed, cm, mean.detach(), log_rates=lr.detach(), wv=cv,
                               vhat=var.detach())
    torch.cuda.synchronize()
    model.close()
    assert torch.equal(lr.grad, g)


@pytest.mark.parametrize("M", [9, 600])
def test_variance_gradient_64_chunk_order(ssa, M):
    """The one-trajectory-per-wave backward (registers up to 8 reactions per lane, LDS rows
    above) with variance weights, against the oracle in the same sum order."""
    if M == 9:
        m = dict(inputs.viral())
        m["sum_order"] = "block64"
        N, t_end, G, seed = 200, 4.0, 13, 8
    else:
        m = inputs.wide_network(M)
        N, t_end, G, seed = 96, 0.5, 11, 13
    grid = inputs.uniform_grid(t_end, G)
    st, ref = orc.run(m, N, t_end, grid, seed)
    assert st == 0
    rng = np.random.default_rng(M)
    w = rng.normal(size=ref["mean"].shape)
    wv = rng.normal(size=ref["mean"].shape) / (1.0 + ref["var"])
    model = ssa.Model.from_dict(m)
    g, _ = ssa.backward_device(model, N, t_end, _t(grid), seed, _t(w), _t(ref["mean"]), wv=_t(wv),
                               vhat=_t(ref["var"]))
    torch.cuda.synchronize()
    model.close()
    st, gref, l1 = orc.grad(m, N, t_end, grid, seed, w, ref["mean"], wv=wv, vhat=ref["var"])
    assert st == 0
    d = np.abs(g.cpu().numpy() - gref)
    assert np.all(d <= 1e-12 * l1 + 1e-300), (d / np.maximum(l1, 1e-300)).max()
