"""GPU checks of the device entry points captured into a HIP graph and replayed.

The step of a fit (forward moments and histogram, loss weights in torch, likelihood-ratio
backward) is captured once with torch.cuda.graph and replayed several times, with other
library calls and zeroed outputs between the replays: every replay must give the eager
step's results bit for bit (both sides run the same kernels in the same order), and the
eager results equal the oracle's.  Cases: a ragged count in two-wave launches, a count in
persistent launches, the variance weights, the Jacobian and covariance passes, and the
autograd functions captured with their backward.  Refusals: statistics under capture and a
network whose kernels were never compiled (SSA_E_INVALID, before any stream operation, so
the capture stays usable).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1007_1768_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
REPLAYS = 4


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1007_1768_amd import ssa as s
    s.load()
    return s


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _warm_then_capture(fn):
    """torch's recipe: run fn on a side stream first (compiles the network's kernels), then
    capture it on the graph's stream."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def _replay_and_compare(g, outs, want, between):
    for r in range(REPLAYS):
        for o in outs:
            o.zero_()
        between(r)
        g.replay()
        torch.cuda.synchronize()
        for o, x in zip(outs, want):
            assert torch.equal(o, x), (r, o, x)


STEP_CASES = {
    # N, t_end, G, seed, histogram: 47 work items (two-wave launches), then 4688 (persistent)
    "ragged_two_wave": (3000, 20.0, 200, 17, (1, 0, 1, 16)),
    "persistent": (300_000, 5.0, 500, 23, None),
}


@pytest.mark.parametrize("case", sorted(STEP_CASES))
@pytest.mark.parametrize("quad", [False, True])
def test_captured_step_replays_equal_eager_and_oracle(ssa, case, quad):
    N, t_end, G, seed, hist = STEP_CASES[case]
    m = inputs.viral()
    model = ssa.Model.from_dict(m)
    grid = _t(inputs.uniform_grid(t_end, G))
    prates = _t(inputs.perturbed_rates(m, 404))
    target, tvar, _, _ = ssa.run_device(model, N, t_end, grid, seed + 1, rates=prates)
    S, M = m["reac"].shape[1], m["reac"].shape[0]
    mean = torch.empty((G, S), dtype=torch.float64, device=DEV)
    var = torch.empty_like(mean)
    h = torch.empty((G, hist[3]), dtype=torch.int32, device=DEV) if hist else None
    w = torch.empty_like(mean)
    wv = torch.empty_like(mean)
    grad = torch.empty(M, dtype=torch.float64, device=DEV)
    print("graph step %s quad %s N %d G %d" % (case, quad, N, G), flush=True)

    def step():
        ssa.run_device(model, N, t_end, grid, seed, hist=hist, out=(mean, var, h))
        torch.sub(mean, target, out=w)
        w.mul_(2.0)
        if quad:
            torch.sub(var, tvar, out=wv)
            wv.mul_(2.0)
            ssa.backward_device(model, N, t_end, grid, seed, w, mean, out=grad, wv=wv, vhat=var)
        else:
            ssa.backward_device(model, N, t_end, grid, seed, w, mean, out=grad)

    step()
    torch.cuda.synchronize()
    outs = [mean, var, grad] + ([h] if hist else [])
    want = [o.clone() for o in outs]
    g = _warm_then_capture(step)
    other = torch.empty_like(mean), torch.empty_like(var), (torch.empty_like(h) if hist else None)

    def between(r):
        # eager library work between the replays (another seed, other buffers)
        ssa.run_device(model, 500, t_end, grid, 1000 + r, hist=hist, out=other)

    _replay_and_compare(g, outs, want, between)
    del g
    torch.cuda.synchronize()
    model.close()
    if case == "ragged_two_wave":
        grid_np = inputs.uniform_grid(t_end, G)
        st, ref = orc.run(m, N, t_end, grid_np, seed, hist=hist)
        assert st == 0
        assert np.array_equal(want[0].cpu().numpy(), ref["mean"]) and np.array_equal(want[1].cpu().numpy(), ref["var"])
        assert np.array_equal(want[3].cpu().numpy().astype(np.int64), ref["hist"].astype(np.int64))
        wn = want[0].cpu().numpy()
        w_np = 2.0 * (wn - target.cpu().numpy())
        if quad:
            wv_np = 2.0 * (want[1].cpu().numpy() - tvar.cpu().numpy())
            st, gref, l1 = orc.grad(m, N, t_end, grid_np, seed, w_np, wn, wv=wv_np, vhat=want[1].cpu().numpy())
        else:
            st, gref, l1 = orc.grad(m, N, t_end, grid_np, seed, w_np, wn)
        assert st == 0
        assert np.all(np.abs(want[2].cpu().numpy() - gref) <= 1e-12 * l1)


def test_captured_jacobian_and_covariance(ssa):
    m = inputs.viral()
    N, t_end, G, seed = 2000, 10.0, 41, 9
    model = ssa.Model.from_dict(m)
    grid = _t(inputs.uniform_grid(t_end, G))
    S, M = m["reac"].shape[1], m["reac"].shape[0]
    mj = torch.empty((G, S), dtype=torch.float64, device=DEV)
    vj = torch.empty_like(mj)
    jac = torch.empty((G, S, M), dtype=torch.float64, device=DEV)
    res = {}

    def fn():
        ssa.run_jacobian_device(model, N, t_end, grid, seed, out=(mj, vj, jac))
        res["cov"] = ssa.run_cov_device(model, N, t_end, grid, seed)

    fn()
    torch.cuda.synchronize()
    want = [mj.clone(), vj.clone(), jac.clone(), res["cov"][0].clone(), res["cov"][1].clone()]
    g = _warm_then_capture(fn)
    outs = [mj, vj, jac, res["cov"][0], res["cov"][1]]    # the captured call's own outputs
    _replay_and_compare(g, outs, want, lambda r: None)
    del g
    torch.cuda.synchronize()
    model.close()


def test_captured_autograd_step(ssa):
    """ssa_moments forward, a torch loss and loss.backward() captured as one graph: the
    replayed gradient equals the eager one."""
    m = inputs.viral()
    N, t_end, G, seed = 4000, 10.0, 101, 31
    model = ssa.Model.from_dict(m)
    grid = _t(inputs.uniform_grid(t_end, G))
    theta = _t(np.log(m["rates"])).requires_grad_(True)
    target = torch.full((G, m["reac"].shape[1]), 5.0, dtype=torch.float64, device=DEV)

    def fn():
        mean, var = ssa.ssa_moments(theta, model, N, t_end, grid, seed)
        loss = ((mean - target) ** 2).sum() + 1e-3 * var.sum()
        loss.backward()

    fn()
    torch.cuda.synchronize()
    want = theta.grad.clone()
    theta.grad = None
    g = _warm_then_capture(fn)
    for r in range(REPLAYS):
        theta.grad.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(theta.grad, want), (r, theta.grad, want)
    del g
    torch.cuda.synchronize()
    model.close()


def test_refusals_under_capture(ssa):
    m = inputs.viral()
    N, t_end, G, seed = 1000, 5.0, 21, 3
    model = ssa.Model.from_dict(m)
    grid = _t(inputs.uniform_grid(t_end, G))
    mean = torch.empty((G, 4), dtype=torch.float64, device=DEV)
    var = torch.empty_like(mean)
    ssa.run_device(model, N, t_end, grid, seed, out=(mean, var, None))
    fresh = dict(m)
    fresh["x0"] = np.array(m["x0"]) + 7            # a network source no call has compiled yet
    mfresh = ssa.Model.from_dict(fresh)
    torch.cuda.synchronize()
    errors = []
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        try:
            ssa.run_device(model, N, t_end, grid, seed, out=(mean, var, None), with_stats=True)
        except ssa.SSAError as e:
            errors.append(e.status)
        try:
            ssa.run_device(mfresh, N, t_end, grid, seed, out=(mean, var, None))
        except ssa.SSAError as e:
            errors.append(e.status)
        ssa.run_device(model, N, t_end, grid, seed, out=(mean, var, None))      # the capture is intact
    torch.cuda.synchronize()
    assert errors == [ssa.E_INVALID, ssa.E_INVALID], errors
    want = mean.clone()
    mean.zero_()
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(mean, want)
    del g
    torch.cuda.synchronize()
    model.close()
    mfresh.close()
