"""GPU checks of the boundary's device-side inputs.

* log rate constants: ssa_rates_from_log gives the oracle's e^theta bit for bit (over the
  whole accepted range, at its ends and for invalid values); ssa_run_device and
  ssa_backward_device with log_rates equal the oracle run with those rate constants
  (moments bit-exact, gradient within 1e-12 of its L1 scale); rates and log_rates together
  are rejected;
* device grids: a reversed, NaN or beyond-t_end grid and a NaN or too large log rate refuse
  the run on the device -- SSA_E_INVALID when statistics are requested, NaN moments,
  Jacobian, covariance and gradient, all-ones histogram counts -- and a valid call right
  after a refused one gives the oracle's results again.
"""
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


def test_rates_from_log_bitwise_equal_to_oracle(ssa):
    rng = np.random.default_rng(23)
    th = np.concatenate([rng.uniform(-708.0, 709.0, 3000), rng.normal(0.0, 4.0, 3000),
                         np.log(inputs.viral()["rates"]),
                         [0.0, -708.0, 709.0, -708.0000001, -1e4, -np.inf, 709.0000001, np.inf, np.nan, 1e-300]])
    ln2 = np.log(2.0)
    ks = np.arange(-1020, 1022, 5)
    th = np.concatenate([th, (ks + 0.5) * ln2, np.nextafter((ks + 0.5) * ln2, np.inf)])
    got = ssa.rates_from_log(_t(th)).cpu().numpy()
    want = orc.exp_rates(th)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    assert np.array_equal(got[ok].view(np.uint64), want[ok].view(np.uint64))


def test_log_rates_forward_and_backward_match_oracle(ssa):
    m = inputs.viral()
    N, t_end, G, seed = 500, 10.0, 51, 31
    grid = inputs.uniform_grid(t_end, G)
    theta = np.log(m["rates"]) + np.random.default_rng(5).normal(0.0, 0.1, 9)
    c = orc.exp_rates(theta)
    st, ref = orc.run(m, N, t_end, grid, seed, rates=c)
    assert st == 0
    model = ssa.Model.from_dict(m)
    mean, var, _, sf = ssa.run_device(model, N, t_end, _t(grid), seed, log_rates=_t(theta), with_stats=True)
    w = np.random.default_rng(6).normal(size=ref["mean"].shape)
    g, sb = ssa.backward_device(model, N, t_end, _t(grid), seed, _t(w), _t(ref["mean"]), log_rates=_t(theta),
                                with_stats=True)
    torch.cuda.synchronize()
    assert sf["events"] == ref["events"] == sb["events"]
    assert np.array_equal(mean.cpu().numpy(), ref["mean"]) and np.array_equal(var.cpu().numpy(), ref["var"])
    st, gref, l1 = orc.grad(m, N, t_end, grid, seed, w, ref["mean"], rates=c)
    assert st == 0
    assert np.all(np.abs(g.cpu().numpy() - gref) <= 1e-12 * l1)
    with pytest.raises(ssa.SSAError) as e:
        ssa.run_device(model, N, t_end, _t(grid), seed, rates=_t(c), log_rates=_t(theta))
    assert e.value.status == ssa.E_INVALID
    model.close()


def _bad_grids(t_end, G):
    good = inputs.uniform_grid(t_end, G)
    nan = good.copy()
    nan[G // 2] = np.nan
    beyond = good.copy()
    beyond[-1] = np.nextafter(t_end, np.inf)
    neg = good.copy()
    neg[0] = -1e-9
    return {"reversed": good[::-1].copy(), "nan": nan, "beyond_t_end": beyond, "negative": neg}


@pytest.mark.parametrize("kind", ["reversed", "nan", "beyond_t_end", "negative"])
def test_invalid_device_grid_refuses_the_run(ssa, kind):
    m = inputs.viral()
    N, t_end, G, seed = 300, 5.0, 41, 3
    bad = _t(_bad_grids(t_end, G)[kind])
    model = ssa.Model.from_dict(m)
    print("grid %s" % kind, flush=True)
    with pytest.raises(ssa.SSAError) as e:
        ssa.run_device(model, N, t_end, bad, seed, hist=(1, 0, 1, 8), with_stats=True)
    assert e.value.status == ssa.E_INVALID
    # without statistics the call is asynchronous and the outputs say it
    mean, var, h, _ = ssa.run_device(model, N, t_end, bad, seed, hist=(1, 0, 1, 8))
    w = torch.ones((G, 4), dtype=torch.float64, device=DEV)
    g, _ = ssa.backward_device(model, N, t_end, bad, seed, w, w)
    mj, vj, jac, _ = ssa.run_jacobian_device(model, N, t_end, bad, seed)
    mc, cov, _ = ssa.run_cov_device(model, N, t_end, bad, seed)
    torch.cuda.synchronize()
    for x in (mean, var, g, mj, vj, jac, mc, cov):
        assert torch.isnan(x).all()
    assert bool((h == -1).all())          # 0xffffffff counts, read back as int32
    with pytest.raises(ssa.SSAError) as e:
        ssa.backward_device(model, N, t_end, bad, seed, w, w, with_stats=True)
    assert e.value.status == ssa.E_INVALID
    # the next valid call is unaffected
    grid = inputs.uniform_grid(t_end, G)
    mean, var, _, st = ssa.run_device(model, N, t_end, _t(grid), seed, with_stats=True)
    torch.cuda.synchronize()
    s2, ref = orc.run(m, N, t_end, grid, seed)
    assert s2 == 0 and st["events"] == ref["events"]
    assert np.array_equal(mean.cpu().numpy(), ref["mean"])
    model.close()


@pytest.mark.parametrize("bad_theta", [np.nan, 709.5, np.inf])
def test_invalid_log_rate_refuses_the_run(ssa, bad_theta):
    m = inputs.viral()
    N, t_end, G, seed = 200, 5.0, 21, 4
    grid = _t(inputs.uniform_grid(t_end, G))
    theta = np.log(m["rates"])
    theta[3] = bad_theta
    model = ssa.Model.from_dict(m)
    with pytest.raises(ssa.SSAError) as e:
        ssa.run_device(model, N, t_end, grid, seed, log_rates=_t(theta), with_stats=True)
    assert e.value.status == ssa.E_INVALID
    w = torch.ones((G, 4), dtype=torch.float64, device=DEV)
    g, _ = ssa.backward_device(model, N, t_end, grid, seed, w, w, log_rates=_t(theta))
    torch.cuda.synchronize()
    assert torch.isnan(g).all()
    # a theta below the normal range switches the reaction off (c = 0) and is valid
    theta[3] = -800.0
    rates = orc.exp_rates(theta)
    assert rates[3] == 0.0
    mean, _, _, st = ssa.run_device(model, N, t_end, grid, seed, log_rates=_t(theta), with_stats=True)
    torch.cuda.synchronize()
    s2, ref = orc.run(m, N, t_end, inputs.uniform_grid(t_end, G), seed, rates=rates)
    assert s2 == 0 and st["events"] == ref["events"]
    assert np.array_equal(mean.cpu().numpy(), ref["mean"])
    model.close()
