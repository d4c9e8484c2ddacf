"""The two-wave launches (one wave simulates a generation of 64 trajectories, the other
computes its draws into an LDS ring): the forward, the backward and the event log of the
adaptive memory give the same bits as the one-wave kernels, including when lanes wait on
the selective-memory window (so they consume draws at different paces), when a block runs
several generations, when the event log runs in epochs (lanes resume at their own draws),
for ragged and tiny trajectory counts, with the histogram and with variance weights."""
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


def _both(monkeypatch, fn):
    """fn() with the two-wave launches, then with them turned off."""
    monkeypatch.delenv("SSA_DRAW_WAVE", raising=False)
    a = fn()
    monkeypatch.setenv("SSA_DRAW_WAVE", "0")
    b = fn()
    monkeypatch.delenv("SSA_DRAW_WAVE", raising=False)
    return a, b


CASES = [
    # (trajectories, t_end, grid points, seed, window bytes or None, block cap or None)
    (3000, 20.0, 400, 11, None, None),
    (3000, 20.0, 2000, 12, 2048, None),      # small window over a dense grid: lanes wait often
    (1000, 15.0, 300, 13, None, 3),          # 16 work items (the last ragged) on 3 blocks
    (5, 30.0, 100, 14, None, None),          # one work item of 5 lanes
    (200, 25.0, 250, 15, 2048, 1),           # one block running every generation
]


@pytest.mark.parametrize("N,t_end,G,seed,win,cap", CASES)
def test_forward_same_bits(ssa, monkeypatch, N, t_end, G, seed, win, cap):
    if win:
        monkeypatch.setenv("SSA_WIN_BYTES", str(win))
    if cap:
        monkeypatch.setenv("SSA_DRAW_WAVE_BLOCKS", str(cap))
    model = ssa.Model.from_dict(inputs.viral())
    grid = torch.tensor(inputs.uniform_grid(t_end, G), device=DEV)
    for hist in (None, (1, 0, 1, 32)):
        def run():
            m, v, h, st = ssa.run_device(model, N, t_end, grid, seed, hist=hist, with_stats=True)
            torch.cuda.synchronize()
            return m, v, h, st
        (m1, v1, h1, s1), (m2, v2, h2, s2) = _both(monkeypatch, run)
        assert s1["flags"] == 0 and s1["events"] == s2["events"] and s1["max_steps"] == s2["max_steps"]
        assert torch.equal(m1, m2) and torch.equal(v1, v2)
        if hist is not None:
            assert torch.equal(h1, h2)
    model.close()


@pytest.mark.parametrize("N,t_end,G,seed,win,cap", CASES)
def test_backward_same_bits(ssa, monkeypatch, N, t_end, G, seed, win, cap):
    if cap:
        monkeypatch.setenv("SSA_DRAW_WAVE_BLOCKS", str(cap))
    model = ssa.Model.from_dict(inputs.viral())
    grid = torch.tensor(inputs.uniform_grid(t_end, G), device=DEV)
    mean, var, _, _ = ssa.run_device(model, N, t_end, grid, seed)
    gen = torch.Generator().manual_seed(seed)
    w = torch.randn(G, model.S, generator=gen, dtype=torch.float64).to(DEV)
    wv = torch.randn(G, model.S, generator=gen, dtype=torch.float64).to(DEV) * 1e-3
    for quad in (False, True):
        def run():
            if quad:
                g, st = ssa.backward_device(model, N, t_end, grid, seed, w, mean, wv=wv, vhat=var, with_stats=True)
            else:
                g, st = ssa.backward_device(model, N, t_end, grid, seed, w, mean, with_stats=True)
            torch.cuda.synchronize()
            return g, st
        (g1, s1), (g2, s2) = _both(monkeypatch, run)
        assert s1["events"] == s2["events"] and s1["flags"] == s2["flags"]
        assert torch.equal(g1, g2), (g1 - g2).abs().max().item()
    model.close()


@pytest.mark.parametrize("N,t_end,seed,k,epochs,cap", [
    (1500, 10.0, 21, 50, False, None),
    (1500, 10.0, 22, 50, True, None),     # epochs of 4096 records: lanes resume at their own draws
    (300, 6.0, 23, 7, True, 2),           # several generations per block, in epochs
])
def test_event_log_same_bits(ssa, monkeypatch, N, t_end, seed, k, epochs, cap):
    if epochs:
        monkeypatch.setenv("SSA_ADAPTIVE_RECORDS", "4096")
    if cap:
        monkeypatch.setenv("SSA_DRAW_WAVE_BLOCKS", str(cap))
    model = ssa.Model.from_dict(inputs.viral())

    def run():
        out = ssa.adaptive_device(model, N, t_end, seed, k, with_y=True, with_stats=True)
        torch.cuda.synchronize()
        return out
    a, b = _both(monkeypatch, run)
    assert a["stats"]["events"] == b["stats"]["events"] and a["stats"]["flags"] == b["stats"]["flags"]
    for key in ("xy_time", "xy_mean", "xy_var", "y_time", "y_mean", "y_var"):
        assert torch.equal(a[key], b[key]), key
    model.close()
