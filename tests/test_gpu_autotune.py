"""The forward autotuner: it times the launch configurations on the caller's problem,
keeps the fastest for later calls and in the SSA_TUNE_FILE cache, and never changes the
results."""
import json

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


@pytest.mark.parametrize("generic", [False, True])
def test_autotune_keeps_results_and_writes_cache(ssa, tmp_path, monkeypatch, generic):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("SSA_TUNE_FILE", str(cache))
    if generic:
        monkeypatch.setenv("SSA_KERNEL", "generic")
    m = inputs.viral()
    N, t_end, G, seed = 2000, 10.0, 200, 3
    model = ssa.Model.from_dict(m)
    grid = torch.tensor(inputs.uniform_grid(t_end, G), device=DEV)
    m1, v1, _, s1 = ssa.run_device(model, N, t_end, grid, seed, with_stats=True)
    r = ssa.autotune_forward(model, N, t_end, grid, seed)
    assert r["best_ms"] > 0 and r["best_ms"] <= r["default_ms"] * 1.0001
    assert r["win_bytes"] in (0, 2048, 4096, 8192, 16384) and r["slab"] in (-1, 0, 1)
    m2, v2, _, s2 = ssa.run_device(model, N, t_end, grid, seed, with_stats=True)
    torch.cuda.synchronize()
    assert torch.equal(m1, m2) and torch.equal(v1, v2) and s1["events"] == s2["events"]
    entries = json.loads(cache.read_text())["entries"]
    kind = "table" if generic else "jit"
    keys = [k for k in entries if ("|%s|S4|M9|G256|N2048|" % kind) in k]
    assert len(keys) == 1
    assert entries[keys[0]]["win_bytes"] == r["win_bytes"] and entries[keys[0]]["slab"] == r["slab"]
    model.close()


def test_batch_autotune_keeps_results(ssa):
    """Batch autotuning times the window sizes on scratch outputs (the caller's last outputs
    stay as they were), rebuilds the graph with the fastest and changes no result."""
    nets = inputs.random_networks(count=8, G=100)
    models = [ssa.Model.from_dict(n) for n in nets]
    n_traj = [min(n["n_traj"], 2048) for n in nets]
    bt = ssa.Batch(models, n_traj, [n["t_end"] for n in nets], [n["grid"] for n in nets],
                   [n["seed"] for n in nets])
    m1, v1, _ = bt.run(DEV)
    torch.cuda.synchronize()
    keep = [m.clone() for m in m1]
    r = bt.autotune()
    torch.cuda.synchronize()
    assert r["win_bytes"] in (0, 2048, 4096, 8192, 16384)
    assert r["best_ms"] > 0 and r["best_ms"] <= r["default_ms"] * 1.0001
    assert all(torch.equal(a, b) for a, b in zip(m1, keep))
    m2, v2, _ = bt.run(DEV)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(m1, m2))
    assert all(torch.equal(a, b) for a, b in zip(v1, v2))
    bt.close()
    for m in models:
        m.close()
