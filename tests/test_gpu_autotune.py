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


def test_forward_autotune_reports_form_and_grid(ssa, tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("SSA_TUNE_FILE", str(cache))
    m = inputs.viral()
    N, t_end, G, seed = 40000, 5.0, 100, 6
    model = ssa.Model.from_dict(m)
    grid = torch.tensor(inputs.uniform_grid(t_end, G), device=DEV)
    m1, v1, _, _ = ssa.run_device(model, N, t_end, grid, seed)
    r = ssa.autotune_forward(model, N, t_end, grid, seed)
    assert r["form"] in ("none", "two_wave", "generations") and r["blocks"] >= 0
    m2, v2, _, s2 = ssa.run_device(model, N, t_end, grid, seed, with_stats=True)
    torch.cuda.synchronize()
    assert torch.equal(m1, m2) and torch.equal(v1, v2)
    if r["form"] != "none":
        assert s2["form"] == r["form"]
    if r["blocks"]:
        assert s2["blocks"] == r["blocks"]
    entries = json.loads(cache.read_text())["entries"]
    e = [v for k, v in entries.items() if "|jit|S4|M9|G128|N65536|" in k and not k.startswith("bwd|")]
    assert len(e) == 1 and "form" in e[0] and "blocks" in e[0]
    model.close()


def test_backward_autotune_keeps_the_gradient(ssa, tmp_path, monkeypatch):
    """The backward tuner times the launch forms (two-wave blocks, generations, refilled
    lanes) and grids; the gradient after tuning is the same bits, and the next call runs
    the chosen form."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("SSA_TUNE_FILE", str(cache))
    m = inputs.viral()
    N, t_end, G, seed = 30000, 5.0, 200, 8
    model = ssa.Model.from_dict(m)
    grid = torch.tensor(inputs.uniform_grid(t_end, G), device=DEV)
    w = torch.tensor(np.random.default_rng(3).normal(size=(G, 4)), device=DEV)
    mean, _, _, _ = ssa.run_device(model, N, t_end, grid, seed)
    g1, _ = ssa.backward_device(model, N, t_end, grid, seed, w, mean)
    r = ssa.autotune_backward(model, N, t_end, grid, seed)
    assert r["form"] in ("none", "two_wave", "generations", "refill")
    assert r["best_ms"] > 0 and r["best_ms"] <= r["default_ms"] * 1.0001
    g2, s2 = ssa.backward_device(model, N, t_end, grid, seed, w, mean, with_stats=True)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    if r["form"] != "none":
        assert s2["form"] == r["form"]
    entries = json.loads(cache.read_text())["entries"]
    assert any(k.startswith("bwd|") and "|jit|S4|M9|G256|N32768|" in k for k in entries)
    model.close()


_CHILD = r"""
import hashlib, json, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_1007_1768_amd import inputs, ssa
m = inputs.viral()
N, t_end, G, seed = 3000, 5.0, 120, 9
model = ssa.Model.from_dict(m)
grid = torch.tensor(inputs.uniform_grid(t_end, G), device="cuda:0")
w = torch.tensor(np.random.default_rng(4).normal(size=(G, 4)), device="cuda:0")
mean, _, _, _ = ssa.run_device(model, N, t_end, grid, seed)
g, st = ssa.backward_device(model, N, t_end, grid, seed, w, mean, with_stats=True)
torch.cuda.synchronize()
print(json.dumps({"form": st["form"], "blocks": st["blocks"], "grad": g.cpu().numpy().tobytes().hex()}))
"""


@pytest.mark.parametrize("form,blocks", [("refill", 7), ("generations", 5), ("two_wave", 3)])
def test_tuned_backward_form_from_cache(ssa, tmp_path, monkeypatch, form, blocks):
    """A tuned launch read from the cache file by a later process: the backward runs in that
    form on that many blocks and gives the same gradient as the default launch."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    m = inputs.viral()
    N, t_end, G, seed = 3000, 5.0, 120, 9
    model = ssa.Model.from_dict(m)
    grid = torch.tensor(inputs.uniform_grid(t_end, G), device=DEV)
    w = torch.tensor(np.random.default_rng(4).normal(size=(G, 4)), device=DEV)
    mean, _, _, _ = ssa.run_device(model, N, t_end, grid, seed)
    g1, s1 = ssa.backward_device(model, N, t_end, grid, seed, w, mean, with_stats=True)
    torch.cuda.synchronize()
    # the key of this problem as the tuner writes it (tuned in this process into a scratch file)
    scratch = tmp_path / "scratch.json"
    monkeypatch.setenv("SSA_TUNE_FILE", str(scratch))
    ssa.autotune_backward(model, N, t_end, grid, seed)
    key = [k for k in json.loads(scratch.read_text())["entries"] if k.startswith("bwd|")][0]
    model.close()
    cache = tmp_path / "tune.json"
    code = {"two_wave": 1, "generations": 2, "refill": 3}[form]
    cache.write_text('{\n  "entries": {\n    "%s": {"win_bytes": 0, "slab": -1, "form": %d, "blocks": %d, "ms": 1.0}\n'
                     '  }\n}\n' % (key, code, blocks))
    env = dict(os.environ, SSA_TUNE_FILE=str(cache))
    out = subprocess.run([sys.executable, "-c", _CHILD, root], env=env, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    r = json.loads(out.stdout.strip().splitlines()[-1])
    assert r["form"] == form and r["blocks"] == blocks, r
    assert bytes.fromhex(r["grad"]) == g1.cpu().numpy().tobytes()
