"""Pins of the oracle's rate laws (species-dependent rate constants, the infectivities
beta -/+ K F of Section 2.1) and of the HIV network built on them.

* A law driven by a species that no reaction changes is a constant rate: trajectories are
  bit-identical to the mass-action network with that constant (below, inside and above
  the clamp bounds).
* A birth rate min(max(c0 + k X, 0), hi) on X itself, with death d X: the oracle's mean and
  variance at t follow the chemical master equation of that one-species process (matrix
  exponential of its generator), within sampling error.
* The HIV network: U0 stays 1, counts stay non-negative, and the final state equals the
  initial state plus the fired counts times the net changes.
"""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import oracle as orc
from paper_1007_1768_amd import inputs


def _with_law(m, j, species, slope, lo=0.0, hi=np.inf):
    M = m["reac"].shape[0]
    laws = dict(species=np.full(M, -1, np.int32), slope=np.zeros(M), lo=np.zeros(M), hi=np.full(M, np.inf))
    laws["species"][j], laws["slope"][j], laws["lo"][j], laws["hi"][j] = species, slope, lo, hi
    m = dict(m)
    m["laws"] = laws
    return m


@pytest.mark.parametrize("slope,lo,hi", [(0.03, 0.0, np.inf), (-0.5, 0.05, np.inf), (0.2, 0.0, 0.4)])
def test_law_on_constant_species_is_mass_action(slope, lo, hi):
    # A -> B (law on C), B -> A; C is a catalyst no reaction changes (C = 7)
    base = inputs._model("cat", ["A", "B", "C"], [({"A": 1}, {"B": 1}, 0.3), ({"B": 1}, {"A": 1}, 0.2)], [40, 5, 7])
    law = _with_law(base, 0, 2, slope, lo, hi)
    c_eff = min(max(0.3 + slope * 7.0, lo), hi)
    plain = dict(base)
    plain["rates"] = np.array([c_eff, 0.2])
    grid = inputs.uniform_grid(10.0, 21)
    for i in range(20):
        s1, r1 = orc.trajectory(law, 3, i, 10.0, grid)
        s2, r2 = orc.trajectory(plain, 3, i, 10.0, grid)
        assert s1 == 0 and s2 == 0
        assert np.array_equal(r1["states"], r2["states"]) and r1["events"] == r2["events"]
        assert r1["t_last"] == r2["t_last"]


def test_state_dependent_birth_follows_the_master_equation():
    c0, k, hi, d = 2.0, 0.5, 6.0, 0.4
    m = _with_law(inputs._model("bd", ["X"], [({}, {"X": 1}, c0), ({"X": 1}, {}, d)], [0]), 0, 0, k, 0.0, hi)
    t = 6.0
    n_max = 120
    Q = np.zeros((n_max + 1, n_max + 1))
    for x in range(n_max + 1):
        b = min(max(c0 + k * x, 0.0), hi)
        if x < n_max:
            Q[x, x + 1] = b
        if x > 0:
            Q[x, x - 1] = d * x
        Q[x, x] = -Q[x].sum()
    p0 = np.zeros(n_max + 1)
    p0[0] = 1.0
    p = p0 @ expm(Q * t)
    xs = np.arange(n_max + 1)
    mean, var = (p * xs).sum(), (p * xs ** 2).sum() - (p * xs).sum() ** 2
    N = 20000
    st, r = orc.run(m, N, t, np.array([t]), 12)
    assert st == 0
    se = np.sqrt(var / N)
    assert abs(r["mean"][0, 0] - mean) < 5 * se, (r["mean"][0, 0], mean, se)
    assert abs(r["var"][0, 0] - var) < 5 * var * np.sqrt(2.0 / (N - 1)), (r["var"][0, 0], var)


def test_hiv_invariants():
    m = inputs.hiv()
    grid = inputs.uniform_grid(1.0, 11)
    S = m["reac"].shape[1]
    nu = (m["prod"] - m["reac"]).astype(np.int64)
    for i in range(4):
        st, r = orc.trajectory(m, 5, i, 1.0, grid)
        assert st == 0
        assert np.all(r["states"][:, 0] == 1)              # U0 is only a catalyst
        assert np.all(r["states"] >= 0)
        x_end = np.asarray(m["x0"], np.int64) + r["n_fired"].astype(np.int64) @ nu
        assert np.array_equal(x_end, r["states"][-1].astype(np.int64))
        assert r["events"] == int(r["n_fired"].sum()) and r["events"] > 100
