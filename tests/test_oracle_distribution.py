"""Distributional pins for the oracle's simulation (independent of any implementation detail).

* Immigration-death (0 -> X at c1, X -> 0 at c2 X, X0 = 0): X(t) is Poisson with mean
  (c1/c2)(1 - exp(-c2 t)), so mean = variance at every grid point, and the whole
  distribution is known.
* Pure death (X -> 0 at c X): X(t) ~ Binomial(X0, exp(-c t)).
* Isomerisation A <-> B: A(t) ~ Binomial(n, p(t)) with the two-state Markov chain's p(t).
* Tiny networks whose chemical master equation is solved by brute force (oracle/cme.py):
  homodimerisation 2A <-> B (pins the x(x-1)/2 pair count), heterodimerisation
  A + B <-> C, and a two-species catalytic birth-death process.

Each check uses fixed seeds, compares means within 5 standard errors, variances within 5
standard errors of the sample variance (from the fourth central moment), and whole
marginal distributions with a chi-square test at the 1e-6 level.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import cme
from oracle import oracle as orc
from paper_1007_1768_amd import inputs


def _z_mean(mean, mu, var, N):
    se = math.sqrt(max(var, 1e-300) / N)
    return abs(mean - mu) / se


def _z_var(v, var, mu4, N):
    se = math.sqrt(max(mu4 - var * var, 1e-300) / N)
    return abs(v - var) / se


def _chi2_ok(counts, probs, N):
    """Pool the tail bins so that every expected count is at least 5; test at p = 1e-6."""
    exp = probs * N
    obs = counts.astype(np.float64)
    pooled_o, pooled_e = [], []
    acc_o = acc_e = 0.0
    for o, e in zip(obs, exp):
        acc_o += o
        acc_e += e
        if acc_e >= 5.0:
            pooled_o.append(acc_o)
            pooled_e.append(acc_e)
            acc_o = acc_e = 0.0
    if pooled_e:
        pooled_o[-1] += acc_o
        pooled_e[-1] += acc_e
    o = np.array(pooled_o)
    e = np.array(pooled_e)
    e *= o.sum() / e.sum()
    chi = float(((o - e) ** 2 / e).sum())
    df = len(o) - 1
    return chi <= stats.chi2.ppf(1 - 1e-6, df), chi, df


def test_immigration_death_poisson_moments_and_distribution():
    m = inputs.immigration_death()
    N, t_end, G = 20000, 100.0, 101
    grid = inputs.uniform_grid(t_end, G)
    st, out = orc.run(m, N, t_end, grid, seed=101, hist=(0, 0, 1, 256))
    assert st == orc.OK
    lam = 100.0 * (1.0 - np.exp(-0.1 * grid))
    assert out["mean"][0, 0] == 0.0 and out["var"][0, 0] == 0.0
    for g in range(1, G):
        L = lam[g]
        assert _z_mean(out["mean"][g, 0], L, L, N) < 5.0, g
        assert _z_var(out["var"][g, 0], L, L + 3 * L * L, N) < 5.0, g
    for t in (10, 50, 100):
        g = int(t)
        L = lam[g]
        probs = stats.poisson.pmf(np.arange(256), L)
        probs[-1] += stats.poisson.sf(255, L)
        ok, chi, df = _chi2_ok(out["hist"][g], probs, N)
        assert ok, (t, chi, df)
    # histogram rows count every trajectory
    assert (out["hist"].sum(axis=1) == N).all()


def test_pure_death_binomial():
    m = inputs._model("pure_death", ["X"], [({"X": 1}, {}, 0.5)], [50])
    N, t_end = 20000, 6.0
    grid = inputs.uniform_grid(t_end, 13)
    st, out = orc.run(m, N, t_end, grid, seed=7, hist=(0, 0, 1, 51))
    assert st == orc.OK
    for g, t in enumerate(grid):
        p = math.exp(-0.5 * t)
        mu, var = 50 * p, 50 * p * (1 - p)
        if var == 0:
            assert out["mean"][g, 0] == 50 and out["var"][g, 0] == 0
            continue
        dist = stats.binom(50, p)
        mu4 = dist.moment(4) - 4 * mu * dist.moment(3) + 6 * mu * mu * dist.moment(2) - 3 * mu**4
        assert _z_mean(out["mean"][g, 0], mu, var, N) < 5.0
        assert _z_var(out["var"][g, 0], var, mu4, N) < 5.0
        ok, chi, df = _chi2_ok(out["hist"][g], dist.pmf(np.arange(51)), N)
        assert ok, (t, chi, df)


def test_isomerisation_binomial_and_conservation():
    c1, c2, n = 1.0, 0.5, 20
    m = inputs._model("iso", ["A", "B"], [({"A": 1}, {"B": 1}, c1), ({"B": 1}, {"A": 1}, c2)], [n, 0])
    N, t_end = 20000, 4.0
    grid = inputs.uniform_grid(t_end, 9)
    st, out = orc.run(m, N, t_end, grid, seed=9, hist=(0, 0, 1, n + 1))
    assert st == orc.OK
    # A + B is conserved in every trajectory: its sample variance is 0, so var(A) == var(B)
    assert np.all(out["mean"].sum(axis=1) == n)
    assert np.array_equal(out["var"][:, 0], out["var"][:, 1])
    for g, t in enumerate(grid):
        p = c2 / (c1 + c2) + c1 / (c1 + c2) * math.exp(-(c1 + c2) * t)
        dist = stats.binom(n, p)
        mu, var = dist.mean(), dist.var()
        if var == 0:
            continue
        mu4 = float(stats.binom(n, p).expect(lambda k: (k - mu) ** 4))
        assert _z_mean(out["mean"][g, 0], mu, var, N) < 5.0
        assert _z_var(out["var"][g, 0], var, mu4, N) < 5.0
        ok, chi, df = _chi2_ok(out["hist"][g], dist.pmf(np.arange(n + 1)), N)
        assert ok, (t, chi, df)


CME_CASES = [
    # homodimerisation: the pair count x(x-1)/2 is what the CME uses for 2A
    ("homodimer", ["A", "B"], [({"A": 2}, {"B": 1}, 0.1), ({"B": 1}, {"A": 2}, 1.0)], [20, 0], [20, 10], 3.0),
    ("heterodimer", ["A", "B", "C"], [({"A": 1, "B": 1}, {"C": 1}, 0.05), ({"C": 1}, {"A": 1, "B": 1}, 0.5)],
     [15, 10, 0], [15, 10, 10], 3.0),
    ("catalytic_birth_death", ["A", "B"],
     [({}, {"A": 1}, 5.0), ({"A": 1}, {}, 0.5), ({"A": 1}, {"A": 1, "B": 1}, 1.0), ({"B": 1}, {}, 0.2)],
     [0, 0], [45, 160], 6.0),
    # dimer decay 2A -> 0 from 30 plus an inflow: nonlinear, pins order-2 handling once more
    ("dimer_decay_inflow", ["A"], [({}, {"A": 1}, 2.0), ({"A": 2}, {}, 0.05)], [30], [80], 5.0),
]


# A birth-death process written as 40 inflow and 40 degradation reactions of a fifth of
# the rates each plus a catalytic second species (M = 81 > 64): in the 64-chunk sum order
# two reactions share a chunk, so a chunk-offset slip would bias birth against death.
_SPLIT = ([({}, {"A": 1}, 4.0 / 40)] * 40 + [({"A": 1}, {}, 0.5 / 40)] * 40 +
          [({"A": 1}, {"A": 1, "B": 1}, 0.3)])
CME_CASES_BLOCK64 = [
    ("split_birth_death_block64", ["A", "B"], _SPLIT, [0, 0], [40, 60], 4.0),
    ("homodimer_block64", ["A", "B"], CME_CASES[0][2], [20, 0], [20, 10], 3.0),
]


@pytest.mark.parametrize("case", CME_CASES + CME_CASES_BLOCK64,
                         ids=[c[0] for c in CME_CASES + CME_CASES_BLOCK64])
def test_against_master_equation(case):
    name, species, reactions, x0, caps, t_end = case
    m = inputs._model(name, species, reactions, x0)
    if name.endswith("_block64"):
        m["sum_order"] = "block64"
    grid = inputs.uniform_grid(t_end, 7)
    sol = cme.solve(m, caps, grid)
    assert np.all(sol["leak"] < 1e-9), sol["leak"]
    N = 20000
    S = len(species)
    for s in range(S):
        nb = caps[s] + 1
        st, out = orc.run(m, N, t_end, grid, seed=1000 + s, hist=(s, 0, 1, nb))
        assert st == orc.OK
        for g in range(len(grid)):
            vals, probs = cme.marginal(sol, s, g)
            mu = float((vals * probs).sum())
            var = float(((vals - mu) ** 2 * probs).sum())
            if var < 1e-12:
                assert out["var"][g, s] == 0.0
                assert out["mean"][g, s] == round(mu)
                continue
            mu4 = float(((vals - mu) ** 4 * probs).sum())
            assert _z_mean(out["mean"][g, s], mu, var, N) < 5.0, (name, s, g)
            assert _z_var(out["var"][g, s], var, mu4, N) < 5.0, (name, s, g)
            p = np.zeros(nb)
            p[:len(probs)] = probs[:nb]
            ok, chi, df = _chi2_ok(out["hist"][g], p, N)
            assert ok, (name, s, g, chi, df)


def test_covariance_pins():
    """Species covariance: its diagonal is the pinned variance; a conserved total makes
    cov(A, B) = -var(A) exactly (every trajectory has A + B = n); two decoupled
    birth-death species have covariance zero within sampling error; symmetry."""
    n = 20
    iso = inputs._model("iso", ["A", "B"], [({"A": 1}, {"B": 1}, 1.0), ({"B": 1}, {"A": 1}, 0.5)], [n, 0])
    grid = inputs.uniform_grid(4.0, 9)
    st, mean, cov = orc.covariance(iso, 3000, 4.0, grid, seed=5)
    assert st == orc.OK
    st, ref = orc.run(iso, 3000, 4.0, grid, seed=5)
    assert np.array_equal(mean, ref["mean"])
    assert np.array_equal(cov[:, 0, 0], ref["var"][:, 0]) and np.array_equal(cov[:, 1, 1], ref["var"][:, 1])
    assert np.array_equal(cov[:, 0, 1], -cov[:, 0, 0]) and np.array_equal(cov[:, 0, 1], cov[:, 1, 0])
    two = inputs._model("two", ["X", "Y"], [({}, {"X": 1}, 5.0), ({"X": 1}, {}, 0.5),
                                            ({}, {"Y": 1}, 3.0), ({"Y": 1}, {}, 0.2)], [0, 0])
    N = 20000
    st, mean, cov = orc.covariance(two, N, 10.0, np.array([10.0]), seed=6)
    assert st == orc.OK
    # sample covariance of independent variables: standard error sqrt(var_x var_y / N)
    se = math.sqrt(cov[0, 0, 0] * cov[0, 1, 1] / N)
    assert abs(cov[0, 0, 1]) < 5 * se
