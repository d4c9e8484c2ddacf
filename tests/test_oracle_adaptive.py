"""Pins of the oracle's adaptive selective memory (Avg-Y over the union of event times,
Avg-XY over groups of successive Avg-Y points; Section 3.2.1, Figure 3).

Avg-Y is pinned to its definition through properties the union of event times must have:
the curve is constant between consecutive points (checked with the grid reduction at the
midpoints, a separate code path) and changes at every point (no point without an event);
one trajectory reproduces itself; a closed network conserves its total exactly.  Avg-XY:
k = 1 gives Avg-Y back, groups have k points (the last one fewer), and for the
immigration-death process the averaged points follow the exact mean (b/d)(1 - exp(-d t)).
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1007_1768_amd import inputs


def _iso():
    # A <-> B, closed: A + B = 40 in every trajectory
    return inputs._model("iso", ["A", "B"], [({"A": 1}, {"B": 1}, 0.7), ({"B": 1}, {"A": 1}, 0.3)], [30, 10])


def test_points_are_the_change_points():
    m = inputs.viral()
    N, t_end, seed = 40, 2.0, 5
    st, r = orc.adaptive(m, N, t_end, seed, 7)
    assert st == 0
    t = r["y_time"]
    assert t[0] == 0.0 and np.all(np.diff(t) > 0) and t[-1] <= t_end
    assert len(t) == r["events"] + 1          # distinct event times (ties have probability 0)
    # constant between points: the grid reduction at the midpoints (and at t_end) sees the
    # value of the point on the left
    mid = np.concatenate([(t[:-1] + t[1:]) / 2.0, [t_end]])
    st, g = orc.run(m, N, t_end, mid, seed)
    assert st == 0
    assert np.array_equal(g["mean"], r["y_mean"]) and np.array_equal(g["var"], r["y_var"])
    # and it changes at every point after the first: each is some trajectory's event
    assert np.all(np.any(r["y_mean"][1:] != r["y_mean"][:-1], axis=1))


def test_single_trajectory_is_itself():
    m = inputs.viral()
    t_end, seed = 3.0, 11
    st, r = orc.adaptive(m, 1, t_end, seed, 4)
    assert st == 0
    st, rec = orc.trajectory(m, seed, 0, t_end, r["y_time"])
    assert st == 0
    assert rec["events"] == len(r["y_time"]) - 1
    assert np.array_equal(rec["states"].astype(np.float64), r["y_mean"])
    assert np.all(r["y_var"] == 0.0)


def test_k1_is_avg_y_and_group_sizes():
    m = inputs.viral()
    st, r1 = orc.adaptive(m, 25, 1.5, 2, 1)
    assert st == 0
    assert np.array_equal(r1["xy_time"], r1["y_time"])
    assert np.array_equal(r1["xy_mean"], r1["y_mean"]) and np.array_equal(r1["xy_var"], r1["y_var"])
    for k in (2, 7, 64):
        st, r = orc.adaptive(m, 25, 1.5, 2, k)
        U, P = len(r["y_time"]), len(r["xy_time"])
        assert P == -(-U // k)
        for p in range(P):
            seg = r["y_time"][p * k:(p + 1) * k]
            assert seg[0] <= r["xy_time"][p] <= seg[-1]
        # last group: the mean of its own points only
        last = r["y_mean"][(P - 1) * k:]
        assert np.allclose(r["xy_mean"][-1], last.mean(axis=0), rtol=1e-14, atol=0)


def test_closed_network_conserves():
    m = _iso()
    st, r = orc.adaptive(m, 300, 4.0, 9, 50)
    assert st == 0
    assert np.all(np.abs(r["y_mean"].sum(axis=1) - 40.0) <= 1e-12 * 40)
    assert np.all(np.abs(r["xy_mean"].sum(axis=1) - 40.0) <= 1e-12 * 40)
    # B = 40 - A in every trajectory: the exact variance numerators are equal integers
    assert np.array_equal(r["y_var"][:, 0], r["y_var"][:, 1])


def test_immigration_death_follows_the_exact_mean():
    b, d = 10.0, 0.1
    m = inputs.immigration_death(b, d, 0)
    N, t_end, k = 400, 30.0, 400
    st, r = orc.adaptive(m, N, t_end, 21, k)
    assert st == 0
    for p in range(len(r["xy_time"])):
        seg = r["y_time"][p * k:(p + 1) * k]
        exact = np.mean((b / d) * (1.0 - np.exp(-d * seg)))     # exact mean at the group's times
        sd = math.sqrt(max(exact, 1.0) / N)                        # Poisson: var = mean
        assert abs(r["xy_mean"][p, 0] - exact) <= 5.0 * sd, (p, r["xy_mean"][p, 0], exact)


def test_groups_equal_whole_reduction():
    """The per-group evaluation (used at sizes where Avg-Y is too long to evaluate whole)
    gives the whole reduction's Avg-XY points bit for bit."""
    m = inputs.viral()
    N, t_end, seed, k = 30, 1.0, 4, 9
    st, r = orc.adaptive(m, N, t_end, seed, k)
    P = len(r["xy_time"])
    groups = [0, 1, P // 2, P - 1]
    st, g = orc.adaptive_groups(m, N, t_end, seed, k, groups)
    assert st == 0
    assert np.array_equal(g["y_time"], r["y_time"])
    assert np.array_equal(g["xy_time"], r["xy_time"][groups])
    assert np.array_equal(g["xy_mean"], r["xy_mean"][groups]) and np.array_equal(g["xy_var"], r["xy_var"][groups])
