"""The oracle's cross-trajectory reduction pinned to per-trajectory records.

Section 3.2.1 reduces the time-aligned trajectories with associative, commutative
functions and Section 4 reports their mean and variance over the runs.  The reading used
here: mean = fl(sum X) / N and the unbiased variance fl(N sum X^2 - (sum X)^2) / (N (N - 1))
(0 when N = 1), each from exact integer sums; the species covariance likewise from the
exact cross sums; the histogram counts trajectories per bin clamp((x - lo) div width).

Pins: the per-trajectory states of orc.trajectory (a code path that reduces nothing) are
summed here in Python integers, the exact moments formed with fractions.Fraction, and
their binary64 roundings computed independently of the oracle's C code.  A divisor of N
(or N^2) instead of N - 1 (or N (N - 1)), a dropped square, a sum over the wrong axis or a
wrong histogram bin fails these exact comparisons; the statistical bands of the
distribution tests are far too wide to see such slips at large N.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1007_1768_amd import inputs


def _burst():
    """0 -> 10^4 X (rate 1) and 0 -> X (rate 5): counts near 10^6 with a variance near
    10^10, so N sum X^2 - (sum X)^2 exceeds 2^53 at N = 1000 and its rounding to binary64
    (one rounding of the exact integer) is exercised."""
    reac = np.zeros((2, 1), np.int32)
    prod = np.array([[10000], [1]], np.int32)
    return dict(name="burst", reac=reac, prod=prod, rates=np.array([1.0, 5.0]), x0=np.array([7], np.int32))


CASES = {
    "viral": (inputs.viral, 5.0, 11, 31),
    "immigration_death": (inputs.immigration_death, 40.0, 9, 32),
    "burst": (_burst, 100.0, 6, 33),
}


def _states(m, N, t_end, grid, seed):
    out = []
    for i in range(N):
        st, r = orc.trajectory(m, seed, i, t_end, grid)
        assert st == 0
        out.append(r["states"].astype(np.int64))
    return out


def _contract_var(n, sx, sx2):
    """fl(N sum X^2 - (sum X)^2) / (N (N - 1)): the exact numerator rounded once to binary64
    (Python's int -> float conversion rounds to nearest even), divided in binary64."""
    if n == 1:
        return 0.0
    return float(n * sx2 - sx * sx) / float(n * (n - 1))


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("N", [1, 2, 3, 7, 64, 1000])
def test_mean_and_variance_equal_exact_moments(case, N):
    make, t_end, G, seed = CASES[case]
    if case == "viral" and N == 1000:
        N = 600   # keeps the CPU suite short; still several hundred ragged trajectories
    m = make()
    grid = inputs.uniform_grid(t_end, G)
    xs = _states(m, N, t_end, grid, seed)
    st, ref = orc.run(m, N, t_end, grid, seed, threads=2)
    assert st == 0
    S = m["reac"].shape[1]
    big = False
    for g in range(G):
        for s in range(S):
            vals = [int(x[g, s]) for x in xs]
            sx, sx2 = sum(vals), sum(v * v for v in vals)
            # mean: the exact sum is below 2^53 here, so fl(sum) / N is the correctly
            # rounded value of the exact rational mean
            assert ref["mean"][g, s] == float(Fraction(sx, N)), (g, s)
            v = ref["var"][g, s]
            assert v == _contract_var(N, sx, sx2), (g, s, v)
            if N > 1:
                exact = Fraction(N * sx2 - sx * sx, N * (N - 1))
                # one rounding of the numerator and one of the quotient: within 2 ulp
                assert abs(Fraction(v) - exact) <= 2 * np.spacing(abs(float(exact))) + 0, (g, s)
                # the sample-variance identity sum (x - mean)^2 / (N - 1), exactly
                mu = Fraction(sx, N)
                assert exact == sum((Fraction(x) - mu) ** 2 for x in vals) / (N - 1)
                big = big or abs(N * sx2 - sx * sx) > 2 ** 53
            else:
                assert v == 0.0
    if case == "burst" and N == 1000:
        assert big, "the burst case must exercise the rounding of a numerator beyond 2^53"


@pytest.mark.parametrize("N", [2, 7, 64, 300])
def test_covariance_equals_exact_cross_moments(N):
    m = inputs.viral()
    t_end, G, seed = 5.0, 6, 41
    grid = inputs.uniform_grid(t_end, G)
    xs = _states(m, N, t_end, grid, seed)
    st, mean, cov = orc.covariance(m, N, t_end, grid, seed, threads=2)
    assert st == 0
    S = 4
    for g in range(G):
        for s in range(S):
            xs_s = [int(x[g, s]) for x in xs]
            assert mean[g, s] == float(Fraction(sum(xs_s), N))
            for r in range(S):
                xs_r = [int(x[g, r]) for x in xs]
                num = N * sum(a * b for a, b in zip(xs_s, xs_r)) - sum(xs_s) * sum(xs_r)
                assert cov[g, s, r] == float(num) / float(N * (N - 1)), (g, s, r)
                # symmetric, and the diagonal is the variance routine's value
                assert cov[g, s, r] == cov[g, r, s]
    st, ref = orc.run(m, N, t_end, grid, seed, threads=2)
    assert np.array_equal(np.diagonal(cov, axis1=1, axis2=2), ref["var"])


@pytest.mark.parametrize("spec", [(1, 0, 1, 64), (0, 990, 3, 7), (2, 50, 10, 4)])
def test_histogram_counts_trajectories_per_bin(spec):
    m = inputs.viral()
    N, t_end, G, seed = 200, 5.0, 11, 43
    grid = inputs.uniform_grid(t_end, G)
    xs = _states(m, N, t_end, grid, seed)
    st, ref = orc.run(m, N, t_end, grid, seed, hist=spec, threads=2)
    assert st == 0
    sp, lo, width, nb = spec
    want = np.zeros((G, nb), np.int64)
    for x in xs:
        for g in range(G):
            v = int(x[g, sp])
            b = 0 if v < lo else min((v - lo) // width, nb - 1)
            want[g, b] += 1
    assert np.array_equal(ref["hist"].astype(np.int64), want)
    assert np.all(want.sum(axis=1) == N)
