"""Pins for the oracle's random stream and exponential draw.

* Philox4x32-10 block: the known-answer vectors published with Random123 (Salmon et al.,
  SC'11) in tests/golden, and rocRAND's independent engine run on the host.
* Counter layout (key = seed, counter = (step, trajectory)): rocRAND with
  subsequence = trajectory and offset = 4 * step must give the same block.
* -ln r: against mpmath at 60 digits on random and boundary
  inputs (error at most 2 ulp), and exact special values.
"""
import math
import os
import random
import shutil
import struct
import subprocess

import mpmath
import numpy as np
import pytest

from oracle import mirror
from oracle import oracle as orc

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert orc.philox(ctr, key) == out
        assert mirror.philox4x32_10(ctr, key) == out


def test_philox_oracle_matches_mirror_random_blocks():
    rng = random.Random(5)
    for _ in range(2000):
        ctr = [rng.getrandbits(32) for _ in range(4)]
        key = [rng.getrandbits(32) for _ in range(2)]
        assert orc.philox(ctr, key) == mirror.philox4x32_10(ctr, key)


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("rr") / "probe")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "rocrand_philox_probe.cpp"), "-o", exe], check=True,
                   capture_output=True)
    return exe


def test_philox_stream_layout_matches_rocrand(rocrand_probe):
    rng = random.Random(11)
    queries = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2**64 - 1, 2**32 + 5, 2**33 + 7)]
    for _ in range(300):
        queries.append((rng.getrandbits(64), rng.getrandbits(rng.choice([8, 20, 40, 64])),
                        rng.getrandbits(rng.choice([4, 16, 34, 60]))))
    text = "".join("%x %x %x\n" % (s, i, 4 * k) for s, i, k in queries)
    out = subprocess.run([rocrand_probe], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    for (seed, traj, k), line in zip(queries, out):
        want = [int(t, 16) for t in line.split()]
        ctr = [k & 0xFFFFFFFF, (k >> 32) & 0xFFFFFFFF, traj & 0xFFFFFFFF, traj >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert orc.philox(ctr, key) == want, (seed, traj, k)


def test_uniform_ranges_and_construction():
    for seed, traj, k in [(0, 0, 0), (123, 4, 5), (2**63 + 3, 2**33, 2**40)]:
        r1, r2 = orc.uniforms(seed, traj, k)
        assert (r1, r2) == mirror.uniforms(seed, traj, k)
        o = orc.philox([k & 0xFFFFFFFF, k >> 32, traj & 0xFFFFFFFF, traj >> 32], [seed & 0xFFFFFFFF, seed >> 32])
        assert r1 == (((o[1] << 32 | o[0]) >> 11) + 1) / 2.0**53
        assert r2 == ((o[3] << 32 | o[2]) >> 11) / 2.0**53
        assert 0.0 < r1 <= 1.0 and 0.0 <= r2 < 1.0
    # first moments of a long stream: U(0,1) mean 1/2, variance 1/12
    r = np.array([orc.uniforms(7, 3, k) for k in range(20000)])
    assert abs(r[:, 0].mean() - 0.5) < 5 * math.sqrt(1 / 12 / 20000)
    assert abs(r[:, 1].mean() - 0.5) < 5 * math.sqrt(1 / 12 / 20000)
    assert abs(np.corrcoef(r[:, 0], r[:, 1])[0, 1]) < 5 / math.sqrt(20000)


def _ulp(x):
    return math.ulp(x)


def test_neglog_special_values():
    assert orc.neglog(1.0) == 0.0
    assert mirror.neglog(1.0) == 0.0
    assert orc.neglog(0.5) == float(mpmath.log(2))
    v = orc.neglog(2.0**-53)
    mpmath.mp.dps = 60
    exact = 53 * mpmath.log(2)
    assert abs(mpmath.mpf(v) - exact) <= _ulp(v)
    # powers of two are exact multiples of ln 2 split; error stays within 1 ulp
    for e in range(1, 54):
        v = orc.neglog(2.0**-e)
        assert abs(mpmath.mpf(v) - e * mpmath.log(2)) <= _ulp(v), e


def test_neglog_accuracy_against_mpmath():
    mpmath.mp.dps = 60
    rng = random.Random(3)
    inputs = []
    for _ in range(3000):
        inputs.append((rng.getrandbits(53) + 1) * 2.0**-53)          # the r1 distribution
    for e in range(0, 54):
        inputs.append(math.ldexp(1.0, -e) * (1 - 2**-53))
        inputs.append(math.ldexp(1.0, -e) * (1 + 2**-52) if e > 0 else 1.0)
    s2 = float.fromhex("0x1.6a09e667f3bcdp+0")
    for d in range(-4, 5):
        m = struct.unpack("<d", struct.pack("<Q", struct.unpack("<Q", struct.pack("<d", s2))[0] + d))[0]
        inputs.append(m / 2.0)
        inputs.append(m / 4.0)
    worst = 0.0
    for r in inputs:
        v = orc.neglog(r)
        exact = -mpmath.log(mpmath.mpf(r))
        if exact == 0:
            assert v == 0.0
            continue
        err = abs(mpmath.mpf(v) - exact) / mpmath.mpf(_ulp(float(exact)))
        worst = max(worst, float(err))
    # the series and its final combination round a few times; 2 ulp is the contract bound
    assert worst <= 2.0, worst


def test_neglog_oracle_matches_mirror_bitwise():
    rng = random.Random(9)
    for _ in range(2000):
        r = (rng.getrandbits(53) + 1) * 2.0**-53
        assert orc.neglog(r) == mirror.neglog(r)


def test_exp_rates_accuracy_against_mpmath():
    """Rate constants from log rate constants: within 2 ulp of e^theta (mpmath, 60 digits)
    over the whole accepted range, densely near 0 and at the ends of the argument
    reduction's intervals (theta near (k + 1/2) ln 2)."""
    mpmath.mp.dps = 60
    rng = np.random.default_rng(17)
    thetas = list(rng.uniform(-708.0, 709.0, 4000)) + list(rng.normal(0.0, 3.0, 4000))
    thetas += list(rng.uniform(-1e-6, 1e-6, 200)) + [0.0, 1.0, -1.0, 709.0, -708.0, 1e-300, -1e-300]
    ln2 = float(mpmath.log(2))
    for k in range(-1020, 1022, 7):
        thetas += [(k + 0.5) * ln2, np.nextafter((k + 0.5) * ln2, np.inf), np.nextafter((k + 0.5) * ln2, -np.inf)]
    thetas = [t for t in thetas if -708.0 <= t <= 709.0]
    got = orc.exp_rates(np.array(thetas))
    worst = 0.0
    for t, v in zip(thetas, got):
        exact = mpmath.exp(mpmath.mpf(float(t)))
        err = abs(mpmath.mpf(float(v)) - exact) / mpmath.mpf(math.ulp(float(exact)))
        worst = max(worst, float(err))
    assert worst <= 2.0, worst


def test_exp_rates_special_values():
    assert orc.exp_rates([0.0])[0] == 1.0
    # below the normal range of c the rate is zero; above 709 (and NaN) invalid
    assert list(orc.exp_rates([-708.0000001, -1000.0, -np.inf])) == [0.0, 0.0, 0.0]
    assert np.all(np.isnan(orc.exp_rates([709.0000001, 1000.0, np.inf, np.nan])))
    # monotone on a sorted sample, and e^a e^-a within a few ulp of 1
    t = np.sort(np.random.default_rng(3).uniform(-50, 50, 5000))
    c = orc.exp_rates(t)
    assert np.all(np.diff(c) >= 0)
    assert np.all(np.abs(c * orc.exp_rates(-t) - 1.0) <= 4 * 2.0**-52)
    # e^(fl(ln c)) returns c for the workload's rate constants, up to the rounding of ln c
    # (half an ulp of theta, times c) and 2 ulp of c
    for v in (10.0, 0.01, 2e-5, 0.5, 20.0, 3.0, 1e-3, 1e-4, 0.1):
        th = math.log(v)
        assert abs(orc.exp_rates([th])[0] - v) <= v * math.ulp(th) / 2 + 2 * math.ulp(v)
