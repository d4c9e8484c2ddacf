"""Pure-Python second implementation of the oracle's arithmetic contract (test infrastructure).

Written independently of ``ssa_oracle.c`` from the same readings of the paper: Philox4x32-10
(Salmon et al., SC'11), the 53-bit uniforms, the atanh-series -ln r, the direct method of
Section 2 with right-continuous grid alignment (Section 3.2.1).  It is slow (Python ints
and fractions) and meant for a handful of trajectories, to catch a misreading that a single
implementation would carry silently.

Python 3.10 has no math.fma; ``_fma`` forms the exact a*b + c with Fraction and rounds it
once (float(Fraction) rounds to nearest-even).
"""
from fractions import Fraction
import struct

MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    c = [int(v) & MASK32 for v in ctr]
    k0, k1 = int(key[0]) & MASK32, int(key[1]) & MASK32
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & MASK32
            k1 = (k1 + 0xBB67AE85) & MASK32
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & MASK32, p1 & MASK32,
             ((p0 >> 32) ^ c[3] ^ k1) & MASK32, p0 & MASK32]
    return c


def uniforms(seed, traj, k):
    o = philox4x32_10([k & MASK32, k >> 32, traj & MASK32, traj >> 32], [seed & MASK32, seed >> 32])
    w1 = (o[1] << 32) | o[0]
    w2 = (o[3] << 32) | o[2]
    r1 = float((w1 >> 11) + 1) * 2.0 ** -53
    r2 = float(w2 >> 11) * 2.0 ** -53
    return r1, r2


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


LN2_HI = float.fromhex("0x1.62e42fee00000p-1")
LN2_LO = float.fromhex("0x1.a39ef35793c76p-33")
SQRT2 = float.fromhex("0x1.6a09e667f3bcdp+0")


def neglog(r):
    bits = struct.unpack("<Q", struct.pack("<d", r))[0]
    E = ((bits >> 52) & 0x7FF) - 1023
    m = struct.unpack("<d", struct.pack("<Q", (bits & ((1 << 52) - 1)) | (1023 << 52)))[0]
    if m > SQRT2:
        m = m * 0.5
        E += 1
    f = (m - 1.0) / (m + 1.0)
    s = f * f
    P = 2.0 / 21.0
    for n in range(9, 0, -1):
        P = _fma(P, s, 2.0 / (2 * n + 1))
    t = s * P
    lnm = _fma(f, t, f + f)
    Ed = float(E)
    return -_fma(Ed, LN2_HI, _fma(Ed, LN2_LO, lnm))


def _h(reac_row, x):
    idx = [s for s, v in enumerate(reac_row) for _ in range(int(v))]
    if not idx:
        return 1
    if len(idx) == 1:
        return int(x[idx[0]])
    a, b = idx
    if a == b:
        return int(x[a]) * (int(x[a]) - 1) // 2
    return int(x[a]) * int(x[b])


def _partial_sums(a, order):
    """Cumulative propensity sums in the network's order: left to right ("seq"), or the
    64-chunk form ("block64": sequential inside chunks of ceil(M/64), chunk totals combined
    by a six-step doubling scan, each chunk offset by the scanned total of the chunks
    before it)."""
    if order == "seq":
        out = []
        for v in a:
            out.append(v if not out else out[-1] + v)
        return out
    q = -(-len(a) // 64)
    local = []
    for lane in range(64):
        run = []
        for v in a[lane * q:(lane + 1) * q]:
            run.append(v if not run else run[-1] + v)
        local.append(run)
    scan = [r[-1] if r else 0.0 for r in local]
    step = 1
    while step < 64:
        scan = [scan[i] + scan[i - step] if i >= step else scan[i] for i in range(64)]
        step *= 2
    offset = [0.0] + scan[:-1]
    return [offset[lane] + v for lane, run in enumerate(local) for v in run]


def trajectory(model, seed, traj, t_end, grid, rates=None):
    """Mirror of the oracle's single-trajectory record: (states, events, draws, t_last, n_fired, a_int)."""
    reac = [[int(v) for v in row] for row in model["reac"]]
    prod = [[int(v) for v in row] for row in model["prod"]]
    c = [float(v) for v in (model["rates"] if rates is None else rates)]
    x = [int(v) for v in model["x0"]]
    M, S = len(reac), len(x)
    G = len(grid)
    states = [[0] * S for _ in range(G)]
    nf = [0] * M
    A = [0.0] * M
    t = 0.0
    k = 0
    events = 0
    g = 0
    while True:
        a = [c[j] * float(_h(reac[j], x)) for j in range(M)]
        Ssum = _partial_sums(a, model.get("sum_order", "seq"))
        a0 = Ssum[-1]
        if a0 == 0.0:
            tau, r2 = float("inf"), 0.0
        else:
            r1, r2 = uniforms(seed, traj, k)
            tau = neglog(r1) / a0
            k += 1
        t_next = t + tau
        while g < G and grid[g] < t_next:
            states[g] = list(x)
            g += 1
        if t_next > t_end:
            break
        u = r2 * a0
        sel = next((j for j in range(M) if Ssum[j] > u), None)
        if sel is None:
            sel = max(j for j in range(M) if a[j] > 0.0)
        x = [x[s] + prod[sel][s] - reac[sel][s] for s in range(S)]
        nf[sel] += 1
        A = [A[j] + a[j] * tau for j in range(M)]
        t = t_next
        events += 1
    tail = t_end - t
    a_end = [c[j] * float(_h(reac[j], x)) for j in range(M)]
    a_int = [A[j] + a_end[j] * tail for j in range(M)]
    return dict(states=states, events=events, draws=k, t_last=t, n_fired=nf, a_int=a_int)
