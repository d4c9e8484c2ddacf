"""Chemical master equation by brute force on a truncated state space (test infrastructure).

Section 2 of the paper describes the master equation as the differential-difference
equation for the state distribution, solvable numerically only for tiny systems; for
such systems it gives the exact time-dependent distribution that the simulated
trajectories must sample.  Here the states are enumerated in a box
0 <= x_s <= cap_s, the generator Q is assembled with mass-action propensities
(x_A; x_A x_B; x_A (x_A - 1) / 2), and p(t) = exp(t Q^T) p(0) is evaluated with
scipy's expm_multiply.  Transitions that leave the box are dropped; the returned
``leak`` (1 - total probability) bounds the truncation error.
"""
import itertools

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import expm_multiply


def _h(reac_row, x):
    need = [(s, int(v)) for s, v in enumerate(reac_row) if v]
    h = 1
    for s, v in need:
        if v == 1:
            h *= x[s]
        elif v == 2:
            h *= x[s] * (x[s] - 1) // 2
        else:
            raise ValueError("order > 2")
    return h


def solve(model, caps, times):
    """Returns dict(p=(T, n_states), states=(n_states, S), mean=(T,S), var=(T,S), leak=(T,))."""
    reac = np.asarray(model["reac"], dtype=np.int64)
    prod = np.asarray(model["prod"], dtype=np.int64)
    rates = np.asarray(model["rates"], dtype=np.float64)
    x0 = tuple(int(v) for v in model["x0"])
    M, S = reac.shape
    caps = [int(c) for c in caps]
    states = list(itertools.product(*[range(c + 1) for c in caps]))
    index = {s: i for i, s in enumerate(states)}
    nu = prod - reac
    rows, cols, vals = [], [], []
    diag = np.zeros(len(states))
    for i, x in enumerate(states):
        for j in range(M):
            a = rates[j] * _h(reac[j], x)
            if a == 0.0:
                continue
            y = tuple(x[s] + int(nu[j, s]) for s in range(S))
            diag[i] -= a
            k = index.get(y)
            if k is not None:
                rows.append(k)
                cols.append(i)
                vals.append(a)
    n = len(states)
    QT = sp.csr_matrix((vals, (rows, cols)), shape=(n, n)) + sp.diags(diag)
    p0 = np.zeros(n)
    p0[index[x0]] = 1.0
    times = np.asarray(times, dtype=np.float64)
    P = np.zeros((len(times), n))
    for ti, t in enumerate(times):
        P[ti] = p0 if t == 0.0 else expm_multiply(QT * t, p0)
    st = np.asarray(states, dtype=np.float64)
    mass = P.sum(axis=1)
    mean = (P @ st) / mass[:, None]
    ex2 = (P @ (st * st)) / mass[:, None]
    return dict(p=P, states=np.asarray(states), mean=mean, var=ex2 - mean * mean, leak=1.0 - mass)


def marginal(sol, species, ti):
    """Marginal distribution of one species at time index ti: (values, probabilities)."""
    vals = sol["states"][:, species]
    probs = np.bincount(vals, weights=sol["p"][ti], minlength=int(vals.max()) + 1)
    return np.arange(len(probs)), probs
