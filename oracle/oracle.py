"""ctypes wrapper around the C oracle (``liboracle.so``).  Test infrastructure only.

A network is passed as plain arrays: ``reac`` and ``prod`` of shape (M, S) with
non-negative integer coefficients, ``rates`` (M,) binary64 stochastic rate constants and
``x0`` (S,) int32 initial counts.
"""
import ctypes
import os

import numpy as np

from . import build_oracle

OK, INVALID, NOMEM, OVERFLOW, EVENT_LIMIT = 0, 1, 2, 4, 5

_lib = None


class _Net(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int32), ("M", ctypes.c_int32),
                ("reac", ctypes.c_void_p), ("prod", ctypes.c_void_p),
                ("rate", ctypes.c_void_p), ("x0", ctypes.c_void_p), ("sum_order", ctypes.c_int32),
                ("law_species", ctypes.c_void_p), ("law_slope", ctypes.c_void_p), ("law_lo", ctypes.c_void_p),
                ("law_hi", ctypes.c_void_p)]

SUM_ORDERS = {"seq": 0, "block64": 1}


def lib():
    global _lib
    if _lib is None:
        path = build_oracle.build()
        L = ctypes.CDLL(path)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_neglog.argtypes = [ctypes.c_double]
        L.orc_neglog.restype = ctypes.c_double
        L.orc_exp.argtypes = [ctypes.c_double]
        L.orc_exp.restype = ctypes.c_double
        L.orc_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.orc_uniforms.restype = None
        vp = ctypes.c_void_p
        L.orc_trajectory.argtypes = [ctypes.POINTER(_Net), ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                     vp, ctypes.c_int32, ctypes.c_uint64,
                                     vp, vp, vp, vp, vp, vp]
        L.orc_trajectory.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.POINTER(_Net), ctypes.c_int64, ctypes.c_double, vp, ctypes.c_int32,
                              ctypes.c_uint64, ctypes.c_uint64,
                              ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              vp, vp, vp, vp, vp, ctypes.c_int]
        L.orc_run.restype = ctypes.c_int
        L.orc_grad.argtypes = [ctypes.POINTER(_Net), ctypes.c_int64, ctypes.c_double, vp, ctypes.c_int32,
                               ctypes.c_uint64, ctypes.c_uint64, vp, vp, vp, vp, ctypes.c_int]
        L.orc_grad.restype = ctypes.c_int
        L.orc_grad_moments.argtypes = [ctypes.POINTER(_Net), ctypes.c_int64, ctypes.c_double, vp, ctypes.c_int32,
                                       ctypes.c_uint64, ctypes.c_uint64, vp, vp, vp, vp, vp, vp, ctypes.c_int]
        L.orc_grad_moments.restype = ctypes.c_int
        L.orc_jacobian.argtypes = [ctypes.POINTER(_Net), ctypes.c_int64, ctypes.c_double, vp, ctypes.c_int32,
                                   ctypes.c_uint64, ctypes.c_uint64, vp, vp, vp, ctypes.c_int]
        L.orc_jacobian.restype = ctypes.c_int
        L.orc_covariance.argtypes = [ctypes.POINTER(_Net), ctypes.c_int64, ctypes.c_double, vp, ctypes.c_int32,
                                     ctypes.c_uint64, ctypes.c_uint64, vp, vp, ctypes.c_int]
        L.orc_covariance.restype = ctypes.c_int
        L.orc_adaptive.argtypes = [ctypes.POINTER(_Net), ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                   ctypes.c_uint64, ctypes.c_int64,
                                   ctypes.c_int64, vp, vp, vp, vp, ctypes.c_int64, vp, vp, vp, vp, ctypes.c_int]
        L.orc_adaptive.restype = ctypes.c_int
        L.orc_adaptive_groups.argtypes = [ctypes.POINTER(_Net), ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                          ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, vp, ctypes.c_int64, vp, vp,
                                          vp, vp, vp, ctypes.c_int]
        L.orc_adaptive_groups.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Net:
    """Holds contiguous copies of a network's arrays and the ctypes struct that points at them."""

    def __init__(self, reac, prod, rates, x0, sum_order="seq", laws=None):
        self.reac = np.ascontiguousarray(reac, dtype=np.int32)
        self.prod = np.ascontiguousarray(prod, dtype=np.int32)
        self.rates = np.ascontiguousarray(rates, dtype=np.float64)
        self.x0 = np.ascontiguousarray(x0, dtype=np.int32)
        self.M, self.S = self.reac.shape
        ptrs = [None, None, None, None]
        if laws is not None:
            self.law_species = np.ascontiguousarray(laws["species"], dtype=np.int32)
            self.law_slope = np.ascontiguousarray(laws["slope"], dtype=np.float64)
            self.law_lo = np.ascontiguousarray(laws["lo"], dtype=np.float64)
            self.law_hi = np.ascontiguousarray(laws["hi"], dtype=np.float64)
            ptrs = [self.law_species.ctypes.data, self.law_slope.ctypes.data, self.law_lo.ctypes.data,
                    self.law_hi.ctypes.data]
        self.c = _Net(self.S, self.M, self.reac.ctypes.data, self.prod.ctypes.data,
                      self.rates.ctypes.data, self.x0.ctypes.data, SUM_ORDERS[sum_order], *ptrs)


def as_net(model, rates=None):
    """model: dict with reac, prod, rates, x0 and optionally sum_order ("seq" or "block64")."""
    return Net(model["reac"], model["prod"], model["rates"] if rates is None else rates, model["x0"],
               model.get("sum_order", "seq"), model.get("laws"))


def default_threads():
    n = os.environ.get("ORACLE_THREADS")
    if n:
        return int(n)
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def neglog(r):
    return lib().orc_neglog(float(r))


def exp_rates(theta):
    """Rate constants c = e^theta from log rate constants, element by element (orc_exp)."""
    th = np.asarray(theta, dtype=np.float64)
    return np.array([lib().orc_exp(float(v)) for v in th.ravel()], dtype=np.float64).reshape(th.shape)


def uniforms(seed, traj, k):
    r1, r2 = ctypes.c_double(), ctypes.c_double()
    lib().orc_uniforms(seed, traj, k, ctypes.byref(r1), ctypes.byref(r2))
    return r1.value, r2.value


def trajectory(model, seed, traj, t_end, grid, max_events=2**62, rates=None):
    """Returns (status, dict) with states (G,S) int32, events, draws, t_last, n_fired (M,), a_int (M,)."""
    net = as_net(model, rates)
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    G = grid.shape[0]
    states = np.zeros((G, net.S), dtype=np.int32)
    ev = np.zeros(1, dtype=np.uint64)
    dr = np.zeros(1, dtype=np.uint64)
    tl = np.zeros(1, dtype=np.float64)
    nf = np.zeros(net.M, dtype=np.int64)
    ai = np.zeros(net.M, dtype=np.float64)
    st = lib().orc_trajectory(ctypes.byref(net.c), seed, traj, t_end, _ptr(grid), G, max_events,
                              _ptr(states), _ptr(ev), _ptr(dr), _ptr(tl), _ptr(nf), _ptr(ai))
    return st, dict(states=states, events=int(ev[0]), draws=int(dr[0]), t_last=float(tl[0]),
                    n_fired=nf, a_int=ai)


def run(model, N, t_end, grid, seed, hist=None, max_events=2**62, rates=None, threads=None,
        want_sums=False):
    """Mean / variance per (grid point, species); optional histogram spec (species, lo, width, nbins).

    Returns (status, dict(mean (G,S), var (G,S), hist (G,nbins) or None, events, sums)).
    ``sums`` holds the exact (sum X, sum X^2) as Python ints, shape (G,S,2), if requested.
    """
    net = as_net(model, rates)
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    G = grid.shape[0]
    mean = np.zeros((G, net.S))
    var = np.zeros((G, net.S))
    h = None
    hs = (0, 0, 1, 1)
    if hist is not None:
        hs = tuple(int(v) for v in hist)
        h = np.zeros((G, hs[3]), dtype=np.uint32)
    sums = np.zeros((G, net.S, 4), dtype=np.int64) if want_sums else None
    ev = np.zeros(1, dtype=np.uint64)
    st = lib().orc_run(ctypes.byref(net.c), int(N), float(t_end), _ptr(grid), G, seed, max_events,
                       hs[0], hs[1], hs[2], hs[3], _ptr(mean), _ptr(var), _ptr(h), _ptr(sums), _ptr(ev),
                       threads or default_threads())
    out = dict(mean=mean, var=var, hist=h, events=int(ev[0]))
    if want_sums:
        def i128(hi, lo):
            return (int(hi) << 64) | (int(lo) & 0xFFFFFFFFFFFFFFFF)
        out["sums"] = [[(i128(sums[g, s, 0], sums[g, s, 1]), i128(sums[g, s, 2], sums[g, s, 3]))
                        for s in range(net.S)] for g in range(G)]
    return st, out


def grad(model, N, t_end, grid, seed, w, mhat, max_events=2**62, rates=None, threads=None, wv=None, vhat=None):
    """Likelihood-ratio gradient wrt log rate constants of a loss on the grid means (weights
    w = dL/dmean, centring mhat) and optionally the variances (wv = dL/dvar, centring vhat).
    Returns (status, grad (M,), l1 (M,))."""
    net = as_net(model, rates)
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    G = grid.shape[0]
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(G, net.S)
    mhat = np.ascontiguousarray(mhat, dtype=np.float64).reshape(G, net.S)
    if wv is not None:
        wv = np.ascontiguousarray(wv, dtype=np.float64).reshape(G, net.S)
        vhat = np.ascontiguousarray(vhat, dtype=np.float64).reshape(G, net.S)
    g_out = np.zeros(net.M)
    l1 = np.zeros(net.M)
    st = lib().orc_grad_moments(ctypes.byref(net.c), int(N), float(t_end), _ptr(grid), G, seed, max_events,
                                _ptr(w), _ptr(mhat), _ptr(wv), _ptr(vhat), _ptr(g_out), _ptr(l1),
                                threads or default_threads())
    return st, g_out, l1


def jacobian(model, N, t_end, grid, seed, mhat, max_events=2**62, rates=None, threads=None):
    """LR Jacobian J[g, s, j] = (1/N) sum_i (X_s(t_g) - mhat[g, s]) z_j(t_g) and its L1 scale."""
    net = as_net(model, rates)
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    G = grid.shape[0]
    mh = np.ascontiguousarray(mhat, dtype=np.float64).reshape(G, net.S)
    jac = np.zeros((G, net.S, net.M))
    l1 = np.zeros((G, net.S, net.M))
    st = lib().orc_jacobian(ctypes.byref(net.c), int(N), float(t_end), _ptr(grid), G, int(seed), int(max_events),
                            _ptr(mh), _ptr(jac), _ptr(l1), int(threads or default_threads()))
    return st, jac, l1


def covariance(model, N, t_end, grid, seed, max_events=2**62, rates=None, threads=None):
    """Grid means (G, S) and species covariance matrices (G, S, S) from exact sums."""
    net = as_net(model, rates)
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    G = grid.shape[0]
    mean = np.zeros((G, net.S))
    cov = np.zeros((G, net.S, net.S))
    st = lib().orc_covariance(ctypes.byref(net.c), int(N), float(t_end), _ptr(grid), G, int(seed), int(max_events),
                              _ptr(mean), _ptr(cov), int(threads or default_threads()))
    return st, mean, cov


def adaptive(model, N, t_end, seed, k, max_events=2**62, rates=None, threads=None):
    """Adaptive selective memory: Avg-Y over {0} and every distinct event time, Avg-XY over
    groups of k successive Avg-Y points.  Returns (status, dict(y_time (U,), y_mean (U,S),
    y_var (U,S), xy_time (P,), xy_mean (P,S), xy_var (P,S), events))."""
    net = as_net(model, rates)
    st, r = run(model, N, t_end, np.array([float(t_end)]), seed, max_events=max_events, rates=rates,
                threads=threads)
    if st != 0:
        return st, None
    cap = r["events"] + 1
    capxy = (cap + k - 1) // k
    S = net.S
    yt, ym, yv = np.zeros(cap), np.zeros((cap, S)), np.zeros((cap, S))
    xt, xm, xv = np.zeros(capxy), np.zeros((capxy, S)), np.zeros((capxy, S))
    ny, nxy = np.zeros(1, np.int64), np.zeros(1, np.int64)
    st = lib().orc_adaptive(ctypes.byref(net.c), int(N), float(t_end), int(seed), int(max_events), int(k),
                            cap, _ptr(ny), _ptr(yt), _ptr(ym), _ptr(yv), capxy, _ptr(nxy), _ptr(xt), _ptr(xm),
                            _ptr(xv), int(threads or default_threads()))
    if st != 0:
        return st, None
    U, P = int(ny[0]), int(nxy[0])
    return st, dict(y_time=yt[:U], y_mean=ym[:U], y_var=yv[:U], xy_time=xt[:P], xy_mean=xm[:P], xy_var=xv[:P],
                    events=r["events"])


def adaptive_groups(model, N, t_end, seed, k, groups, max_events=2**62, rates=None, threads=None):
    """All Avg-Y point times and the Avg-XY points of the chosen groups only (each from the
    grid reduction at its own points).  Returns (status, dict(y_time (U,), xy_time (n,),
    xy_mean (n,S), xy_var (n,S), events))."""
    net = as_net(model, rates)
    st, r = run(model, N, t_end, np.array([float(t_end)]), seed, max_events=max_events, rates=rates,
                threads=threads)
    if st != 0:
        return st, None
    cap = r["events"] + 1
    g = np.ascontiguousarray(groups, dtype=np.int64)
    S = net.S
    yt = np.zeros(cap)
    gt, gm, gv = np.zeros(len(g)), np.zeros((len(g), S)), np.zeros((len(g), S))
    ny = np.zeros(1, np.int64)
    st = lib().orc_adaptive_groups(ctypes.byref(net.c), int(N), float(t_end), int(seed), int(max_events), int(k),
                                   len(g), _ptr(g), cap, _ptr(ny), _ptr(yt), _ptr(gt), _ptr(gm), _ptr(gv),
                                   int(threads or default_threads()))
    if st != 0:
        return st, None
    return st, dict(y_time=yt[:int(ny[0])], xy_time=gt, xy_mean=gm, xy_var=gv, events=r["events"])
