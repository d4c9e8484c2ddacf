"""Python binding of libssa (include/ssa.h): argument marshalling only.

Every step of the simulation, alignment, reduction and gradient runs in the library's HIP
kernels.  PyTorch provides device memory (tensors) and the current HIP stream; numpy
arrays are used for host-side model descriptions.  Importing this module does not need a
GPU; calling into the library does, and a missing library raises instead of falling back
to anything else.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libssa.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_OVERFLOW, E_EVENT_LIMIT, E_UNSUPPORTED = range(7)
_NAMES = {1: "SSA_E_INVALID", 2: "SSA_E_NOMEM", 3: "SSA_E_DEVICE", 4: "SSA_E_OVERFLOW",
          5: "SSA_E_EVENT_LIMIT", 6: "SSA_E_UNSUPPORTED"}

EXPORTS = ["ssa_model_create", "ssa_model_create_laws", "ssa_model_destroy", "ssa_run", "ssa_rates_from_log",
           "ssa_run_device", "ssa_run_device_static", "ssa_run_begin", "ssa_run_advance", "ssa_run_finish",
           "ssa_run_destroy",
           "ssa_backward_device", "ssa_backward_moments_device",
           "ssa_run_jacobian_device", "ssa_jacobian_vjp", "ssa_autotune_forward", "ssa_autotune_backward",
           "ssa_run_cov_device",
           "ssa_hist_quantiles", "ssa_adaptive_device",
           "ssa_record", "ssa_batch_create", "ssa_batch_run", "ssa_batch_autotune", "ssa_batch_destroy",
           "ssa_last_error"]


class SSAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_NAMES.get(status, str(status)), msg))
        self.status = status


class HistSpec(ctypes.Structure):
    _fields_ = [("species", ctypes.c_int32), ("lo", ctypes.c_int32), ("width", ctypes.c_int32),
                ("nbins", ctypes.c_int32)]


FORMS = {0: "none", 1: "two_wave", 2: "generations", 3: "refill", 4: "table", 5: "wave"}


class Stats(ctypes.Structure):
    _fields_ = [("events", ctypes.c_uint64), ("max_steps", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("kernel_ms", ctypes.c_float), ("form", ctypes.c_uint32), ("blocks", ctypes.c_uint32),
                ("ordered", ctypes.c_uint32)]

    def as_dict(self):
        return dict(events=int(self.events), max_steps=int(self.max_steps), flags=int(self.flags),
                    kernel_ms=float(self.kernel_ms), form=FORMS.get(int(self.form), str(self.form)),
                    blocks=int(self.blocks), ordered=bool(self.ordered))


_lib = None


def load(path=None):
    """Load libssa.so (built by paper_1007_1768_amd/build.py); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError("libssa.so not built (%s); run python paper_1007_1768_amd/build.py" % path)
    L = ctypes.CDLL(path)
    vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    L.ssa_model_create.argtypes = [i32, i32, vp, vp, vp, vp, i32, ctypes.POINTER(vp)]
    L.ssa_model_create_laws.argtypes = [i32, i32, vp, vp, vp, vp, i32, vp, ctypes.POINTER(vp)]
    L.ssa_model_destroy.argtypes = [vp]
    L.ssa_model_destroy.restype = None
    L.ssa_run.argtypes = [vp, i64, dbl, vp, i32, u64, vp, vp, vp]
    L.ssa_rates_from_log.argtypes = [vp, i32, vp, vp]
    L.ssa_run_device.argtypes = [vp, vp, vp, i64, dbl, vp, i32, u64, u64, vp, vp, vp, vp, vp, vp]
    L.ssa_run_device_static.argtypes = [vp, vp, vp, i64, dbl, vp, i32, u64, u64, vp, vp, vp, vp, vp, vp]
    L.ssa_run_begin.argtypes = [vp, vp, i64, dbl, vp, i32, u64, u64, vp, ctypes.POINTER(vp)]
    L.ssa_run_advance.argtypes = [vp, dbl, vp, vp]
    L.ssa_run_finish.argtypes = [vp, vp, vp, vp, vp, vp]
    L.ssa_run_destroy.argtypes = [vp]
    L.ssa_run_destroy.restype = None
    L.ssa_backward_device.argtypes = [vp, vp, vp, i64, dbl, vp, i32, u64, u64, vp, vp, vp, vp, vp]
    L.ssa_backward_moments_device.argtypes = [vp, vp, vp, i64, dbl, vp, i32, u64, u64, vp, vp, vp, vp, vp, vp, vp]
    L.ssa_autotune_forward.argtypes = [vp, vp, i64, dbl, vp, i32, u64, vp, vp]
    L.ssa_autotune_backward.argtypes = [vp, vp, i64, dbl, vp, i32, u64, vp, vp]
    L.ssa_run_cov_device.argtypes = [vp, vp, i64, dbl, vp, i32, u64, u64, vp, vp, vp, vp]
    L.ssa_hist_quantiles.argtypes = [vp, i32, vp, i64, vp, i32, vp, vp]
    L.ssa_adaptive_device.argtypes = [vp, vp, i64, dbl, u64, u64, i64, vp, vp, vp, i64, vp, vp, vp, i64, vp, vp, vp]
    L.ssa_run_jacobian_device.argtypes = [vp, vp, vp, i64, dbl, vp, i32, u64, u64, vp, vp, vp, vp, vp]
    L.ssa_jacobian_vjp.argtypes = [vp, vp, i32, i32, i32, vp, vp]
    L.ssa_record.argtypes = [vp, vp, i64, i64, dbl, vp, i32, u64, u64, vp, vp, vp, vp, vp, vp]
    L.ssa_batch_create.argtypes = [i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
    L.ssa_batch_run.argtypes = [vp, vp, vp, vp, vp]
    L.ssa_batch_destroy.argtypes = [vp]
    L.ssa_batch_autotune.argtypes = [vp, vp, vp]
    L.ssa_batch_destroy.restype = None
    L.ssa_last_error.argtypes = []
    L.ssa_last_error.restype = ctypes.c_char_p
    for f in EXPORTS:
        if f not in ("ssa_model_destroy", "ssa_batch_destroy", "ssa_run_destroy", "ssa_last_error"):
            getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status != OK:
        raise SSAError(status, load().ssa_last_error().decode())


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _tp(t):
    """Device pointer of a torch tensor (None passes NULL)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


SUM_ORDERS = {"seq": 0, "block64": 1}


class RateLaw(ctypes.Structure):
    _fields_ = [("species", ctypes.c_int32), ("slope", ctypes.c_double), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double)]


class Model:
    """A network on the current device (ssa_model_create / ssa_model_create_laws).
    sum_order: "seq" (left-to-right propensity sums, one trajectory per lane) or "block64"
    (64-chunk sums, one trajectory per wave).  laws: optional dict of [M] arrays species,
    slope, lo, hi (species -1 = mass action) for species-dependent rate constants."""

    def __init__(self, reac, prod, rates, x0, sum_order="seq", laws=None):
        L = load()
        self.reac = np.ascontiguousarray(reac, dtype=np.int32)
        self.prod = np.ascontiguousarray(prod, dtype=np.int32)
        self.rates = np.ascontiguousarray(rates, dtype=np.float64)
        self.x0 = np.ascontiguousarray(x0, dtype=np.int32)
        self.M, self.S = self.reac.shape
        h = ctypes.c_void_p()
        self.sum_order = sum_order
        if laws is None:
            _check(L.ssa_model_create(self.S, self.M, _p(self.reac), _p(self.prod), _p(self.rates), _p(self.x0),
                                      SUM_ORDERS[sum_order], ctypes.byref(h)))
        else:
            arr = (RateLaw * self.M)()
            for j in range(self.M):
                arr[j] = RateLaw(int(laws["species"][j]), float(laws["slope"][j]), float(laws["lo"][j]),
                                 float(laws["hi"][j]))
            _check(L.ssa_model_create_laws(self.S, self.M, _p(self.reac), _p(self.prod), _p(self.rates),
                                           _p(self.x0), SUM_ORDERS[sum_order], arr, ctypes.byref(h)))
        self.handle = h

    @classmethod
    def from_dict(cls, m):
        return cls(m["reac"], m["prod"], m["rates"], m["x0"], m.get("sum_order", "seq"), m.get("laws"))

    def close(self):
        if getattr(self, "handle", None):
            load().ssa_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(model, n_traj, t_end, grid, seed):
    """Host form (ssa_run): numpy grid in, numpy (mean, var, stats) out."""
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    G = grid.shape[0]
    mean = np.zeros((G, model.S))
    var = np.zeros((G, model.S))
    st = Stats()
    _check(load().ssa_run(model.handle, int(n_traj), float(t_end), _p(grid), G, int(seed), _p(mean), _p(var),
                          ctypes.byref(st)))
    return mean, var, st.as_dict()


def rates_from_log(log_rates, stream=None, out=None):
    """c = e^theta on the device with the library's fixed roundings (ssa_rates_from_log)."""
    import torch
    theta = log_rates.contiguous()
    c = torch.empty_like(theta) if out is None else out
    _check(load().ssa_rates_from_log(_tp(theta), theta.shape[0], _tp(c), _stream(stream)))
    return c


def run_device(model, n_traj, t_end, grid, seed, rates=None, hist=None, max_events=0, stream=None,
               with_stats=False, out=None, log_rates=None):
    """Device form (ssa_run_device).  grid and rates (or log_rates) are float64 CUDA tensors;
    returns (mean, var, hist or None, stats or None) as tensors on grid's device."""
    import torch
    G = grid.shape[0]
    if out is None:
        mean = torch.empty((G, model.S), dtype=torch.float64, device=grid.device)
        var = torch.empty_like(mean)
        h = torch.empty((G, hist[3]), dtype=torch.int32, device=grid.device) if hist is not None else None
    else:
        mean, var, h = out
    spec = HistSpec(*[int(v) for v in hist]) if hist is not None else None
    st = Stats() if with_stats else None
    _check(load().ssa_run_device(model.handle, _tp(rates), _tp(log_rates), int(n_traj), float(t_end), _tp(grid), G,
                                 int(seed), int(max_events), _tp(mean), _tp(var),
                                 ctypes.byref(spec) if spec is not None else None, _tp(h), _stream(stream),
                                 ctypes.byref(st) if st is not None else None))
    return mean, var, h, (st.as_dict() if st is not None else None)


def run_device_static(model, n_traj, t_end, grid, seed, out, rates=None, log_rates=None, hist=None, max_events=0,
                      stream=None, with_stats=False):
    """ssa_run_device_static: run_device into caller-given outputs out = (mean, var, hist or
    None), with the library's static scratch area (no allocation); returns stats or None."""
    mean, var, h = out
    spec = HistSpec(*[int(v) for v in hist]) if hist is not None else None
    st = Stats() if with_stats else None
    _check(load().ssa_run_device_static(model.handle, _tp(rates), _tp(log_rates), int(n_traj), float(t_end),
                                        _tp(grid), grid.shape[0], int(seed), int(max_events), _tp(mean), _tp(var),
                                        ctypes.byref(spec) if spec is not None else None, _tp(h), _stream(stream),
                                        ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def backward_device(model, n_traj, t_end, grid, seed, w, mhat, rates=None, max_events=0, stream=None,
                    with_stats=False, out=None, wv=None, vhat=None, log_rates=None):
    """LR gradient d loss / d log c (ssa_backward_device; with variance weights wv = dL/dvar
    and centring vhat, ssa_backward_moments_device); returns (grad (M,), stats or None)."""
    import torch
    grad = torch.empty(model.M, dtype=torch.float64, device=grid.device) if out is None else out
    st = Stats() if with_stats else None
    L = load()
    if wv is None:
        _check(L.ssa_backward_device(model.handle, _tp(rates), _tp(log_rates), int(n_traj), float(t_end), _tp(grid),
                                     grid.shape[0], int(seed), int(max_events), _tp(w.contiguous()),
                                     _tp(mhat.contiguous()), _tp(grad), _stream(stream),
                                     ctypes.byref(st) if st is not None else None))
    else:
        _check(L.ssa_backward_moments_device(model.handle, _tp(rates), _tp(log_rates), int(n_traj), float(t_end),
                                             _tp(grid), grid.shape[0], int(seed), int(max_events), _tp(w.contiguous()),
                                             _tp(mhat.contiguous()), _tp(wv.contiguous()), _tp(vhat.contiguous()),
                                             _tp(grad), _stream(stream),
                                             ctypes.byref(st) if st is not None else None))
    return grad, (st.as_dict() if st is not None else None)


class Run:
    """A run taken in epochs of simulation time (ssa_run_begin / advance / finish): the same
    results as run_device, with the caller advancing it to successive times."""

    def __init__(self, model, n_traj, t_end, grid, seed, rates=None, hist=None, max_events=0):
        self.model = model
        self.grid = np.ascontiguousarray(grid, dtype=np.float64)
        self.hist = hist
        r = None if rates is None else np.ascontiguousarray(rates, dtype=np.float64)
        spec = HistSpec(*[int(v) for v in hist]) if hist is not None else None
        h = ctypes.c_void_p()
        _check(load().ssa_run_begin(model.handle, _p(r), int(n_traj), float(t_end), _p(self.grid), self.grid.shape[0],
                                    int(seed), int(max_events), ctypes.byref(spec) if spec is not None else None,
                                    ctypes.byref(h)))
        self.handle = h

    def advance(self, t_until, stream=None):
        st = Stats()
        _check(load().ssa_run_advance(self.handle, float(t_until), _stream(stream), ctypes.byref(st)))
        return st.as_dict()

    def finish(self, device="cuda:0", stream=None):
        import torch
        G, S = self.grid.shape[0], self.model.S
        mean = torch.empty((G, S), dtype=torch.float64, device=device)
        var = torch.empty_like(mean)
        h = torch.empty((G, self.hist[3]), dtype=torch.int32, device=device) if self.hist is not None else None
        st = Stats()
        _check(load().ssa_run_finish(self.handle, _tp(mean), _tp(var), _tp(h), _stream(stream), ctypes.byref(st)))
        return mean, var, h, st.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            load().ssa_run_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TuneResult(ctypes.Structure):
    _fields_ = [("win_bytes", ctypes.c_int32), ("slab", ctypes.c_int32), ("best_ms", ctypes.c_float),
                ("default_ms", ctypes.c_float), ("form", ctypes.c_int32), ("blocks", ctypes.c_int32)]

    def as_dict(self):
        return dict(win_bytes=self.win_bytes, slab=self.slab, best_ms=self.best_ms, default_ms=self.default_ms,
                    form=FORMS.get(int(self.form), str(self.form)), blocks=int(self.blocks))


def autotune_forward(model, n_traj, t_end, grid, seed, rates=None, stream=None):
    """Time the forward launch configurations on this problem and keep the fastest
    (ssa_autotune_forward); returns the chosen configuration and the two kernel times."""
    r = TuneResult()
    _check(load().ssa_autotune_forward(model.handle, _tp(rates), int(n_traj), float(t_end), _tp(grid), grid.shape[0],
                                       int(seed), _stream(stream), ctypes.byref(r)))
    return r.as_dict()


def autotune_backward(model, n_traj, t_end, grid, seed, rates=None, stream=None):
    """Time the backward launch forms and grids on this problem and keep the fastest
    (ssa_autotune_backward); returns the chosen form, grid and the two kernel times."""
    r = TuneResult()
    _check(load().ssa_autotune_backward(model.handle, _tp(rates), int(n_traj), float(t_end), _tp(grid),
                                        grid.shape[0], int(seed), _stream(stream), ctypes.byref(r)))
    return r.as_dict()


def run_jacobian_device(model, n_traj, t_end, grid, seed, rates=None, max_events=0, stream=None,
                        with_stats=False, out=None, log_rates=None):
    """Forward pass with the likelihood-ratio Jacobian (ssa_run_jacobian_device); returns
    (mean (G,S), var (G,S), jac (G,S,M), stats or None)."""
    import torch
    G = grid.shape[0]
    if out is None:
        mean = torch.empty((G, model.S), dtype=torch.float64, device=grid.device)
        var = torch.empty_like(mean)
        jac = torch.empty((G, model.S, model.M), dtype=torch.float64, device=grid.device)
    else:
        mean, var, jac = out
    st = Stats() if with_stats else None
    _check(load().ssa_run_jacobian_device(model.handle, _tp(rates), _tp(log_rates), int(n_traj), float(t_end),
                                          _tp(grid), G, int(seed), int(max_events), _tp(mean), _tp(var), _tp(jac),
                                          _stream(stream), ctypes.byref(st) if st is not None else None))
    return mean, var, jac, (st.as_dict() if st is not None else None)


def run_cov_device(model, n_traj, t_end, grid, seed, rates=None, max_events=0, stream=None, with_stats=False):
    """Grid means (G, S) and species covariance matrices (G, S, S) (ssa_run_cov_device)."""
    import torch
    G = grid.shape[0]
    mean = torch.empty((G, model.S), dtype=torch.float64, device=grid.device)
    cov = torch.empty((G, model.S, model.S), dtype=torch.float64, device=grid.device)
    st = Stats() if with_stats else None
    _check(load().ssa_run_cov_device(model.handle, _tp(rates), int(n_traj), float(t_end), _tp(grid), G, int(seed),
                                     int(max_events), _tp(mean), _tp(cov), _stream(stream),
                                     ctypes.byref(st) if st is not None else None))
    return mean, cov, (st.as_dict() if st is not None else None)


def adaptive_device(model, n_traj, t_end, seed, k, rates=None, max_events=0, stream=None, with_y=False,
                    with_stats=False, device="cuda:0"):
    """Adaptive selective memory (ssa_adaptive_device): Avg-XY points (time (P,), mean and
    variance (P, S)) and, with with_y, the Avg-Y points (time (U,), mean, var (U, S)).
    Sizes come from a first call that only counts (the simulation runs twice)."""
    import torch
    dev = rates.device if rates is not None else torch.device(device)
    L = load()
    npts = (ctypes.c_int64 * 2)()
    _check(L.ssa_adaptive_device(model.handle, _tp(rates), int(n_traj), float(t_end), int(seed), int(max_events),
                                 int(k), None, None, None, 0, None, None, None, 0, npts, _stream(stream), None))
    U, P = int(npts[0]), int(npts[1])
    f64 = dict(dtype=torch.float64, device=dev)
    xt, xm, xv = torch.empty(P, **f64), torch.empty((P, model.S), **f64), torch.empty((P, model.S), **f64)
    yt = ym = yv = None
    if with_y:
        yt, ym, yv = torch.empty(U, **f64), torch.empty((U, model.S), **f64), torch.empty((U, model.S), **f64)
    st = Stats() if with_stats else None
    _check(L.ssa_adaptive_device(model.handle, _tp(rates), int(n_traj), float(t_end), int(seed), int(max_events),
                                 int(k), _tp(xt), _tp(xm), _tp(xv), P, _tp(yt), _tp(ym), _tp(yv), U if with_y else 0,
                                 npts, _stream(stream), ctypes.byref(st) if st is not None else None))
    out = dict(xy_time=xt, xy_mean=xm, xy_var=xv)
    if with_y:
        out.update(y_time=yt, y_mean=ym, y_var=yv)
    if st is not None:
        out["stats"] = st.as_dict()
    return out


def hist_quantiles(hist, spec, n_traj, qs, stream=None):
    """Per-grid-point quantiles from a histogram of run_device (ssa_hist_quantiles);
    hist (G, nbins) int32/uint32 device tensor, spec = (species, lo, width, nbins), qs a
    float64 device tensor; returns (G, len(qs)) int32."""
    import torch
    G = hist.shape[0]
    out = torch.empty((G, qs.shape[0]), dtype=torch.int32, device=hist.device)
    sp = HistSpec(*[int(v) for v in spec])
    _check(load().ssa_hist_quantiles(_tp(hist.contiguous()), G, ctypes.byref(sp), int(n_traj), _tp(qs.contiguous()),
                                     qs.shape[0], _tp(out), _stream(stream)))
    return out


def jacobian_vjp(jac, w, stream=None, out=None):
    """grad[j] = sum_{g,s} w[g,s] jac[g,s,j] on the device (ssa_jacobian_vjp)."""
    import torch
    G, S, M = jac.shape
    grad = torch.empty(M, dtype=torch.float64, device=jac.device) if out is None else out
    _check(load().ssa_jacobian_vjp(_tp(jac.contiguous()), _tp(w.contiguous()), G, S, M, _tp(grad),
                                   _stream(stream)))
    return grad


def record(model, traj_begin, count, t_end, grid, seed, rates=None, max_events=0):
    """Per-trajectory record (ssa_record), host arrays; returns (status, dict) like the oracle's."""
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    G = grid.shape[0]
    states = np.zeros((count, G, model.S), dtype=np.int32)
    events = np.zeros(count, dtype=np.uint64)
    draws = np.zeros(count, dtype=np.uint64)
    t_last = np.zeros(count, dtype=np.float64)
    nf = np.zeros((count, model.M), dtype=np.int64)
    ai = np.zeros((count, model.M), dtype=np.float64)
    r = None if rates is None else np.ascontiguousarray(rates, dtype=np.float64)
    status = load().ssa_record(model.handle, _p(r), int(traj_begin), int(count), float(t_end), _p(grid), G,
                               int(seed), int(max_events), _p(states), _p(events), _p(draws), _p(t_last),
                               _p(nf), _p(ai))
    return status, dict(states=states, events=events, draws=draws, t_last=t_last, n_fired=nf, a_int=ai)


class Batch:
    """Many networks in one persistent launch (ssa_batch_create / ssa_batch_run)."""

    def __init__(self, models, n_traj, t_end, grids, seeds):
        L = load()
        B = len(models)
        self.models = list(models)
        self.grids = [np.ascontiguousarray(g, dtype=np.float64) for g in grids]
        self.G = [g.shape[0] for g in self.grids]
        self.n_traj = [int(v) for v in n_traj]
        hm = (ctypes.c_void_p * B)(*[m.handle.value for m in models])
        nt = (ctypes.c_int64 * B)(*self.n_traj)
        te = (ctypes.c_double * B)(*[float(v) for v in t_end])
        gp = (ctypes.c_void_p * B)(*[g.ctypes.data for g in self.grids])
        ng = (ctypes.c_int32 * B)(*self.G)
        sd = (ctypes.c_uint64 * B)(*[int(v) for v in seeds])
        h = ctypes.c_void_p()
        _check(L.ssa_batch_create(B, hm, nt, te, gp, ng, sd, ctypes.byref(h)))
        self.handle = h

    def run(self, device, stream=None, with_stats=False, outs=None):
        import torch
        B = len(self.models)
        if outs is None:
            means = [torch.empty((self.G[b], self.models[b].S), dtype=torch.float64, device=device) for b in range(B)]
            vars_ = [torch.empty_like(m) for m in means]
        else:
            means, vars_ = outs
        mp = (ctypes.c_void_p * B)(*[m.data_ptr() for m in means])
        vp = (ctypes.c_void_p * B)(*[v.data_ptr() for v in vars_])
        st = Stats() if with_stats else None
        _check(load().ssa_batch_run(self.handle, mp, vp, _stream(stream), ctypes.byref(st) if st is not None else None))
        return means, vars_, (st.as_dict() if st is not None else None)

    def autotune(self, stream=None):
        """Time the LDS window sizes on this batch and keep the fastest (ssa_batch_autotune)."""
        r = TuneResult()
        _check(load().ssa_batch_autotune(self.handle, _stream(stream), ctypes.byref(r)))
        return dict(win_bytes=r.win_bytes, best_ms=r.best_ms, default_ms=r.default_ms)

    def close(self):
        if getattr(self, "handle", None):
            load().ssa_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_function():
    import torch

    class SSAMean(torch.autograd.Function):
        """mean = E[X(t_g)] over n_traj trajectories, differentiable in log rate constants.

        mode "resim": forward ssa_run_device on the log rates (the library forms the rate
        constants on the device); backward the likelihood-ratio kernel (ssa_backward_device)
        re-simulates the same trajectories, centred on the forward mean.  mode "jacobian": the forward pass also forms the
        likelihood-ratio Jacobian (ssa_run_jacobian_device) and the backward is its
        vector-Jacobian product (ssa_jacobian_vjp): one simulation pass in all."""

        @staticmethod
        def forward(ctx, log_rates, model, n_traj, t_end, grid, seed, mode):
            theta = log_rates.detach().contiguous()
            if mode == "jacobian":
                mean, _, jac, _ = run_jacobian_device(model, n_traj, t_end, grid, seed, log_rates=theta)
                ctx.save_for_backward(jac)
            else:
                mean, _, _, _ = run_device(model, n_traj, t_end, grid, seed, log_rates=theta)
                ctx.save_for_backward(theta, mean)
            ctx.cfg = (model, n_traj, t_end, grid, seed, mode)
            return mean

        @staticmethod
        def backward(ctx, grad_mean):
            model, n_traj, t_end, grid, seed, mode = ctx.cfg
            if mode == "jacobian":
                (jac,) = ctx.saved_tensors
                g = jacobian_vjp(jac, grad_mean.contiguous())
            else:
                theta, mean = ctx.saved_tensors
                g, _ = backward_device(model, n_traj, t_end, grid, seed, grad_mean.contiguous(), mean, log_rates=theta)
            return g, None, None, None, None, None, None

    class SSAMoments(torch.autograd.Function):
        """(mean, var) = E[X(t_g)], Var[X(t_g)] over n_traj trajectories, differentiable in log
        rate constants.  Forward ssa_run_device on the log rates; backward one
        re-simulation (ssa_backward_moments_device) with both weight tensors, centred on the
        forward mean and variance."""

        @staticmethod
        def forward(ctx, log_rates, model, n_traj, t_end, grid, seed):
            theta = log_rates.detach().contiguous()
            mean, var, _, _ = run_device(model, n_traj, t_end, grid, seed, log_rates=theta)
            ctx.save_for_backward(theta, mean, var)
            ctx.cfg = (model, n_traj, t_end, grid, seed)
            return mean, var

        @staticmethod
        def backward(ctx, grad_mean, grad_var):
            model, n_traj, t_end, grid, seed = ctx.cfg
            theta, mean, var = ctx.saved_tensors
            if grad_mean is None:
                grad_mean = torch.zeros_like(mean)
            if grad_var is None:
                g, _ = backward_device(model, n_traj, t_end, grid, seed, grad_mean.contiguous(), mean, log_rates=theta)
            else:
                g, _ = backward_device(model, n_traj, t_end, grid, seed, grad_mean.contiguous(), mean, log_rates=theta,
                                       wv=grad_var.contiguous(), vhat=var)
            return g, None, None, None, None, None

    SSAMean.moments = SSAMoments
    return SSAMean


_fn = None


def ssa_moments(log_rates, model, n_traj, t_end, grid, seed):
    """Differentiable grid means and variances (torch.autograd.Function over the HIP
    kernels): returns (mean, var); gradients of a loss on either or both reach log_rates
    through one re-simulating backward."""
    global _fn
    if _fn is None:
        _fn = _make_function()
    return _fn.moments.apply(log_rates, model, n_traj, t_end, grid, seed)


def ssa_mean(log_rates, model, n_traj, t_end, grid, seed, mode="resim"):
    """Differentiable grid means (torch.autograd.Function over the HIP kernels); mode
    "resim" (re-simulating backward) or "jacobian" (Jacobian formed in the forward pass)."""
    global _fn
    if _fn is None:
        _fn = _make_function()
    if mode not in ("resim", "jacobian"):
        raise ValueError("mode must be 'resim' or 'jacobian'")
    return _fn.apply(log_rates, model, n_traj, t_end, grid, seed, mode)
