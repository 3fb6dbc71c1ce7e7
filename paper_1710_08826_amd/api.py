"""Python surface of libfitnll: argument marshalling only.

Device memory and streams come from PyTorch (ROCm build): event tensors are
float64 CUDA tensors of shape (n_obs, n) (structure of arrays), and calls run
on ``torch.cuda.current_stream()`` unless a stream is given.  Every
computation runs in the HIP kernels behind the C ABI.
"""
from __future__ import annotations

import ctypes as C
import json
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check

_ctx = {}


def context(device: int = 0):
    """The library context of a device (created once)."""
    if device not in _ctx:
        lib = _lib.load()
        h = C.c_void_p()
        check(lib.fn_ctx_create(int(device), C.byref(h)))
        _ctx[device] = h
    return _ctx[device]


def _dbl(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _events(ev: torch.Tensor, n_obs: int):
    if not isinstance(ev, torch.Tensor) or not ev.is_cuda or ev.dtype != torch.float64:
        raise TypeError("events must be a float64 CUDA tensor")
    if ev.dim() == 1:
        ev = ev.unsqueeze(0)
    if ev.dim() != 2 or ev.shape[0] != n_obs:
        raise ValueError(f"events must have shape ({n_obs}, n)")
    n = ev.shape[1]
    if n > 1 and ev.stride(1) != 1:
        raise ValueError("events must be contiguous along the event axis")
    ld = ev.stride(0) if n_obs > 1 else n
    return C.c_void_p(ev.data_ptr() if n > 0 else 0), n, ld


@dataclass
class FitResult:
    theta: np.ndarray
    errors: np.ndarray
    nll: float
    n_iter: int
    n_calls: int
    status: int


class Model:
    """A compiled model on one device (see fn_model_create for descriptions)."""

    def __init__(self, desc: dict | str, device: int = 0):
        lib = _lib.load()
        self._lib = lib
        self.desc = desc if isinstance(desc, dict) else json.loads(desc)
        self.device = device
        h = C.c_void_p()
        check(lib.fn_model_create(context(device), json.dumps(self.desc).encode(), C.byref(h)))
        self._h = h
        p, o, c = C.c_int32(), C.c_int32(), C.c_int32()
        check(lib.fn_model_info(h, C.byref(p), C.byref(o), C.byref(c)))
        self.n_params, self.n_obs, self.chunk = p.value, o.value, c.value
        self.events_per_thread = int(self.desc.get("events_per_thread", 1))
        self.tune_table = {}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fn_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _theta(self, theta):
        a, ptr = _dbl(theta)
        if a.size != self.n_params:
            raise ValueError(f"theta must have {self.n_params} entries")
        return a, ptr

    def nll(self, theta, events: torch.Tensor, grad: bool = False, stream=None):
        """NLL (and gradient as a numpy array when grad=True)."""
        th, thp = self._theta(theta)
        evp, n, ld = _events(events, self.n_obs)
        out = C.c_double()
        g = np.zeros(self.n_params)
        gp = g.ctypes.data_as(C.POINTER(C.c_double)) if grad else None
        check(self._lib.fn_nll(self._h, thp, evp, n, ld, C.byref(out), gp, _stream_ptr(stream)))
        return (out.value, g) if grad else out.value

    def nll_async(self, theta_dev: torch.Tensor, events: torch.Tensor, out_dev: torch.Tensor,
                  with_grad: bool = True, stream=None):
        """Enqueue NLL (+grad) with device theta; out_dev gets 1+P doubles."""
        evp, n, ld = _events(events, self.n_obs)
        assert theta_dev.is_cuda and theta_dev.dtype == torch.float64 and theta_dev.numel() >= self.n_params
        assert out_dev.is_cuda and out_dev.dtype == torch.float64 and out_dev.numel() >= 1 + self.n_params
        check(self._lib.fn_nll_async(self._h, C.c_void_p(theta_dev.data_ptr()), evp, n, ld,
                                     C.c_void_p(out_dev.data_ptr()), 1 if with_grad else 0,
                                     _stream_ptr(stream)))

    def nll_async_noalloc(self, theta_dev: torch.Tensor, events: torch.Tensor, out_dev: torch.Tensor,
                          with_grad: bool = True, stream=None):
        """nll_async whose partial rows live in the library's static scratch
        array: no allocation; calls on one device must not overlap."""
        evp, n, ld = _events(events, self.n_obs)
        assert theta_dev.is_cuda and theta_dev.dtype == torch.float64 and theta_dev.numel() >= self.n_params
        assert out_dev.is_cuda and out_dev.dtype == torch.float64 and out_dev.numel() >= 1 + self.n_params
        check(self._lib.fn_nll_async_noalloc(self._h, C.c_void_p(theta_dev.data_ptr()), evp, n, ld,
                                             C.c_void_p(out_dev.data_ptr()), 1 if with_grad else 0,
                                             _stream_ptr(stream)))

    def norm(self, theta, stream=None):
        """(I, dI/dtheta)."""
        th, thp = self._theta(theta)
        out = C.c_double()
        g = np.zeros(self.n_params)
        check(self._lib.fn_norm(self._h, thp, C.byref(out), g.ctypes.data_as(C.POINTER(C.c_double)),
                                _stream_ptr(stream)))
        return out.value, g

    def eval(self, theta, events: torch.Tensor, stream=None) -> torch.Tensor:
        """Normalized density per event (device tensor)."""
        th, thp = self._theta(theta)
        evp, n, ld = _events(events, self.n_obs)
        p = torch.empty(n, dtype=torch.float64, device=events.device)
        check(self._lib.fn_eval(self._h, thp, evp, n, ld, C.c_void_p(p.data_ptr() if n else 0),
                                _stream_ptr(stream)))
        return p

    def set_norm_sample(self, mc: torch.Tensor, stream=None):
        """td4: phase-space sample (5, n_mc) float64 CUDA tensor defining I."""
        if not isinstance(mc, torch.Tensor) or not mc.is_cuda or mc.dtype != torch.float64:
            raise TypeError("the sample must be a float64 CUDA tensor")
        if mc.dim() != 2 or mc.shape[0] != 5 or mc.stride(1) != 1:
            raise ValueError("the sample must have shape (5, n_mc), contiguous along points")
        check(self._lib.fn_model_set_norm_sample(self._h, C.c_void_p(mc.data_ptr()), mc.shape[1], mc.stride(0),
                                                 _stream_ptr(stream)))

    def generate_norm_sample(self, n_mc: int, seed: int, fit: int = 0, stream=None):
        """td4: generate the n_mc-point phase-space normalization sample on the
        device (fn_model_generate_norm_sample)."""
        check(self._lib.fn_model_generate_norm_sample(self._h, C.c_uint32(seed & 0xFFFFFFFF),
                                                      C.c_uint32(fit & 0xFFFFFFFF), int(n_mc),
                                                      _stream_ptr(stream)))

    def fixed(self) -> np.ndarray:
        """td4: the description's fixed-constant vector."""
        n = C.c_int32()
        check(self._lib.fn_model_fixed(self._h, C.byref(n), None))
        v = np.zeros(n.value)
        check(self._lib.fn_model_fixed(self._h, None, v.ctypes.data_as(C.POINTER(C.c_double))))
        return v

    def generate(self, theta, n: int, seed: int, fit: int = 0, envelope: float = 0.0, stream=None):
        """dalitz3, tddp3, td4: n toy events at theta by accept-reject on the
        device, as an (n_obs, n) float64 CUDA tensor, and the envelope used
        (fn_generate)."""
        th, thp = self._theta(theta)
        ev = torch.empty((self.n_obs, n), dtype=torch.float64, device=f"cuda:{self.device}")
        used = C.c_double()
        check(self._lib.fn_generate(self._h, thp, C.c_uint32(seed & 0xFFFFFFFF), C.c_uint32(fit & 0xFFFFFFFF),
                                    int(n), float(envelope), C.c_void_p(ev.data_ptr() if n else 0), int(n),
                                    C.byref(used), _stream_ptr(stream)))
        return ev, used.value

    TUNE_MAX = 16  # FN_TUNE_MAX
    TUNE_EPT = 2   # FN_TUNE_EPT

    def autotune(self, theta, events: torch.Tensor, reps: int = 20, stream=None):
        """Pick the summation chunk (and for dalitz3 the events per thread and
        loop iteration, 1 or 2) for these events (fn_model_autotune: among the
        candidates within 2% of the fastest, one event per thread if any, then
        the largest chunk; chunk candidates are the powers of two 256..16384
        and the chunks giving j x (compute units) workgroups, j = 1..8);
        returns (chunk, {candidate chunk: median microseconds per NLL +
        gradient at the chosen events per thread}); every timing is in
        self.tune_table, keyed by (chunk, events per thread)."""
        th, thp = self._theta(theta)
        evp, n, ld = _events(events, self.n_obs)
        best, ept = C.c_int32(), C.c_int32()
        chunks = (C.c_int32 * self.TUNE_MAX)()
        us = (C.c_double * (self.TUNE_EPT * self.TUNE_MAX))()
        check(self._lib.fn_model_autotune(self._h, thp, evp, n, ld, int(reps), C.byref(best), C.byref(ept), chunks,
                                          us, _stream_ptr(stream)))
        self.chunk = best.value
        self.events_per_thread = ept.value
        self.tune_table = {}
        for e in range(self.TUNE_EPT):
            for i, c in enumerate(chunks):
                t = us[e * self.TUNE_MAX + i]
                if c > 0 and not math.isnan(t):
                    self.tune_table[(c, e + 1)] = t
        return best.value, {c: t for (c, e), t in self.tune_table.items() if e == ept.value}

    def set_timing(self, enable: bool, every: int = 1, span: bool = False):
        """Time every `every`-th per-event kernel launch (the dispatch records its own
        start and end into a pair of HIP events); span=True (dalitz3): every
        launch, graph replays included, measures its own span on the device."""
        check(self._lib.fn_model_timing(self._h, (-1 if span else every) if enable else 0))

    def kernel_time(self):
        """(total ms, launches) of timed per-event kernels since the last query."""
        ms = C.c_double()
        cnt = C.c_int64()
        check(self._lib.fn_model_kernel_time(self._h, C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    def check_events(self, events: torch.Tensor, stream=None) -> int:
        """Number of events outside the observable domain (0 if all inside)."""
        evp, n, ld = _events(events, self.n_obs)
        bad = C.c_int64()
        st = self._lib.fn_events_check(self._h, evp, n, ld, C.byref(bad), _stream_ptr(stream))
        if st not in (_lib.FN_OK, _lib.FN_E_DOMAIN):
            check(st)
        return bad.value

    def fit(self, theta0, events: torch.Tensor, free=None, grad_mode: str = "adjoint",
            tol: float = 1e-7, max_iter: int = 500, errors: bool = True, stream=None,
            raise_on_fail: bool = True) -> FitResult:
        """Quasi-Newton fit on the device NLL (grad_mode 'adjoint' or 'fd')."""
        th, thp = self._theta(theta0)
        evp, n, ld = _events(events, self.n_obs)
        mask = None
        if free is not None:
            m = np.ascontiguousarray(np.asarray(free, dtype=np.int32))
            mask = m.ctypes.data_as(C.POINTER(C.c_int32))
        out_t = np.zeros(self.n_params)
        out_e = np.zeros(self.n_params)
        nll = C.c_double()
        it, calls = C.c_int32(), C.c_int32()
        st = self._lib.fn_fit(self._h, thp, mask, evp, n, ld, 0 if grad_mode == "adjoint" else 1, tol, max_iter,
                              out_t.ctypes.data_as(C.POINTER(C.c_double)),
                              out_e.ctypes.data_as(C.POINTER(C.c_double)) if errors else None,
                              C.byref(nll), C.byref(it), C.byref(calls), _stream_ptr(stream))
        if st != _lib.FN_OK and raise_on_fail:
            check(st)
        return FitResult(out_t, out_e, nll.value, it.value, calls.value, st)

    _STATS = {"poisson": 0, "chi2": 1}

    @staticmethod
    def _counts(counts: torch.Tensor):
        if not isinstance(counts, torch.Tensor) or not counts.is_cuda or counts.dtype != torch.float64:
            raise TypeError("counts must be a float64 CUDA tensor")
        if counts.dim() != 1 or (counts.numel() > 1 and counts.stride(0) != 1):
            raise ValueError("counts must be a contiguous 1-D tensor")
        return C.c_void_p(counts.data_ptr() if counts.numel() else 0), counts.numel()

    def nll_binned(self, theta, counts: torch.Tensor, stat: str = "poisson", grad: bool = False, stream=None):
        """mix1d: binned Poisson NLL or chi^2 of histogram counts on uniform bins
        over [lo, hi] (fn_nll_binned); (value, gradient) when grad=True."""
        th, thp = self._theta(theta)
        cp, nb = self._counts(counts)
        v = C.c_double()
        g = np.zeros(self.n_params)
        check(self._lib.fn_nll_binned(self._h, thp, cp, nb, self._STATS[stat], C.byref(v),
                                      g.ctypes.data_as(C.POINTER(C.c_double)) if grad else None,
                                      _stream_ptr(stream)))
        return (v.value, g) if grad else v.value

    def fit_binned(self, theta0, counts: torch.Tensor, stat: str = "poisson", free=None,
                   grad_mode: str = "adjoint", tol: float = 1e-7, max_iter: int = 500, errors: bool = True,
                   stream=None, raise_on_fail: bool = True) -> FitResult:
        """Quasi-Newton fit of binned data (fn_fit_binned); FitResult.nll holds
        the minimum of the statistic."""
        th, thp = self._theta(theta0)
        cp, nb = self._counts(counts)
        mask = None
        if free is not None:
            mk = np.ascontiguousarray(np.asarray(free, dtype=np.int32))
            mask = mk.ctypes.data_as(C.POINTER(C.c_int32))
        out_t = np.zeros(self.n_params)
        out_e = np.zeros(self.n_params)
        val = C.c_double()
        it, calls = C.c_int32(), C.c_int32()
        st = self._lib.fn_fit_binned(self._h, thp, mask, cp, nb, self._STATS[stat],
                                     0 if grad_mode == "adjoint" else 1, tol, max_iter,
                                     out_t.ctypes.data_as(C.POINTER(C.c_double)),
                                     out_e.ctypes.data_as(C.POINTER(C.c_double)) if errors else None,
                                     C.byref(val), C.byref(it), C.byref(calls), _stream_ptr(stream))
        if st != _lib.FN_OK and raise_on_fail:
            check(st)
        return FitResult(out_t, out_e, val.value, it.value, calls.value, st)


class NLLFunction(torch.autograd.Function):
    """NLL as a differentiable function of theta (a float64 tensor, CPU or
    CUDA): ``NLLFunction.apply(theta, model, events)``.

    forward runs the device NLL with the adjoint gradient (fn_nll); backward
    returns grad_output times that gradient.  The result and the gradient live
    on theta's device.
    """

    @staticmethod
    def forward(ctx, theta: torch.Tensor, model: Model, events: torch.Tensor):
        v, g = model.nll(theta.detach().cpu().numpy(), events, grad=True)
        ctx.save_for_backward(torch.from_numpy(g).to(device=theta.device, dtype=theta.dtype))
        return torch.tensor(v, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None


@dataclass
class BatchResults:
    status: np.ndarray
    theta: np.ndarray
    nll: np.ndarray
    errors: np.ndarray
    iters: np.ndarray
    n_evals: np.ndarray


class Batch:
    """Slots of independent fits of one mix1d model advanced together on the
    device (see fn_batch_* in include/fitnll.h)."""

    def __init__(self, model: Model, max_fits: int, max_events_per_fit: int):
        self.model = model
        self._lib = model._lib
        self.max_fits = max_fits
        h = C.c_void_p()
        check(self._lib.fn_batch_create(model._h, int(max_fits), int(max_events_per_fit), C.byref(h)))
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fn_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def config(self, tol: float = 1e-7, max_iter: int = 500, use_graph: bool = True):
        check(self._lib.fn_batch_config(self._h, float(tol), int(max_iter), 1 if use_graph else 0))

    def set_slot(self, slot: int, events: torch.Tensor, theta0, free=None):
        evp, n, _ = _events(events, 1)
        th, thp = _dbl(theta0)
        mask = None
        if free is not None:
            m = np.ascontiguousarray(np.asarray(free, dtype=np.int32))
            mask = m.ctypes.data_as(C.POINTER(C.c_int32))
        check(self._lib.fn_batch_set_slot(self._h, int(slot), evp, n, thp, mask))
        self._keep[slot] = events  # the slot reads these events until cleared

    def clear_slot(self, slot: int):
        check(self._lib.fn_batch_clear_slot(self._h, int(slot)))
        self._keep.pop(slot, None)

    def set(self, events, theta0_dev: torch.Tensor):
        """fn_batch_set: fit f of len(events) reads events[f] (a (1, n_f)
        float64 CUDA tensor) from theta0_dev[f] (device, n_fits x P), all
        parameters free; the remaining slots become idle."""
        evs = list(events)
        F = len(evs)
        P = self.model.n_params
        if F > 0:
            assert theta0_dev.is_cuda and theta0_dev.dtype == torch.float64 and theta0_dev.is_contiguous()
            assert theta0_dev.numel() >= F * P
        ptrs = (C.c_void_p * max(F, 1))()
        ns = (C.c_int64 * max(F, 1))()
        lds = (C.c_int64 * max(F, 1))()
        for f, ev in enumerate(evs):
            p, n, ld = _events(ev, 1)
            ptrs[f], ns[f], lds[f] = p.value, n, ld
        torch.cuda.current_stream().synchronize()  # theta0_dev must be ready
        check(self._lib.fn_batch_set(self._h, F, ptrs, ns, lds,
                                     C.c_void_p(theta0_dev.data_ptr() if F > 0 else 0)))
        self._keep = dict(enumerate(evs))

    def step(self, stream=None):
        """fn_batch_step: one NLL + gradient + BFGS step of every running fit,
        enqueued on the stream (capturable into the caller's graph)."""
        check(self._lib.fn_batch_step(self._h, _stream_ptr(stream)))

    def status(self):
        """fn_batch_status: (status, theta, nll, errors) per slot."""
        n, P = self.max_fits, self.model.n_params
        st = np.zeros(n, np.int32)
        th = np.zeros((n, P))
        nll = np.zeros(n)
        er = np.zeros((n, P))
        f64p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        check(self._lib.fn_batch_status(self._h, st.ctypes.data_as(C.POINTER(C.c_int32)), f64p(th), f64p(nll),
                                        f64p(er)))
        return st, th, nll, er

    def run(self, max_steps: int = 2000, poll_every: int = 8):
        done, running = C.c_int32(), C.c_int32()
        check(self._lib.fn_batch_run(self._h, int(max_steps), int(poll_every), C.byref(done), C.byref(running)))
        return done.value, running.value

    def results(self) -> BatchResults:
        n, P = self.max_fits, self.model.n_params
        st = np.zeros(n, np.int32)
        th = np.zeros((n, P))
        nll = np.zeros(n)
        er = np.zeros((n, P))
        it = np.zeros(n, np.int32)
        ne = np.zeros(n, np.int32)
        i32p = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        f64p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        check(self._lib.fn_batch_results(self._h, i32p(st), f64p(th), f64p(nll), f64p(er), i32p(it), i32p(ne)))
        return BatchResults(st, th, nll, er, it, ne)


class VariationBatch:
    """Fits of one td4 model to one event sample that differ in their fixed
    constants (see fn_vbatch_* in include/fitnll.h)."""

    def __init__(self, model: Model, n_fits: int):
        self.model = model
        self._lib = model._lib
        self.n_fits = int(n_fits)
        h = C.c_void_p()
        check(self._lib.fn_vbatch_create(model._h, self.n_fits, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fn_vbatch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fixed(self, fit: int, fixed=None):
        if fixed is None:
            check(self._lib.fn_vbatch_set_fixed(self._h, int(fit), None))
            return
        a, p = _dbl(fixed)
        check(self._lib.fn_vbatch_set_fixed(self._h, int(fit), p))

    def _thetas(self, theta):
        a = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        if a.shape != (self.n_fits, self.model.n_params):
            raise ValueError(f"theta must have shape ({self.n_fits}, {self.model.n_params})")
        return a

    def nll(self, theta, events: torch.Tensor, grad: bool = False, stream=None):
        th = self._thetas(theta)
        evp, n, ld = _events(events, self.model.n_obs)
        v = np.zeros(self.n_fits)
        g = np.zeros((self.n_fits, self.model.n_params))
        f64p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        check(self._lib.fn_vbatch_nll(self._h, f64p(th), evp, n, ld, f64p(v), f64p(g) if grad else None,
                                      _stream_ptr(stream)))
        return (v, g) if grad else v

    def fit(self, theta0, events: torch.Tensor, free=None, tol: float = 1e-7, max_iter: int = 500,
            use_graph: bool = True, stream=None) -> BatchResults:
        th = self._thetas(theta0)
        evp, n, ld = _events(events, self.model.n_obs)
        F, P = self.n_fits, self.model.n_params
        mask = None
        if free is not None:
            mk = np.ascontiguousarray(np.asarray(free, dtype=np.int32))
            mask = mk.ctypes.data_as(C.POINTER(C.c_int32))
        st = np.zeros(F, np.int32)
        x = np.zeros((F, P))
        er = np.zeros((F, P))
        v = np.zeros(F)
        it = np.zeros(F, np.int32)
        ne = np.zeros(F, np.int32)
        i32p = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        f64p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        check(self._lib.fn_vbatch_fit(self._h, f64p(th), mask, evp, n, ld, float(tol), int(max_iter),
                                      1 if use_graph else 0, i32p(st), f64p(x), f64p(er), f64p(v), i32p(it),
                                      i32p(ne), _stream_ptr(stream)))
        return BatchResults(st, x, v, er, it, ne)

    def serve(self, requests, events: torch.Tensor, free=None, tol: float = 1e-7, max_iter: int = 500,
              poll_every: int = 2, stream=None) -> dict:
        """Continuous serving of variation requests on this batch's slots.
        requests: sequence of (id, arrival_s, fixed or None, theta0).  Returns
        per-request arrays in request order: id, status, theta, errors, nll,
        iters, n_evals, t_admit, t_done (seconds after the call starts)."""
        evp, n, ld = _events(events, self.model.n_obs)
        P = self.model.n_params
        R = len(requests)
        keep = []
        arr = (_VRequest * max(R, 1))()
        for i, (rid, arrival, fixed, theta0) in enumerate(requests):
            th = np.ascontiguousarray(np.asarray(theta0, dtype=np.float64))
            if th.size != P:
                raise ValueError(f"theta0 must have {P} entries")
            keep.append(th)
            arr[i].id = int(rid)
            arr[i].arrival_s = float(arrival)
            arr[i].theta0 = th.ctypes.data_as(C.POINTER(C.c_double))
            if fixed is None:
                arr[i].fixed = None
            else:
                fx = np.ascontiguousarray(np.asarray(fixed, dtype=np.float64))
                keep.append(fx)
                arr[i].fixed = fx.ctypes.data_as(C.POINTER(C.c_double))
        mask = None
        if free is not None:
            mk = np.ascontiguousarray(np.asarray(free, dtype=np.int32))
            keep.append(mk)
            mask = mk.ctypes.data_as(C.POINTER(C.c_int32))
        out = {"id": np.array([int(r[0]) for r in requests], np.int64), "status": np.zeros(R, np.int32),
               "theta": np.zeros((R, P)), "errors": np.zeros((R, P)), "nll": np.zeros(R),
               "iters": np.zeros(R, np.int32), "n_evals": np.zeros(R, np.int32),
               "t_admit": np.zeros(R), "t_done": np.zeros(R)}
        i32p = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        f64p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        check(self._lib.fn_vbatch_serve(self._h, C.cast(arr, C.c_void_p), R, mask, evp, n, ld, float(tol),
                                        int(max_iter), int(poll_every), i32p(out["status"]), f64p(out["theta"]),
                                        f64p(out["errors"]), f64p(out["nll"]), i32p(out["iters"]),
                                        i32p(out["n_evals"]), f64p(out["t_admit"]), f64p(out["t_done"]),
                                        _stream_ptr(stream)))
        return out


class _VRequest(C.Structure):
    _fields_ = [("id", C.c_int64), ("arrival_s", C.c_double), ("fixed", C.POINTER(C.c_double)),
                ("theta0", C.POINTER(C.c_double))]


def generate_mix1d(n: int, seed: int, fit: int, theta_gen, lo: float = -10.0, hi: float = 10.0,
                   device: str = "cuda", stream=None) -> torch.Tensor:
    """Device toy events of the Gaussian + exponential mixture, shape (1, n)."""
    lib = _lib.load()
    th, thp = _dbl(theta_gen)
    x = torch.empty((1, n), dtype=torch.float64, device=device)
    check(lib.fn_generate_mix1d(C.c_uint32(seed & 0xFFFFFFFF), C.c_uint32(fit & 0xFFFFFFFF), int(n), thp,
                                float(lo), float(hi), C.c_void_p(x.data_ptr() if n else 0), _stream_ptr(stream)))
    return x


class _Request(C.Structure):
    _fields_ = [("id", C.c_int64), ("n_events", C.c_int64), ("seed", C.c_uint32), ("fit", C.c_uint32),
                ("events", C.c_void_p), ("theta_gen", C.c_double * 4), ("theta0", C.c_double * 24),
                ("arrival_s", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("id", C.c_int64), ("status", C.c_int32), ("iters", C.c_int32), ("n_evals", C.c_int32),
                ("pad", C.c_int32), ("nll", C.c_double), ("theta", C.c_double * 24), ("errors", C.c_double * 24),
                ("t_arrival", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


@dataclass
class ServeResult:
    id: int
    status: int
    iters: int
    n_evals: int
    nll: float
    theta: np.ndarray
    errors: np.ndarray
    t_arrival: float
    t_admit: float
    t_done: float

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Server:
    """Continuous-batching request loop for toy fits of a mix1d model (see
    fn_server_* in include/fitnll.h)."""

    def __init__(self, model: Model, max_slots: int, max_events_per_fit: int, budget_bytes: int):
        self.model = model
        self._lib = model._lib
        h = C.c_void_p()
        check(self._lib.fn_server_create(model._h, int(max_slots), int(max_events_per_fit), int(budget_bytes),
                                         C.byref(h)))
        self._h = h
        self._keep = []
        self._n_submitted = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fn_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, requests):
        """requests: iterable of dicts with id, n_events, theta0, arrival_s and
        either (seed, fit, theta_gen) or events (a (1, n) float64 CUDA tensor)."""
        reqs = list(requests)
        arr = (_Request * len(reqs))()
        P = self.model.n_params
        for i, q in enumerate(reqs):
            r = arr[i]
            r.id = int(q["id"])
            r.n_events = int(q["n_events"])
            r.seed = int(q.get("seed", 0)) & 0xFFFFFFFF
            r.fit = int(q.get("fit", 0)) & 0xFFFFFFFF
            ev = q.get("events")
            if ev is not None:
                self._keep.append(ev)
                r.events = ev.data_ptr()
            else:
                r.events = None
            for j, v in enumerate(q.get("theta_gen", [0.0, 1.0, 0.0, 0.0])[:4]):
                r.theta_gen[j] = float(v)
            for j, v in enumerate(list(q["theta0"])[:P]):
                r.theta0[j] = float(v)
            r.arrival_s = float(q.get("arrival_s", 0.0))
        check(self._lib.fn_server_submit(self._h, arr, len(reqs)))
        self._n_submitted += len(reqs)

    def run(self, poll_every: int = 4, max_seconds: float = 0.0) -> int:
        n = C.c_int32()
        check(self._lib.fn_server_run(self._h, int(poll_every), float(max_seconds), C.byref(n)))
        return n.value

    def results(self):
        cap = max(self._n_submitted, 1)
        arr = (_Result * cap)()
        n = C.c_int32()
        check(self._lib.fn_server_results(self._h, arr, cap, C.byref(n)))
        P = self.model.n_params
        out = []
        for i in range(n.value):
            r = arr[i]
            out.append(ServeResult(r.id, r.status, r.iters, r.n_evals, r.nll, np.array(r.theta[:P]),
                                   np.array(r.errors[:P]), r.t_arrival, r.t_admit, r.t_done))
        return out
