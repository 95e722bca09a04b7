"""Multi-messenger Wiener filter on AMD MI355X (gfx950): Python binding.

A thin ctypes layer over ``libwf.so`` (C ABI in ``include/wf.h``).  Every
step of the filter runs in the library's HIP kernels; this module only
checks tensor shapes and dtypes and passes device pointers and the current
HIP stream.  PyTorch provides device memory and streams.  There is no
fallback: if the library is missing, ``load()`` raises.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "load", "Context", "Schedule", "solve", "rfft2", "irfft2", "strerror",
    "WFError", "STATUS", "CHAINS", "solve_batch", "solve_noalloc", "solve_refined",
]

_LIB_PATH = os.environ.get("WF_LIBRARY") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libwf.so")
_lib = None

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "ENOTPD", -3: "ENONFINITE",
          -4: "EDEVICE", -5: "ENOMEM", -6: "EUNSUPPORTED", -7: "ESCRATCH"}
CHAINS = {"three": 0, "merged": 1, "augmented": 2}
# columns of a trace row: sweep, lambda, rho, dd2, rho_mask, chi2_joint
TRACE_COLS = 6


class WFError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({strerror(status)})")


class _Shape(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int32), ("nx", ctypes.c_int32), ("precision", ctypes.c_int32)]


class _Inputs(ctypes.Structure):
    _fields_ = [("d", ctypes.c_void_p), ("s_k", ctypes.c_void_p), ("n_pix", ctypes.c_void_p),
                ("p_oof", ctypes.c_void_p), ("p_stripe", ctypes.c_void_p),
                ("mask", ctypes.c_void_p)]


class _Schedule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("lam", ctypes.POINTER(ctypes.c_double)),
                ("n_lambda", ctypes.c_int32), ("lambda0", ctypes.c_double),
                ("shrink_exp", ctypes.c_double), ("plateau_rtol", ctypes.c_double),
                ("snap_eps", ctypes.c_double), ("rtol", ctypes.c_double),
                ("max_sweeps", ctypes.c_int32), ("monitor_every", ctypes.c_int32),
                ("beta", ctypes.c_double * 3), ("floor_frac", ctypes.c_double),
                ("chain", ctypes.c_int32), ("stop_full", ctypes.c_int32),
                ("field_mode", ctypes.c_int32)]


class _Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("n_records", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("lam", ctypes.c_double), ("rho", ctypes.c_double),
                ("rho_mask", ctypes.c_double), ("dd2", ctypes.c_double),
                ("d2", ctypes.c_double), ("chi2_joint", ctypes.c_double),
                ("masked_x_norm", ctypes.c_double), ("tau", ctypes.c_double * 3),
                ("phi", ctypes.c_double), ("kernel_ms", ctypes.c_double * 4),
                ("kernel_launches", ctypes.c_int32 * 4), ("refine_rounds", ctypes.c_int32)]


EXPORTS = ("wf_ctx_create", "wf_ctx_destroy", "wf_schedule_default", "wf_solve", "wf_rfft2",
           "wf_irfft2", "wf_ctx_set_profiling", "wf_supported", "wf_strerror", "wf_tile_count",
           "wf_ctx_set_tile", "wf_ctx_get_tile", "wf_inverse_noise_weight", "wf_solve_batch",
           "wf_solve_noalloc", "wf_noalloc_scratch_bytes", "wf_solve_refined", "wf_autotune",
           "wf_autotune_batch")


def load():
    """Load libwf.so (built by ``paper_1704_00865_amd.build``).  Raises if it
    is missing: the package has no CPU path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing; build it with "
                          "`python -m paper_1704_00865_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.wf_ctx_create.argtypes = [ctypes.POINTER(_Shape), ctypes.POINTER(vp)]
    lib.wf_ctx_create.restype = i32
    lib.wf_ctx_destroy.argtypes = [vp]
    lib.wf_ctx_destroy.restype = None
    lib.wf_schedule_default.argtypes = [ctypes.POINTER(_Schedule)]
    lib.wf_schedule_default.restype = None
    lib.wf_solve.argtypes = [vp, ctypes.POINTER(_Inputs), ctypes.POINTER(_Schedule), vp, vp,
                             ctypes.POINTER(_Report), ctypes.POINTER(ctypes.c_double), vp]
    lib.wf_solve.restype = i32
    lib.wf_inverse_noise_weight.argtypes = [vp, ctypes.POINTER(_Inputs), ctypes.c_double,
                                            ctypes.POINTER(_Schedule), vp, vp,
                                            ctypes.POINTER(_Report),
                                            ctypes.POINTER(ctypes.c_double), vp]
    lib.wf_inverse_noise_weight.restype = i32
    lib.wf_solve_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(_Inputs),
                                   ctypes.POINTER(_Schedule), ctypes.POINTER(vp),
                                   ctypes.POINTER(vp), ctypes.POINTER(_Report), vp]
    lib.wf_solve_batch.restype = i32
    lib.wf_solve_noalloc.argtypes = [ctypes.POINTER(_Shape), ctypes.POINTER(_Inputs),
                                     ctypes.POINTER(_Schedule), vp, vp, ctypes.POINTER(_Report),
                                     ctypes.POINTER(ctypes.c_double), vp]
    lib.wf_solve_noalloc.restype = i32
    lib.wf_noalloc_scratch_bytes.argtypes = []
    lib.wf_noalloc_scratch_bytes.restype = ctypes.c_size_t
    lib.wf_solve_refined.argtypes = [vp, vp, ctypes.POINTER(_Inputs), ctypes.POINTER(_Schedule),
                                     ctypes.POINTER(_Schedule), i32, ctypes.c_double, vp, vp,
                                     ctypes.POINTER(_Report), ctypes.POINTER(ctypes.c_double), vp]
    lib.wf_solve_refined.restype = i32
    lib.wf_autotune.argtypes = [vp, ctypes.POINTER(_Inputs), i32, vp,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32), vp]
    lib.wf_autotune.restype = i32
    lib.wf_autotune_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(_Inputs), i32,
                                      ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(i32), vp]
    lib.wf_autotune_batch.restype = i32
    lib.wf_rfft2.argtypes = [vp, vp, vp, vp]
    lib.wf_rfft2.restype = i32
    lib.wf_irfft2.argtypes = [vp, vp, vp, vp]
    lib.wf_irfft2.restype = i32
    lib.wf_ctx_set_profiling.argtypes = [vp, i32]
    lib.wf_ctx_set_profiling.restype = i32
    lib.wf_supported.argtypes = [i32, i32, i32]
    lib.wf_supported.restype = i32
    lib.wf_tile_count.argtypes = []
    lib.wf_tile_count.restype = i32
    lib.wf_ctx_set_tile.argtypes = [vp, i32]
    lib.wf_ctx_set_tile.restype = i32
    lib.wf_ctx_get_tile.argtypes = [vp]
    lib.wf_ctx_get_tile.restype = i32
    lib.wf_strerror.argtypes = [i32]
    lib.wf_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(status: int) -> str:
    if _lib is None:
        return STATUS.get(status, str(status))
    return _lib.wf_strerror(int(status)).decode()


@dataclass
class Schedule:
    """Cooling schedule and solver options (mirrors ``wf_schedule``).

    lambdas: a fixed lambda per sweep (last value repeats); None = adaptive
    (Section 3.3: start at lambda0, lambda <- lambda^shrink when the residual
    plateaus, snap to 1)."""
    lambdas: Optional[Sequence[float]] = None
    lambda0: float = 1.0e4
    shrink: float = 0.7
    plateau: float = 1.0e-2
    snap: float = 1.0e-3
    rtol: float = 1.0e-6
    max_sweeps: int = 20000
    monitor_every: int = 16
    beta: Sequence[float] = (0.9, 0.9, 1.0)
    floor_frac: float = 0.5
    chain: str = "three"
    stop_full: bool = False
    chain_field: bool = False

    def _c(self):
        s = _Schedule()
        keep = None
        if self.lambdas is not None:
            arr = np.ascontiguousarray(np.asarray(self.lambdas, dtype=np.float64))
            keep = arr
            s.kind = 0
            s.lam = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            s.n_lambda = arr.size
        else:
            s.kind = 1
            s.n_lambda = 0
        s.lambda0 = self.lambda0
        s.shrink_exp = self.shrink
        s.plateau_rtol = self.plateau
        s.snap_eps = self.snap
        s.rtol = self.rtol
        s.max_sweeps = int(self.max_sweeps)
        s.monitor_every = int(self.monitor_every)
        for i in range(3):
            s.beta[i] = float(self.beta[i])
        s.floor_frac = self.floor_frac
        s.chain = CHAINS[self.chain]
        s.stop_full = 1 if self.stop_full else 0
        s.field_mode = 1 if self.chain_field else 0
        return s, keep


def _inputs(d, s_k, n_pix, p_oof, p_stripe, mask):
    def ptr(t):
        return t.data_ptr() if t is not None else None
    return _Inputs(ptr(d), ptr(s_k), ptr(n_pix), ptr(p_oof), ptr(p_stripe), ptr(mask))


def _report(rep) -> dict:
    return dict(status=STATUS[rep.status], sweeps=rep.sweeps, n_records=rep.n_records,
                n_levels=rep.n_levels, lam=rep.lam, rho=rep.rho, rho_mask=rep.rho_mask,
                dd2=rep.dd2, d2=rep.d2, chi2_joint=rep.chi2_joint,
                masked_x_norm=rep.masked_x_norm, tau=list(rep.tau), phi=rep.phi,
                kernel_ms=list(rep.kernel_ms), kernel_launches=list(rep.kernel_launches),
                refine_rounds=rep.refine_rounds)


def _stream_ptr(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """Device workspace for one map shape and precision (``wf_ctx``)."""

    def __init__(self, ny: int, nx: int, precision: str = "f32", device=None):
        import torch
        lib = load()
        self.ny, self.nx = int(ny), int(nx)
        self.dtype = {"f32": torch.float32, "f64": torch.float64}[precision]
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        shape = _Shape(self.ny, self.nx, 0 if precision == "f32" else 1)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.wf_ctx_create(ctypes.byref(shape), ctypes.byref(h))
        if st != 0:
            raise WFError(st, "wf_ctx_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().wf_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_profiling(self, on: bool):
        load().wf_ctx_set_profiling(self._h, 1 if on else 0)

    @property
    def tile(self) -> int:
        return load().wf_ctx_get_tile(self._h)

    def set_tile(self, tile: int) -> bool:
        """Select a transit-buffer tiling; False if it is not built for this
        context's size and precision."""
        st = load().wf_ctx_set_tile(self._h, int(tile))
        if st == -6:
            return False
        if st != 0:
            raise WFError(st, "wf_ctx_set_tile")
        return True

    def autotune(self, d, s_k, n_pix, p_oof=None, p_stripe=None, mask=None, *, sweeps=48):
        """``wf_autotune``: time a short solve of this map in every built
        tiling and keep the fastest.  Returns {tiling: ms per probe solve}."""
        import torch
        lib = load()
        ny, nx = self.ny, self.nx
        nh = nx // 2 + 1
        self._check(d, (ny, nx), "d")
        self._check(s_k, (ny, nh), "s_k")
        self._check(n_pix, (ny, nx), "n_pix")
        self._check(p_oof, (ny, nh), "p_oof")
        self._check(p_stripe, (ny,), "p_stripe")
        self._check(mask, (ny, nx), "mask", torch.uint8)
        scratch = torch.empty((ny, nx), dtype=self.dtype, device=self.device)
        n = lib.wf_tile_count()
        ms = (ctypes.c_double * n)()
        best = ctypes.c_int32()
        inp = _inputs(d, s_k, n_pix, p_oof, p_stripe, mask)
        with torch.cuda.device(self.device):
            st = lib.wf_autotune(self._h, ctypes.byref(inp), int(sweeps), scratch.data_ptr(), ms,
                                 ctypes.byref(best), _stream_ptr(torch, self.device))
        if st < 0:
            raise WFError(st, "wf_autotune")
        return {i: ms[i] for i in range(n) if ms[i] >= 0}

    def _check(self, t, shape, name, dtype=None):
        import torch
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if t.dtype != (dtype or self.dtype):
            raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype or self.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def solve(self, d, s_k, n_pix, p_oof=None, p_stripe=None, mask=None, *,
              schedule: Schedule = Schedule(), s_init=None, out=None):
        """Wiener filter of d.  Returns (s, report dict, trace array)."""
        import torch
        lib = load()
        ny, nx = self.ny, self.nx
        nh = nx // 2 + 1
        self._check(d, (ny, nx), "d")
        self._check(s_k, (ny, nh), "s_k")
        self._check(n_pix, (ny, nx), "n_pix")
        self._check(p_oof, (ny, nh), "p_oof")
        self._check(p_stripe, (ny,), "p_stripe")
        self._check(mask, (ny, nx), "mask", torch.uint8)
        self._check(s_init, (ny, nx), "s_init")
        if out is None:
            out = torch.empty((ny, nx), dtype=self.dtype, device=self.device)
        self._check(out, (ny, nx), "out")
        inp = _inputs(d, s_k, n_pix, p_oof, p_stripe, mask)
        return self._call(lib.wf_solve, "wf_solve", inp, schedule, s_init, out)

    def inverse_noise_weight(self, d, n_pix, p_oof=None, p_stripe=None, mask=None, *,
                             alpha: float, schedule: Schedule = Schedule(), s_init=None,
                             out=None):
        """Approximate N^-1 d as alpha^-1 S (S + N)^-1 d with S = alpha I
        (Section 4).  Returns (weighted map, report dict, trace array)."""
        import torch
        lib = load()
        ny, nx = self.ny, self.nx
        nh = nx // 2 + 1
        self._check(d, (ny, nx), "d")
        self._check(n_pix, (ny, nx), "n_pix")
        self._check(p_oof, (ny, nh), "p_oof")
        self._check(p_stripe, (ny,), "p_stripe")
        self._check(mask, (ny, nx), "mask", torch.uint8)
        self._check(s_init, (ny, nx), "s_init")
        if out is None:
            out = torch.empty((ny, nx), dtype=self.dtype, device=self.device)
        self._check(out, (ny, nx), "out")
        inp = _Inputs(d.data_ptr(), None, n_pix.data_ptr(),
                      p_oof.data_ptr() if p_oof is not None else None,
                      p_stripe.data_ptr() if p_stripe is not None else None,
                      mask.data_ptr() if mask is not None else None)

        def call(h, i, sch, si, o, rep, tr, st):
            return lib.wf_inverse_noise_weight(h, i, ctypes.c_double(alpha), sch, si, o, rep, tr, st)
        return self._call(call, "wf_inverse_noise_weight", inp, schedule, s_init, out)

    def _call(self, fn, what, inp, schedule, s_init, out):
        import torch
        sch, keep = schedule._c()
        nrec = -(-schedule.max_sweeps // schedule.monitor_every)
        trace = np.zeros((nrec, TRACE_COLS), dtype=np.float64)
        rep = _Report()
        with torch.cuda.device(self.device):
            st = fn(self._h, ctypes.byref(inp), ctypes.byref(sch),
                    s_init.data_ptr() if s_init is not None else None,
                    out.data_ptr(), ctypes.byref(rep),
                    trace.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    _stream_ptr(torch, self.device))
        del keep
        if st < 0:
            raise WFError(st, what)
        return out, _report(rep), trace[: rep.n_records]

    def rfft2(self, x):
        import torch
        self._check(x, (self.ny, self.nx), "x")
        cd = torch.complex64 if self.dtype == torch.float32 else torch.complex128
        X = torch.empty((self.ny, self.nx // 2 + 1), dtype=cd, device=self.device)
        with torch.cuda.device(self.device):
            st = load().wf_rfft2(self._h, x.data_ptr(), X.data_ptr(), _stream_ptr(torch, self.device))
        if st != 0:
            raise WFError(st, "wf_rfft2")
        return X

    def irfft2(self, X):
        import torch
        cd = torch.complex64 if self.dtype == torch.float32 else torch.complex128
        self._check(X, (self.ny, self.nx // 2 + 1), "X", cd)
        x = torch.empty((self.ny, self.nx), dtype=self.dtype, device=self.device)
        with torch.cuda.device(self.device):
            st = load().wf_irfft2(self._h, X.data_ptr(), x.data_ptr(), _stream_ptr(torch, self.device))
        if st != 0:
            raise WFError(st, "wf_irfft2")
        return x


def solve(d, s_k, n_pix, p_oof=None, p_stripe=None, mask=None, *, schedule=Schedule(),
          s_init=None):
    """One-shot solve: creates a context for d's shape and dtype."""
    import torch
    prec = "f64" if d.dtype == torch.float64 else "f32"
    ctx = Context(d.shape[0], d.shape[1], prec, device=d.device)
    try:
        return ctx.solve(d, s_k, n_pix, p_oof, p_stripe, mask, schedule=schedule, s_init=s_init)
    finally:
        ctx.close()


def solve_refined(ctx32, ctx64, d, s_k, n_pix, p_oof=None, p_stripe=None, mask=None, *,
                  first: Schedule, corr: Schedule, max_rounds: int = 4, rtol: float = 1e-6,
                  s_init=None, out=None):
    """``wf_solve_refined``: float32 solves on ``ctx32`` refined with float64
    residuals on ``ctx64`` (same shape).  Inputs are float64 tensors as for
    ``ctx64``; ``s_init`` (float64) warm-starts round 0 in ``first``'s field
    mode.  Returns (s float64, report dict, trace array of (round, sweeps so
    far, rho, rho_mask) after each round)."""
    import torch
    lib = load()
    if ctx32.dtype != torch.float32 or ctx64.dtype != torch.float64:
        raise ValueError("ctx32 must be float32 and ctx64 float64")
    ny, nx = ctx64.ny, ctx64.nx
    nh = nx // 2 + 1
    ctx64._check(d, (ny, nx), "d")
    ctx64._check(s_k, (ny, nh), "s_k")
    ctx64._check(n_pix, (ny, nx), "n_pix")
    ctx64._check(p_oof, (ny, nh), "p_oof")
    ctx64._check(p_stripe, (ny,), "p_stripe")
    ctx64._check(mask, (ny, nx), "mask", torch.uint8)
    ctx64._check(s_init, (ny, nx), "s_init")
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.float64, device=ctx64.device)
    ctx64._check(out, (ny, nx), "out")
    inp = _inputs(d, s_k, n_pix, p_oof, p_stripe, mask)
    s1, k1 = first._c()
    s2, k2 = corr._c()
    rep = _Report()
    trace = np.zeros((int(max_rounds) + 1, 4), dtype=np.float64)
    with torch.cuda.device(ctx64.device):
        st = lib.wf_solve_refined(ctx32._h, ctx64._h, ctypes.byref(inp), ctypes.byref(s1),
                                  ctypes.byref(s2), int(max_rounds), ctypes.c_double(rtol),
                                  None if s_init is None else ctypes.c_void_p(s_init.data_ptr()),
                                  out.data_ptr(), ctypes.byref(rep),
                                  trace.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  _stream_ptr(torch, ctx64.device))
    del k1, k2
    if st < 0:
        raise WFError(st, "wf_solve_refined")
    return out, _report(rep), trace[: rep.refine_rounds]


def solve_noalloc(d, s_k, n_pix, p_oof=None, p_stripe=None, mask=None, *,
                  schedule: Schedule = Schedule(), s_init=None, out=None):
    """``wf_solve_noalloc``: the solve without a context, its workspace in the
    library's static device scratch (no device allocation by the library).
    ``out`` may be given so that the call allocates nothing at all.  Returns
    (s, report dict, trace array); raises WFError on a negative status."""
    import torch
    lib = load()
    ny, nx = d.shape
    nh = nx // 2 + 1
    dt = d.dtype
    if dt not in (torch.float32, torch.float64) or not d.is_cuda:
        raise ValueError("d must be a float32 or float64 CUDA tensor")
    dev = d.device

    def chk(t, shape, name, dtype=dt):
        if t is None:
            return
        if (not isinstance(t, torch.Tensor) or t.device != dev or tuple(t.shape) != shape
                or t.dtype != dtype or not t.is_contiguous()):
            raise ValueError(f"{name}: expected a contiguous {dtype} tensor {shape} on {dev}")
    chk(d, (ny, nx), "d")
    chk(s_k, (ny, nh), "s_k")
    chk(n_pix, (ny, nx), "n_pix")
    chk(p_oof, (ny, nh), "p_oof")
    chk(p_stripe, (ny,), "p_stripe")
    chk(mask, (ny, nx), "mask", torch.uint8)
    chk(s_init, (ny, nx), "s_init")
    if out is None:
        out = torch.empty((ny, nx), dtype=dt, device=dev)
    chk(out, (ny, nx), "out")
    shape = _Shape(ny, nx, 0 if dt == torch.float32 else 1)
    inp = _inputs(d, s_k, n_pix, p_oof, p_stripe, mask)
    sch, keep = schedule._c()
    nrec = -(-schedule.max_sweeps // schedule.monitor_every)
    trace = np.zeros((nrec, TRACE_COLS), dtype=np.float64)
    rep = _Report()
    with torch.cuda.device(dev):
        st = lib.wf_solve_noalloc(ctypes.byref(shape), ctypes.byref(inp), ctypes.byref(sch),
                                  s_init.data_ptr() if s_init is not None else None,
                                  out.data_ptr(), ctypes.byref(rep),
                                  trace.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  _stream_ptr(torch, dev))
    del keep
    if st < 0:
        raise WFError(st, "wf_solve_noalloc")
    return out, _report(rep), trace[: rep.n_records]


def solve_batch(contexts, problems, *, schedule: Schedule = Schedule(), outs=None,
                s_inits=None):
    """Solve many maps at once (``wf_solve_batch``).  contexts: one distinct
    ``Context`` per map (same precision and device); problems: per map a dict
    with keys d, s_k, n_pix and optionally p_oof, p_stripe, mask (device
    tensors checked like ``Context.solve``).  Returns (list of maps, list of
    report dicts).  Maps of one shape share their kernel launches; one chunk
    of sweeps is replayed as a HIP graph.  s_inits: optional per-map warm
    starts (device tensors of each map's shape, or None entries)."""
    import torch
    lib = load()
    n = len(contexts)
    inps, handles, optrs, iptrs, res = _batch_args(contexts, problems, outs, s_inits)
    sch, keep = schedule._c()
    reps = (_Report * n)()
    dev = contexts[0].device
    with torch.cuda.device(dev):
        st = lib.wf_solve_batch(handles, n, inps, ctypes.byref(sch),
                                iptrs if s_inits is not None else None, optrs, reps,
                                _stream_ptr(torch, dev))
    del keep
    if st < 0:
        raise WFError(st, "wf_solve_batch")
    return res, [_report(r) for r in reps]


def autotune_batch(contexts, problems, *, outs=None, sweeps=48):
    """``wf_autotune_batch``: for each shape among the maps, time short
    batched solves of the maps of that shape in every built tiling and keep
    the fastest on their contexts.  Arguments as for ``solve_batch`` (outs,
    if given, are overwritten by the probes).  Returns {(ny, nx): (chosen
    tiling, {tiling: ms per probe solve})}."""
    import torch
    lib = load()
    n = len(contexts)
    inps, handles, optrs, _, probe_outs = _batch_args(contexts, problems, outs, None)
    nt = lib.wf_tile_count()
    ms = (ctypes.c_double * (n * nt))()
    best = (ctypes.c_int32 * n)()
    dev = contexts[0].device
    with torch.cuda.device(dev):
        st = lib.wf_autotune_batch(handles, n, inps, int(sweeps), optrs, ms, best,
                                   _stream_ptr(torch, dev))
    if st < 0:
        raise WFError(st, "wf_autotune_batch")
    out = {}
    for i, ctx in enumerate(contexts):
        out.setdefault((ctx.ny, ctx.nx), (best[i], {t: ms[i * nt + t] for t in range(nt)
                                                   if ms[i * nt + t] >= 0}))
    return out


def _batch_args(contexts, problems, outs, s_inits):
    """ctypes arrays of a batch call: per-map inputs, context handles, output
    and warm-start pointers (outputs allocated where outs has None)."""
    import torch
    n = len(contexts)
    if n != len(problems) or n < 1:
        raise ValueError("need one problem per context")
    if outs is None:
        outs = [None] * n
    inps = (_Inputs * n)()
    handles = (ctypes.c_void_p * n)()
    optrs = (ctypes.c_void_p * n)()
    iptrs = (ctypes.c_void_p * n)()
    res = []
    for i, (ctx, pb) in enumerate(zip(contexts, problems)):
        ny, nx = ctx.ny, ctx.nx
        nh = nx // 2 + 1
        ctx._check(pb["d"], (ny, nx), "d")
        ctx._check(pb["s_k"], (ny, nh), "s_k")
        ctx._check(pb["n_pix"], (ny, nx), "n_pix")
        ctx._check(pb.get("p_oof"), (ny, nh), "p_oof")
        ctx._check(pb.get("p_stripe"), (ny,), "p_stripe")
        ctx._check(pb.get("mask"), (ny, nx), "mask", torch.uint8)
        o = outs[i]
        if o is None:
            o = torch.empty((ny, nx), dtype=ctx.dtype, device=ctx.device)
        ctx._check(o, (ny, nx), "out")
        res.append(o)
        inps[i] = _inputs(pb["d"], pb["s_k"], pb["n_pix"], pb.get("p_oof"),
                          pb.get("p_stripe"), pb.get("mask"))
        handles[i] = ctx._h
        optrs[i] = o.data_ptr()
        si = None if s_inits is None else s_inits[i]
        if si is not None:
            ctx._check(si, (ny, nx), "s_init")
            iptrs[i] = si.data_ptr()
    return inps, handles, optrs, iptrs, res


def rfft2(x):
    import torch
    ctx = Context(x.shape[0], x.shape[1], "f64" if x.dtype == torch.float64 else "f32",
                  device=x.device)
    try:
        return ctx.rfft2(x)
    finally:
        ctx.close()


def irfft2(X, nx: int):
    import torch
    ctx = Context(X.shape[0], nx, "f64" if X.dtype == torch.complex128 else "f32",
                  device=X.device)
    try:
        return ctx.irfft2(X)
    finally:
        ctx.close()
