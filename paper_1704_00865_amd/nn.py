"""ctypes binding of the warm-start network (include/wf_nn.h).

Argument marshalling only: features, convolutions, the loss, back-propagation
and Adam all run in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes
from typing import List, Tuple

import numpy as np

from . import WFError, _stream_ptr, load

CHANNELS = (32, 64, 96, 128)
PAD = 32


class _NNShape(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int32), ("w", ctypes.c_int32), ("batch_max", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


EXPORTS = ("wf_nn_param_count", "wf_nn_create", "wf_nn_destroy", "wf_nn_set_params",
           "wf_nn_get_params", "wf_nn_predict", "wf_nn_train_step", "wf_nn_forward_features",
           "wf_nn_gradient_features", "wf_nn_conv3x3")

_bound = False


def _lib():
    global _bound
    lib = load()
    if not _bound:
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        dp = ctypes.POINTER(ctypes.c_double)
        lib.wf_nn_param_count.argtypes = []
        lib.wf_nn_param_count.restype = ctypes.c_int64
        lib.wf_nn_create.argtypes = [ctypes.POINTER(_NNShape), ctypes.POINTER(vp)]
        lib.wf_nn_create.restype = i32
        lib.wf_nn_destroy.argtypes = [vp]
        lib.wf_nn_destroy.restype = None
        lib.wf_nn_set_params.argtypes = [vp, vp, vp]
        lib.wf_nn_set_params.restype = i32
        lib.wf_nn_get_params.argtypes = [vp, vp, vp]
        lib.wf_nn_get_params.restype = i32
        lib.wf_nn_predict.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        lib.wf_nn_predict.restype = i32
        lib.wf_nn_train_step.argtypes = [vp, i32, vp, vp, vp, vp, ctypes.c_float, dp, vp]
        lib.wf_nn_train_step.restype = i32
        lib.wf_nn_forward_features.argtypes = [vp, i32, vp, vp, vp]
        lib.wf_nn_forward_features.restype = i32
        lib.wf_nn_gradient_features.argtypes = [vp, i32, vp, vp, vp, dp, vp]
        lib.wf_nn_gradient_features.restype = i32
        lib.wf_nn_conv3x3.argtypes = [i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]
        lib.wf_nn_conv3x3.restype = i32
        _bound = True
    return lib


def layer_shapes() -> List[Tuple[int, int]]:
    """(ci, co) of every convolution in network order, padded as stored."""
    c = CHANNELS
    s = [(PAD, c[0]), (c[0], c[0])]
    for l in range(1, len(c)):
        s += [(c[l - 1], c[l]), (c[l], c[l])]
    for l in range(len(c) - 2, -1, -1):
        s += [(c[l + 1], c[l]), (c[l], c[l])]
    s.append((c[0], PAD))
    return s


def layer_offsets() -> List[Tuple[int, int, int, int]]:
    """(ci, co, weight offset, bias offset) of every convolution."""
    out, off = [], 0
    for ci, co in layer_shapes():
        w_off = off
        off += 9 * ci * co
        out.append((ci, co, w_off, off))
        off += co
    return out


def param_count() -> int:
    return int(_lib().wf_nn_param_count())


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / (9 ci)) over the real input channels),
    zero biases, zero padded entries and a zero output layer, so that an
    untrained network predicts 0 (the zero start)."""
    rng = np.random.default_rng(seed)
    offs = layer_offsets()
    p = np.zeros(offs[-1][3] + offs[-1][1], dtype=np.float32)
    for i, (ci, co, wo, _) in enumerate(offs):
        if i == len(offs) - 1:
            continue
        ci_real = 4 if i == 0 else ci
        w = np.zeros((3, 3, ci, co))
        w[:, :, :ci_real, :] = rng.standard_normal((3, 3, ci_real, co)) * np.sqrt(2.0 / (9 * ci_real))
        p[wo:wo + w.size] = w.ravel()
    return p


class WarmNet:
    """Network workspace for maps of one size (``wf_nn_create``)."""

    def __init__(self, h: int, w: int, batch_max: int = 1, precision: str = "f32", device=None):
        import torch
        lib = _lib()
        self.h, self.w, self.batch_max = int(h), int(w), int(batch_max)
        self.dtype = {"f32": torch.float32, "f64": torch.float64}[precision]
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        sh = _NNShape(self.h, self.w, self.batch_max, 0 if precision == "f32" else 1)
        hnd = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.wf_nn_create(ctypes.byref(sh), ctypes.byref(hnd))
        if st != 0:
            raise WFError(st, "wf_nn_create")
        self._h = hnd
        self.nparam = param_count()

    def close(self):
        if getattr(self, "_h", None):
            _lib().wf_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _st(self):
        import torch
        return _stream_ptr(torch, self.device)

    def _call(self, name, *args):
        import torch
        with torch.cuda.device(self.device):
            st = getattr(_lib(), name)(self._h, *args)
        if st != 0:
            raise WFError(st, name)

    def set_params(self, params):
        import torch
        t = torch.as_tensor(np.asarray(params, dtype=np.float32) if not isinstance(params, torch.Tensor)
                            else params, dtype=torch.float32).to(self.device).contiguous()
        if t.numel() != self.nparam:
            raise ValueError(f"expected {self.nparam} parameters")
        self._call("wf_nn_set_params", t.data_ptr(), self._st())

    def get_params(self):
        import torch
        t = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        self._call("wf_nn_get_params", t.data_ptr(), self._st())
        return t

    def _maps(self, d, n_pix, mask):
        import torch
        n = d.shape[0]
        if n < 1 or n > self.batch_max:
            raise ValueError(f"batch of {n} maps; the workspace holds {self.batch_max}")
        for name, t in (("d", d), ("n_pix", n_pix)):
            if t.shape != (n, self.h, self.w) or t.dtype != self.dtype or t.device != self.device \
                    or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {self.dtype} [n, {self.h}, {self.w}] "
                                 f"tensor on {self.device}")
        if mask is not None and (mask.shape != (n, self.h, self.w) or mask.dtype != torch.uint8
                                 or not mask.is_contiguous()):
            raise ValueError("mask must be a contiguous uint8 [n, h, w] tensor")
        return n

    def predict(self, d, n_pix, mask=None, out=None):
        """Predicted Wiener solutions [n, h, w] of a batch of maps."""
        import torch
        n = self._maps(d, n_pix, mask)
        if out is None:
            out = torch.empty_like(d)
        self._call("wf_nn_predict", n, d.data_ptr(), n_pix.data_ptr(),
                   mask.data_ptr() if mask is not None else None, out.data_ptr(), self._st())
        return out

    def train_step(self, d, n_pix, mask, s_target, lr: float) -> float:
        """One Adam step on a batch; returns the loss before the step."""
        n = self._maps(d, n_pix, mask)
        if s_target.shape != d.shape or s_target.dtype != self.dtype:
            raise ValueError("s_target must match d")
        loss = ctypes.c_double()
        self._call("wf_nn_train_step", n, d.data_ptr(), n_pix.data_ptr(),
                   mask.data_ptr() if mask is not None else None, s_target.data_ptr(),
                   ctypes.c_float(lr), ctypes.byref(loss), self._st())
        return loss.value

    def forward_features(self, x):
        import torch
        n = x.shape[0]
        if x.shape != (n, self.h, self.w, 4) or x.dtype != torch.float32:
            raise ValueError("x must be float32 [n, h, w, 4]")
        y = torch.empty((n, self.h, self.w), dtype=torch.float32, device=self.device)
        self._call("wf_nn_forward_features", n, x.contiguous().data_ptr(), y.data_ptr(), self._st())
        return y

    def gradient_features(self, x, target):
        import torch
        n = x.shape[0]
        g = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        self._call("wf_nn_gradient_features", n, x.contiguous().data_ptr(),
                   target.contiguous().data_ptr(), g.data_ptr(), ctypes.byref(loss), self._st())
        return g, loss.value


def conv3x3(mode: int, x, w=None, b=None, g=None, *, ci: int, co: int):
    """One convolution building block (``wf_nn_conv3x3``) on bfloat16
    tensors [n, h, w, c] (torch.bfloat16).  Returns bfloat16 [n, h, w, c_out]
    for modes 0-2 and float32 [3, 3, ci, co] for mode 3."""
    import torch
    n, h, wd, c = x.shape
    if mode == 3:
        out = torch.empty((3, 3, ci, co), dtype=torch.float32, device=x.device)
    else:
        out = torch.empty((n, h, wd, ci if mode == 2 else co), dtype=torch.bfloat16, device=x.device)
    with torch.cuda.device(x.device):
        st = _lib().wf_nn_conv3x3(mode, n, h, wd, ci, co, x.data_ptr(),
                                  w.data_ptr() if w is not None else None,
                                  b.data_ptr() if b is not None else None,
                                  g.data_ptr() if g is not None else None, out.data_ptr(),
                                  _stream_ptr(torch, x.device))
    if st != 0:
        raise WFError(st, "wf_nn_conv3x3")
    return out
