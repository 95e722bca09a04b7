"""Convolutional warm-start predictor, plain float64 NumPy (test infrastructure).

The messenger iteration may start from any field (Section 2 notes that the
start does not change the solution); this module is the reference for a small network that
predicts the Wiener solution from the data so that the iteration can start
from the prediction.  The network is not from the paper.  Everything here is
written for readability: circular 3x3 convolutions as sums of shifted copies,
explicit reverse-mode differentiation, and the Adam update by its formula.

Layout: activations are [N, H, W, C] (channels last); a 3x3 kernel is
W[dy + 1, dx + 1, ci, co] and the convolution is a cross-correlation on the
torus (the maps are periodic):
    out[n, y, x, co] = b[co] + sum_{dy, dx, ci} in[n, (y+dy) % H, (x+dx) % W, ci]
                                               * W[dy+1, dx+1, ci, co].

Architecture (levels l = 0..L-1 with channels C_l, resolution halved per
level by 2x2 averaging, nearest-neighbour upsampling back up):
    e_0 = R(conv(R(conv(x))))                                  at full size
    e_l = R(conv(R(conv(pool(e_{l-1})))))                      l = 1..L-1
    u_{L-1} = e_{L-1}
    b_l = R(conv(up(u_{l+1}))), u_l = R(conv(b_l + e_l))       l = L-2..0
    y   = conv(u_0)                                            one channel
with R = max(0, .).  Inputs are four channels built from (d, N_pix, mask):
d / sigma, log(N_pix / sigma^2) on observed pixels (0 on masked ones), the
mask, and the mean of d / sigma over the observed pixels of the pixel's row
(row-constant stripe noise is visible only over a whole row, wider than the
network's receptive field), where sigma^2 is the mean white variance over
observed pixels; the target is the field to predict divided by sigma.

Pinned (tests, ``not gpu``) by: brute-force loops for the convolution, the
adjoint identities <A x, y> = <x, A^T y> for convolution, pooling and
upsampling, translation equivariance on the torus, and central finite
differences of the loss for every parameter group.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


# --------------------------------------------------------------------------
# single operations and their adjoints
# --------------------------------------------------------------------------

def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """Circular 3x3 cross-correlation: x [N,H,W,Ci], w [3,3,Ci,Co], b [Co]."""
    n, h, wd, ci = x.shape
    co = w.shape[3]
    out = np.zeros((n, h, wd, co))
    for dy, dx in TAPS:
        shifted = np.roll(x, shift=(-dy, -dx), axis=(1, 2))  # shifted[y] = x[y + dy]
        out += shifted @ w[dy + 1, dx + 1]
    if b is not None:
        out += b
    return out


def conv3x3_grad_input(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of conv3x3 in its input: sum over taps of W^T g shifted back."""
    gi = np.zeros(g.shape[:3] + (w.shape[2],))
    for dy, dx in TAPS:
        part = g @ w[dy + 1, dx + 1].T
        gi += np.roll(part, shift=(dy, dx), axis=(1, 2))
    return gi


def conv3x3_grad_weight(x: np.ndarray, g: np.ndarray) -> np.ndarray:
    """dL/dW[dy+1, dx+1] = sum over pixels of x[p + (dy, dx)]^T g[p]."""
    ci, co = x.shape[3], g.shape[3]
    gw = np.zeros((3, 3, ci, co))
    gf = g.reshape(-1, co)
    for dy, dx in TAPS:
        shifted = np.roll(x, shift=(-dy, -dx), axis=(1, 2)).reshape(-1, ci)
        gw[dy + 1, dx + 1] = shifted.T @ gf
    return gw


def relu(x):
    return np.maximum(x, 0.0)


def pool2(x: np.ndarray) -> np.ndarray:
    """2x2 average over non-overlapping blocks."""
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def pool2_adjoint(g: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def up2(x: np.ndarray) -> np.ndarray:
    """Nearest-neighbour upsampling by 2 in both directions."""
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_adjoint(g: np.ndarray) -> np.ndarray:
    n, h, w, c = g.shape
    return g.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


# --------------------------------------------------------------------------
# the network
# --------------------------------------------------------------------------

@dataclass
class Params:
    """Weights and biases of every convolution in network order (see
    ``layer_shapes``)."""
    w: List[np.ndarray]
    b: List[np.ndarray]

    def copy(self) -> "Params":
        return Params([x.copy() for x in self.w], [x.copy() for x in self.b])


def layer_shapes(channels: Sequence[int], c_in: int = 4) -> List[tuple]:
    """(Ci, Co) of each convolution: two per encoder level, two per decoder
    level, then the single-channel output convolution."""
    L = len(channels)
    shapes = [(c_in, channels[0]), (channels[0], channels[0])]
    for l in range(1, L):
        shapes += [(channels[l - 1], channels[l]), (channels[l], channels[l])]
    for l in range(L - 2, -1, -1):
        shapes += [(channels[l + 1], channels[l]), (channels[l], channels[l])]
    shapes.append((channels[0], 1))
    return shapes


def init_params(channels: Sequence[int], seed: int, c_in: int = 4) -> Params:
    """He-normal weights (std sqrt(2 / (9 Ci))), zero biases; the output
    convolution starts at zero so the first prediction is 0 (the zero start)."""
    rng = np.random.default_rng(seed)
    ws, bs = [], []
    shapes = layer_shapes(channels, c_in)
    for i, (ci, co) in enumerate(shapes):
        std = 0.0 if i == len(shapes) - 1 else np.sqrt(2.0 / (9 * ci))
        ws.append(rng.standard_normal((3, 3, ci, co)) * std)
        bs.append(np.zeros(co))
    return Params(ws, bs)


@dataclass
class Tape:
    """Activations kept for the backward pass."""
    x: np.ndarray
    enc: List[tuple] = field(default_factory=list)   # (input, h, e) per level
    dec: List[tuple] = field(default_factory=list)   # (a, b, c, u) per level
    u0: np.ndarray | None = None
    y: np.ndarray | None = None


def forward(p: Params, x: np.ndarray, channels: Sequence[int]) -> Tape:
    L = len(channels)
    tp = Tape(x=x)
    k = 0
    inp = x
    for l in range(L):
        if l > 0:
            inp = pool2(tp.enc[l - 1][2])
        h = relu(conv3x3(inp, p.w[k], p.b[k]))
        e = relu(conv3x3(h, p.w[k + 1], p.b[k + 1]))
        tp.enc.append((inp, h, e))
        k += 2
    u = tp.enc[L - 1][2]
    for l in range(L - 2, -1, -1):
        a = up2(u)
        b = relu(conv3x3(a, p.w[k], p.b[k]))
        c = b + tp.enc[l][2]
        u = relu(conv3x3(c, p.w[k + 1], p.b[k + 1]))
        tp.dec.append((a, b, c, u))
        k += 2
    tp.u0 = u
    tp.y = conv3x3(u, p.w[k], p.b[k])[..., 0]
    return tp


def loss(y: np.ndarray, target: np.ndarray) -> float:
    """Mean squared error over every pixel of every map."""
    return float(np.mean((y - target) ** 2))


def backward(p: Params, tp: Tape, target: np.ndarray, channels: Sequence[int]) -> Params:
    """Gradient of ``loss`` with respect to every weight and bias."""
    L = len(channels)
    nl = len(p.w)
    gw: List[np.ndarray] = [None] * nl
    gb: List[np.ndarray] = [None] * nl
    gy = (2.0 / tp.y.size) * (tp.y - target)[..., None]
    k = nl - 1
    gw[k] = conv3x3_grad_weight(tp.u0, gy)
    gb[k] = gy.sum(axis=(0, 1, 2))
    gu = conv3x3_grad_input(gy, p.w[k])
    g_enc = [np.zeros_like(tp.enc[l][2]) for l in range(L)]
    k -= 1
    for j, l in enumerate(range(0, L - 1)):
        # decoder levels in reverse order of their construction
        a, b, c, u = tp.dec[L - 2 - l]
        gpre = gu * (u > 0)
        gw[k] = conv3x3_grad_weight(c, gpre)
        gb[k] = gpre.sum(axis=(0, 1, 2))
        gc = conv3x3_grad_input(gpre, p.w[k])
        g_enc[l] += gc
        gpre = gc * (b > 0)
        gw[k - 1] = conv3x3_grad_weight(a, gpre)
        gb[k - 1] = gpre.sum(axis=(0, 1, 2))
        gu = up2_adjoint(conv3x3_grad_input(gpre, p.w[k - 1]))
        k -= 2
    g_enc[L - 1] += gu
    for l in range(L - 1, -1, -1):
        inp, h, e = tp.enc[l]
        kk = 2 * l
        gpre = g_enc[l] * (e > 0)
        gw[kk + 1] = conv3x3_grad_weight(h, gpre)
        gb[kk + 1] = gpre.sum(axis=(0, 1, 2))
        gh = conv3x3_grad_input(gpre, p.w[kk + 1]) * (h > 0)
        gw[kk] = conv3x3_grad_weight(inp, gh)
        gb[kk] = gh.sum(axis=(0, 1, 2))
        if l > 0:
            g_enc[l - 1] += pool2_adjoint(conv3x3_grad_input(gh, p.w[kk]))
    return Params(gw, gb)


# --------------------------------------------------------------------------
# inputs, targets and the optimiser
# --------------------------------------------------------------------------

def features(d: np.ndarray, n_pix: np.ndarray, mask: np.ndarray | None):
    """Network inputs [H, W, 4] and the scale sigma (see the module notes)."""
    d = np.asarray(d, dtype=np.float64)
    npix = np.asarray(n_pix, dtype=np.float64)
    obs = np.ones(d.shape, dtype=bool) if mask is None else np.asarray(mask) != 0
    sig2 = float(npix[obs].mean())
    sig = np.sqrt(sig2)
    f = np.zeros(d.shape + (4,))
    f[..., 0] = np.where(obs, d / sig, 0.0)
    f[..., 1] = np.where(obs, np.log(np.where(obs, npix, 1.0) / sig2), 0.0)
    f[..., 2] = obs.astype(np.float64)
    cnt = obs.sum(axis=1)
    rows = np.where(cnt > 0, f[..., 0].sum(axis=1) / np.maximum(cnt, 1), 0.0)
    f[..., 3] = rows[:, None]
    return f, sig


@dataclass
class Adam:
    """Adam (Kingma & Ba 2015) with bias correction:
    m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""
    lr: float = 1e-3
    b1: float = 0.9
    b2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: list = field(default_factory=list)
    v: list = field(default_factory=list)

    def step(self, p: Params, g: Params) -> Params:
        flat_p = p.w + p.b
        flat_g = g.w + g.b
        if not self.m:
            self.m = [np.zeros_like(x) for x in flat_p]
            self.v = [np.zeros_like(x) for x in flat_p]
        self.t += 1
        out = []
        for i, (x, gr) in enumerate(zip(flat_p, flat_g)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * gr
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * gr * gr
            mh = self.m[i] / (1 - self.b1 ** self.t)
            vh = self.v[i] / (1 - self.b2 ** self.t)
            out.append(x - self.lr * mh / (np.sqrt(vh) + self.eps))
        n = len(p.w)
        return Params(out[:n], out[n:])
