"""Flat-sky stand-ins for the paper's dense-noise test problem.

The paper's third test (Section 3.3) filters a CMB temperature map whose noise
is the sum of a harmonic-diagonal part with extra power in the m=0 modes
(horizontal stripes), a pixel-diagonal part whose variance rises near the mask
edge, and a sky mask.  Its spectra, HEALPix maps and mask are not available
here, so this module draws periodic flat-sky maps of the same structure:

* signal: Gaussian random field with C(l) = A l^-2 exp(-(l/1500)^2);
* 1/f noise: isotropic, P(l) = L^2 (1 + (1000/l)^3)  (L in uK-arcmin);
* stripe noise: one value per row, P_st(k_y) = A_st (1 + (l_y0/l_y)^2);
* white noise: sigma_p = sigma_0 exp(z/2) with z a smoothed unit Gaussian;
* mask: random periodic discs of radius 5-20 px covering a target fraction.

Conventions (shared by every consumer of these arrays):

* maps are (ny, nx) row-major, x fastest, periodic, square pixels of
  ``pix_arcmin`` arcminutes (solid angle Omega_pix);
* Fourier-diagonal covariances are given on the numpy ``rfft2`` half
  spectrum, shape (ny, nx//2+1), as the variance of each *unitary* DFT mode in
  pixel-variance units (uK^2): a spectrum C(l) [uK^2 sr] maps to C(l)/Omega_pix,
  so white noise of variance sigma^2 has the flat value sigma^2 (Section 3.1
  states the same correspondence N = (sigma^2/Omega_pix) I <-> N_l = sigma^2);
* the stripe covariance is given per unitary 1-D mode of the row value f(y),
  shape (ny,), numpy ``fftfreq`` order; the stripe map is n(x, y) = f(y);
* mask is uint8, 1 = observed, 0 = masked (infinite noise variance).

Every array handed to a solver is rounded to float32 and promoted back to
float64, so a float32 GPU path and the float64 oracle solve bit-identical
problems.

Random draws come from ``numpy.random.default_rng(seed)`` in a fixed order
(signal, 1/f, stripes, z, white, mask), all of them drawn whether or not a term
is used, so a seed always yields the same signal realisation.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

ARCMIN = np.pi / (180.0 * 60.0)
SIGNAL_AMP = 2.0 * np.pi * 2500.0  # uK^2: l^2 C_l / 2pi ~ 2500 uK^2 at low l
SIGNAL_LDAMP = 1500.0
OOF_KNEE = 1000.0
STRIPE_KNEE = 1000.0


def pixel_size_rad(pix_arcmin: float = 2.0) -> float:
    return pix_arcmin * ARCMIN


def l_of_modes(ny: int, nx: int, dpix: float) -> np.ndarray:
    """Multipole l = |2 pi k / (n dpix)| of every rfft2 mode, floored at the
    fundamental l so that red spectra stay finite at k = 0."""
    ly = 2.0 * np.pi * np.fft.fftfreq(ny, d=dpix)
    lx = 2.0 * np.pi * np.fft.rfftfreq(nx, d=dpix)
    ell = np.hypot(ly[:, None], lx[None, :])
    lfund = 2.0 * np.pi / (max(ny, nx) * dpix)
    return np.maximum(ell, lfund)


def _ly_of_rows(ny: int, dpix: float) -> np.ndarray:
    ly = np.abs(2.0 * np.pi * np.fft.fftfreq(ny, d=dpix))
    return np.maximum(ly, 2.0 * np.pi / (ny * dpix))


def _f32(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _grf(w: np.ndarray, var_modes: np.ndarray) -> np.ndarray:
    """Real Gaussian field whose unitary rfft2 modes have variance var_modes."""
    ny, nx = w.shape
    wk = np.fft.rfft2(w, norm="ortho")
    return np.fft.irfft2(np.sqrt(var_modes) * wk, s=(ny, nx), norm="ortho")


def _smooth_unit(w: np.ndarray, sigma_px: float) -> np.ndarray:
    ny, nx = w.shape
    fy = np.fft.fftfreq(ny)[:, None]
    fx = np.fft.rfftfreq(nx)[None, :]
    kern = np.exp(-2.0 * np.pi**2 * sigma_px**2 * (fx**2 + fy**2))
    z = np.fft.irfft2(np.fft.rfft2(w) * kern, s=(ny, nx))
    z -= z.mean()
    return z / z.std()


def _disc_mask(rng: np.random.Generator, ny: int, nx: int, frac: float,
               rmin: int = 5, rmax: int = 20) -> np.ndarray:
    """1 = observed.  Periodic discs with integer radii in [rmin, rmax] are
    added until at least ``frac`` of the pixels are masked."""
    mask = np.ones((ny, nx), dtype=np.uint8)
    if frac <= 0.0:
        return mask
    yy = np.arange(ny)[:, None]
    xx = np.arange(nx)[None, :]
    target = frac * ny * nx
    while (mask == 0).sum() < target:
        cy = int(rng.integers(ny))
        cx = int(rng.integers(nx))
        r = int(rng.integers(rmin, rmax + 1))
        dy = np.minimum((yy - cy) % ny, (cy - yy) % ny)
        dx = np.minimum((xx - cx) % nx, (cx - xx) % nx)
        mask[(dy * dy + dx * dx) <= r * r] = 0
    return mask


@dataclass
class Problem:
    """One Wiener-filter problem d = s + n with N = N_1/f + N_stripe + N_pix."""

    d: np.ndarray                    # (ny, nx) data, uK
    s_k: np.ndarray                  # (ny, nx//2+1) signal mode variance, uK^2
    n_pix: np.ndarray                # (ny, nx) white pixel variance, uK^2
    p_oof: Optional[np.ndarray]      # (ny, nx//2+1) 1/f mode variance or None
    p_stripe: Optional[np.ndarray]   # (ny,) stripe 1-D mode variance or None
    mask: Optional[np.ndarray]       # (ny, nx) uint8, 1 observed, or None
    s_true: np.ndarray               # (ny, nx) the signal realisation
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.d.shape


def make_problem(ny: int, nx: int, seed: int, *,
                 pix_arcmin: float = 2.0,
                 oof_level: Optional[float] = 10.0,
                 stripe_rms: Optional[float] = 10.0,
                 white_sigma: float = 10.0,
                 white_contrast: float = 0.5,
                 smooth_px: float = 8.0,
                 mask_frac: float = 0.0,
                 signal_amp: float = SIGNAL_AMP) -> Problem:
    """Draw one problem.

    oof_level   : 1/f white floor L in uK-arcmin (None drops the term)
    stripe_rms  : rms of the per-row stripe value in uK (None drops the term)
    white_sigma : sigma_0 in uK per pixel; sigma_p = sigma_0 exp(c z)
    white_contrast : c above (0.5 gives the exp(z/2) law)
    mask_frac   : target masked fraction (0 = no mask)
    """
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((ny, nx))
    w2 = rng.standard_normal((ny, nx))
    w3 = rng.standard_normal(ny)
    w4 = rng.standard_normal((ny, nx))
    w5 = rng.standard_normal((ny, nx))

    dpix = pixel_size_rad(pix_arcmin)
    omega = dpix * dpix
    ell = l_of_modes(ny, nx, dpix)

    s_k = signal_amp * ell**-2.0 * np.exp(-(ell / SIGNAL_LDAMP) ** 2) / omega
    s_k = _f32(s_k)
    s_true = _grf(w1, s_k)

    p_oof = None
    n_oof = np.zeros((ny, nx))
    if oof_level is not None:
        floor = (oof_level * ARCMIN) ** 2 / omega  # uK^2 per unitary mode
        p_oof = _f32(floor * (1.0 + (OOF_KNEE / ell) ** 3))
        n_oof = _grf(w2, p_oof)

    p_stripe = None
    n_st = np.zeros((ny, nx))
    if stripe_rms is not None:
        ly = _ly_of_rows(ny, dpix)
        shape = 1.0 + (STRIPE_KNEE / ly) ** 2
        a_st = stripe_rms**2 * ny / shape.sum()  # (1/ny) sum P_st = rms^2
        p_stripe = _f32(a_st * shape)
        f = np.fft.ifft(np.sqrt(p_stripe) * np.fft.fft(w3, norm="ortho"),
                        norm="ortho").real
        n_st = np.broadcast_to(f[:, None], (ny, nx)).copy()

    z = _smooth_unit(w4, smooth_px)
    sig_p = white_sigma * np.exp(white_contrast * z)
    n_pix = _f32(sig_p**2)
    n_w = np.sqrt(n_pix) * w5

    mask = None
    if mask_frac > 0.0:
        mask = _disc_mask(rng, ny, nx, mask_frac)

    d = _f32(s_true + n_oof + n_st + n_w)
    meta = dict(seed=seed, pix_arcmin=pix_arcmin, oof_level=oof_level,
                stripe_rms=stripe_rms, white_sigma=white_sigma,
                smooth_px=smooth_px, mask_frac=mask_frac,
                masked_frac=0.0 if mask is None else float((mask == 0).mean()))
    return Problem(d=d, s_k=s_k, n_pix=n_pix, p_oof=p_oof, p_stripe=p_stripe,
                   mask=mask, s_true=s_true, meta=meta)


def make_stationary_problem(ny: int, nx: int, seed: int, sigma: float = 10.0,
                            **kw) -> Problem:
    """Three-term problem with uniform white variance sigma^2 and no mask, so
    the whole noise covariance is diagonal in the 2-D Fourier basis."""
    kw = dict(kw)
    kw.update(white_contrast=0.0, white_sigma=sigma, mask_frac=0.0)
    return make_problem(ny, nx, seed, **kw)


def named_config(name: str) -> Problem:
    """The workloads the library is tested and measured on.

    c1      64x64, three terms, no mask, seed 1
    c2      512x512, three terms, no mask, seed 2
    c3      2048x2048, three terms, 10% disc mask, seed 3
    c3_small 256x256 version of c3 (same recipe, seed 3)
    """
    if name == "c1":
        return make_problem(64, 64, 1)
    if name == "c2":
        return make_problem(512, 512, 2)
    if name == "c3":
        return make_problem(2048, 2048, 3, mask_frac=0.10)
    if name == "c3_small":
        return make_problem(256, 256, 3, mask_frac=0.10)
    raise KeyError(name)


def uneven_batch(sizes=(256, 768, 1536), per_size: int = 16, base_seed: int = 4000):
    """Batch of independent maps of uneven size (default 16 each of 256^2,
    768^2 and 1536^2, 48 maps, 48.2 M pixels).  Map i (in order of the sizes)
    uses seed base_seed + i and a noise level L_i drawn uniformly in
    [5, 30] uK-arcmin from its own generator: the 1/f floor is L_i and the
    white level is L_i per 2' pixel (sigma_0 = L_i / 2 uK).  No mask."""
    out = []
    i = 0
    for n in sizes:
        for _ in range(per_size):
            seed = base_seed + i
            lvl = float(np.random.default_rng([seed, 77]).uniform(5.0, 30.0))
            out.append(make_problem(n, n, seed, oof_level=lvl, white_sigma=lvl / 2.0))
            i += 1
    return out


def _compact_problem(args):
    ny, nx, seed, kw = args
    p = make_problem(ny, nx, seed, **kw)
    f32 = np.float32
    return Problem(d=p.d.astype(f32), s_k=p.s_k.astype(f32), n_pix=p.n_pix.astype(f32),
                   p_oof=None if p.p_oof is None else p.p_oof.astype(f32),
                   p_stripe=None if p.p_stripe is None else p.p_stripe.astype(f32),
                   mask=p.mask, s_true=None, meta=p.meta)


def make_problems(ny: int, nx: int, seeds, *, workers: int = 1, **kw):
    """make_problem for many seeds, in ``workers`` forked processes when
    workers > 1 (call it before the process uses a GPU).  The arrays come back
    as float32 (exact: every solver input is float32-representable) and
    without the signal realisation, to keep large sets small."""
    jobs = [(ny, nx, int(s), kw) for s in seeds]
    if workers <= 1:
        return [_compact_problem(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_compact_problem, jobs, chunksize=max(1, len(jobs) // (4 * workers)))

