"""Bases in which each covariance of the problem is diagonal (float64, CPU).

Section 2 of the paper evaluates every messenger equation in the basis where
its covariance is sparse: the pixel-diagonal term in pixel space, the
harmonic-diagonal terms in harmonic space, with the messenger covariances
T_i = tau_i I diagonal everywhere.  On a periodic flat map the harmonic basis
is the unitary 2-D DFT.  The stripe term (noise constant along each row,
Section 3.3) is diagonal in the basis made of row-constant Fourier modes in y
plus anything orthogonal to them; here it is applied literally through row
means and a 1-D DFT over y, not through the 2-D spectrum.

Fields are real (ny, nx) arrays.  An operator f(A) of a covariance A is applied
by going to A's eigenbasis, scaling each coefficient by f(eigenvalue) and
coming back.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft

_WORKERS = 1


def set_workers(n: int) -> None:
    """Threads used by the FFTs of the oracle (scipy.fft ``workers``)."""
    global _WORKERS
    _WORKERS = max(1, int(n))


def get_workers() -> int:
    return _WORKERS


def rfft2u(u: np.ndarray) -> np.ndarray:
    """Unitary 2-D DFT of a real field, half spectrum (ny, nx//2+1)."""
    return sfft.rfft2(u, norm="ortho", workers=_WORKERS)


def irfft2u(uk: np.ndarray, shape) -> np.ndarray:
    """Inverse of ``rfft2u``."""
    return sfft.irfft2(uk, s=shape, norm="ortho", workers=_WORKERS)


def dft_matrix(n: int) -> np.ndarray:
    """Unitary DFT matrix F[k, j] = exp(-2 pi i k j / n) / sqrt(n)."""
    k = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(k, k) / n) / np.sqrt(n)


def full_from_half(half: np.ndarray, nx: int) -> np.ndarray:
    """Eigenvalues on all (ny, nx) modes from those on the rfft2 half spectrum,
    using v(-k) = v(k) for the covariance of a real field."""
    ny = half.shape[0]
    full = np.empty((ny, nx), dtype=half.dtype)
    nh = nx // 2 + 1
    full[:, :nh] = half
    ky_neg = (-np.arange(ny)) % ny
    for kx in range(nh, nx):
        full[:, kx] = half[ky_neg, nx - kx]
    return full


class PixelDiag:
    """A covariance diagonal in pixel space; eigenvalue +inf marks a masked
    pixel (infinite noise variance, zero inverse variance)."""

    def __init__(self, eig: np.ndarray, observed: np.ndarray):
        self.eig = np.asarray(eig, dtype=np.float64)
        self.obs = np.asarray(observed, dtype=bool)

    def messenger_update(self, T: float, nbar_side: np.ndarray,
                         t_side: np.ndarray) -> np.ndarray:
        """(Nbar^-1 + T^-1)^-1 (Nbar^-1 a + T^-1 b), a = nbar_side, b = t_side,
        written as [T a + Nbar b] / (Nbar + T).  A masked pixel has Nbar = inf,
        so the result there is b."""
        e = np.where(self.obs, self.eig, 0.0)
        out = (T * nbar_side + e * t_side) / (e + T)
        return np.where(self.obs, out, t_side)

    def inv_quad(self, u: np.ndarray) -> float:
        """u^T Nbar^-1 u (masked pixels contribute nothing)."""
        e = self.eig[self.obs]
        v = u[self.obs]
        q = np.zeros_like(v)
        nz = e > 0
        q[nz] = v[nz] ** 2 / e[nz]
        if np.any(~nz & (v != 0)):
            return np.inf
        return float(q.sum())


class FourierDiag:
    """A covariance diagonal in the unitary 2-D DFT basis (eigenvalues on the
    rfft2 half spectrum)."""

    def __init__(self, eig_half: np.ndarray, shape):
        self.eig = np.asarray(eig_half, dtype=np.float64)
        self.shape = tuple(shape)

    def apply_fn(self, fn, u: np.ndarray) -> np.ndarray:
        return irfft2u(fn(self.eig) * rfft2u(u), self.shape)

    def messenger_update(self, T: float, nbar_side: np.ndarray,
                         t_side: np.ndarray) -> np.ndarray:
        e = self.eig
        ak = rfft2u(nbar_side)
        bk = rfft2u(t_side)
        return irfft2u((T * ak + e * bk) / (e + T), self.shape)

    def apply(self, u: np.ndarray) -> np.ndarray:
        return irfft2u(self.eig * rfft2u(u), self.shape)

    def inv_quad(self, u: np.ndarray) -> float:
        ny, nx = self.shape
        full = full_from_half(self.eig, nx)
        uk = np.fft.fft2(u, norm="ortho")
        return float(np.sum(np.abs(uk) ** 2 / full))


class StripeDiag:
    """N = N_st + c I where N_st is the covariance of row-constant noise
    n(x, y) = f(y), f stationary with variance P(k_y) per unitary 1-D mode.

    With e_ky(x, y) = exp(2 pi i k_y y / ny) / sqrt(nx ny), N_st = sum_ky
    nx P(k_y) e_ky e_ky^H, so N has eigenvalue nx P(k_y) + c on e_ky and c on
    the complement.  A function f(N) acts as
        f(c) u + broadcast_x( IDFT_y[ (f(nx P + c) - f(c)) DFT_y(rowmean_x u) ] )
    with unitary 1-D DFTs, which is what ``apply_fn`` computes.
    """

    def __init__(self, p_stripe: np.ndarray, c: float, shape):
        self.p = np.asarray(p_stripe, dtype=np.float64)
        self.c = float(c)
        self.shape = tuple(shape)
        ny, nx = self.shape
        self.row_eig = nx * self.p + self.c

    def _row_part(self, u: np.ndarray) -> np.ndarray:
        """Unitary 1-D DFT over y of the row means of u."""
        return np.fft.fft(u.mean(axis=1), norm="ortho")

    def _broadcast(self, vk: np.ndarray) -> np.ndarray:
        ny, nx = self.shape
        col = np.fft.ifft(vk, norm="ortho").real
        return np.broadcast_to(col[:, None], (ny, nx))

    def apply_fn(self, fn, u: np.ndarray) -> np.ndarray:
        fc = fn(np.array(self.c))
        frow = fn(self.row_eig)
        return fc * u + self._broadcast((frow - fc) * self._row_part(u))

    def messenger_update(self, T: float, nbar_side: np.ndarray,
                         t_side: np.ndarray) -> np.ndarray:
        def w_a(e):
            return T / (e + T)

        def w_b(e):
            return e / (e + T)
        return self.apply_fn(w_a, nbar_side) + self.apply_fn(w_b, t_side)

    def apply(self, u: np.ndarray) -> np.ndarray:
        return self.apply_fn(lambda e: e, u)

    def inv_quad(self, u: np.ndarray) -> float:
        """u^T N^-1 u = |u|^2 / c + sum_ky |<e_ky,u>|^2 (1/(nx P + c) - 1/c)."""
        ny, nx = self.shape
        coef = np.sqrt(nx) * self._row_part(u)  # <e_ky, u>
        return float(np.sum(u * u) / self.c
                     + np.sum(np.abs(coef) ** 2 * (1.0 / self.row_eig - 1.0 / self.c)))
