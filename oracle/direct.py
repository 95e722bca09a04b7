"""Wiener filter by its plain definition, for pinning the iteration (CPU, float64).

The converged messenger iteration must equal the Wiener filter
s = S (S + N)^-1 d (eqn wiener-alt).  With a mask (infinite noise variance on
masked pixels, Section 3.3) this reads s = S P^T (P (S+N) P^T)^-1 P d with P
the selection of observed pixels.  Here the dense matrices are built from
their definitions, independently of the FFT-based operators of the iteration:

* a stationary covariance with mode variances V(k) is the circulant whose
  first row is the inverse DFT of V, evaluated as explicit exponential sums;
* the stripe covariance is C_f(y - y') for every pair of pixels, with C_f the
  explicit inverse DFT of the stripe spectrum;
* the white term is diagonal.

Only the S (S+N)^-1 form is used for the solve: S spans more than ten decades
so S^-1 is useless numerically.  Dense solves are for maps up to 64x64.
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from .bases import full_from_half


def _exp_matrix(n: int) -> np.ndarray:
    """E[j, k] = exp(+2 pi i j k / n)."""
    j = np.arange(n)
    return np.exp(2j * np.pi * np.outer(j, j) / n)


def stationary_cov_dense(eig_half: np.ndarray, nx: int) -> np.ndarray:
    """Dense (ny nx) x (ny nx) covariance of a stationary field whose unitary
    2-D DFT modes have variances eig_half (rfft2 layout).  Pixel p = y nx + x.
    c(dy, dx) = (1/(ny nx)) sum_k V(k) exp(2 pi i (ky dy/ny + kx dx/nx))."""
    ny = eig_half.shape[0]
    v = full_from_half(np.asarray(eig_half, dtype=np.float64), nx)
    c = (_exp_matrix(ny) @ v @ _exp_matrix(nx).T).real / (ny * nx)
    y = np.repeat(np.arange(ny), nx)
    x = np.tile(np.arange(nx), ny)
    return c[(y[:, None] - y[None, :]) % ny, (x[:, None] - x[None, :]) % nx]


def stripe_cov_dense(p_stripe: np.ndarray, nx: int) -> np.ndarray:
    """Dense covariance of n(x, y) = f(y): C_f(y - y') for every pixel pair,
    C_f(dy) = (1/ny) sum_ky P(ky) exp(2 pi i ky dy / ny)."""
    p = np.asarray(p_stripe, dtype=np.float64)
    ny = p.size
    cf = (_exp_matrix(ny) @ p).real / ny
    y = np.repeat(np.arange(ny), nx)
    return cf[(y[:, None] - y[None, :]) % ny]


def dense_covariances(problem):
    """(S, N) as dense matrices; N = N_1/f + N_stripe + diag(N_pix)."""
    ny, nx = problem.d.shape
    S = stationary_cov_dense(problem.s_k, nx)
    N = np.diag(np.asarray(problem.n_pix, dtype=np.float64).ravel()).copy()
    if problem.p_oof is not None:
        N += stationary_cov_dense(problem.p_oof, nx)
    if problem.p_stripe is not None:
        N += stripe_cov_dense(problem.p_stripe, nx)
    return S, N


def observed_index(problem) -> np.ndarray:
    if problem.mask is None:
        return np.arange(problem.d.size)
    return np.flatnonzero(np.asarray(problem.mask).ravel() != 0)


def wiener_dense(problem, refine: int = 2) -> np.ndarray:
    """s = S P^T (P (S+N) P^T)^-1 P d by Cholesky, with a few steps of
    iterative refinement (residual in extended precision)."""
    S, _ = dense_covariances(problem)
    return (S @ wiener_dense_x(problem, refine).ravel()).reshape(problem.d.shape)


def wiener_dense_x(problem, refine: int = 2) -> np.ndarray:
    """x = S^-1 s = P^T (P (S+N) P^T)^-1 P d (zero on masked pixels)."""
    S, N = dense_covariances(problem)
    P = observed_index(problem)
    A = (S + N)[np.ix_(P, P)]
    b = np.asarray(problem.d, dtype=np.float64).ravel()[P]
    cf = sla.cho_factor(A, lower=True)
    z = sla.cho_solve(cf, b)
    Al = A.astype(np.longdouble)
    bl = b.astype(np.longdouble)
    for _ in range(refine):
        r = (bl - Al @ z.astype(np.longdouble)).astype(np.float64)
        z = z + sla.cho_solve(cf, r)
    x = np.zeros(problem.d.size)
    x[P] = z
    return x.reshape(problem.d.shape)


def wiener_projected_dense(problem) -> np.ndarray:
    """Wiener filter with infinite noise variance on the Fourier modes where
    the 1/f spectrum is +inf (those modes are projected out of the data,
    Section 4) and on masked pixels, as the exact limit:
        x = Z (Z^T (S + N_f) Z)^-1 Z^T d,   s = S x,
    where N_f is the finite part of N and Z an orthonormal basis of the maps
    that vanish on masked pixels and have no component along the projected
    modes (real and imaginary parts of their unitary DFT vectors)."""
    ny, nx = problem.d.shape
    n = ny * nx
    p = np.asarray(problem.p_oof, dtype=np.float64)
    flag = np.isinf(p)
    fin = dataclasses.replace(problem, p_oof=np.where(flag, 0.0, p))
    S, Nf = dense_covariances(fin)
    full = full_from_half(flag.astype(np.float64), nx) > 0.5
    y = np.repeat(np.arange(ny), nx)
    x = np.tile(np.arange(nx), ny)
    vecs = []
    for ky, kx in zip(*np.nonzero(full)):
        e = np.exp(2j * np.pi * (ky * y / ny + kx * x / nx)) / np.sqrt(n)
        vecs += [e.real, e.imag]
    cols = [np.stack(vecs, axis=1)] if vecs else []
    obs = np.ones(n, bool) if problem.mask is None else np.asarray(problem.mask).ravel() != 0
    masked = np.flatnonzero(~obs)
    if masked.size:
        cols.append(np.eye(n)[:, masked])
    C = np.concatenate(cols, axis=1)
    Z = sla.null_space(C.T)
    A = S + Nf
    d = np.asarray(problem.d, dtype=np.float64).ravel()
    xs = Z @ np.linalg.solve(Z.T @ A @ Z, Z.T @ d)
    return (S @ xs).reshape(ny, nx)


def chi2_dense(problem, s: np.ndarray) -> float:
    """chi^2(s) = s^T S^-1 s + (d - s)^T N^-1 (d - s) (Section 1), with N^-1
    zero on masked pixels: the data term uses (P N P^T)^-1.  The signal term is
    summed over Fourier modes, sum |s_k|^2 / S(k)."""
    ny, nx = problem.d.shape
    sk = np.fft.fft2(s, norm="ortho")
    sfull = full_from_half(np.asarray(problem.s_k, dtype=np.float64), nx)
    prior = float(np.sum(np.abs(sk) ** 2 / sfull))
    _, N = dense_covariances(problem)
    P = observed_index(problem)
    r = (np.asarray(problem.d, dtype=np.float64) - s).ravel()[P]
    cf = sla.cho_factor(N[np.ix_(P, P)], lower=True)
    return prior + float(r @ sla.cho_solve(cf, r))


def grad_chi2_dense(problem, s: np.ndarray) -> np.ndarray:
    """Gradient of chi^2: 2 [S^-1 s - P^T (P N P^T)^-1 P (d - s)]."""
    ny, nx = problem.d.shape
    sfull = full_from_half(np.asarray(problem.s_k, dtype=np.float64), nx)
    prior = np.fft.ifft2(np.fft.fft2(s, norm="ortho") / sfull, norm="ortho").real
    _, N = dense_covariances(problem)
    P = observed_index(problem)
    r = (np.asarray(problem.d, dtype=np.float64) - s).ravel()[P]
    cf = sla.cho_factor(N[np.ix_(P, P)], lower=True)
    g = np.zeros(s.size)
    g[P] = sla.cho_solve(cf, r)
    return 2.0 * (prior - g.reshape(s.shape))


def wiener_stationary(problem) -> np.ndarray:
    """Closed form when the whole N is diagonal in the 2-D Fourier basis (no
    mask, uniform white variance sigma^2): s_k = S/(S + N_1/f + N_st + sigma^2) d_k.
    A row-constant field f(y) has 2-D unitary modes sqrt(nx) f_ky on the
    k_x = 0 column only, so the stripe term contributes nx P(k_y) there."""
    ny, nx = problem.d.shape
    if problem.mask is not None and np.any(np.asarray(problem.mask) == 0):
        raise ValueError("closed form needs no mask")
    npix = np.asarray(problem.n_pix, dtype=np.float64)
    sigma2 = float(npix.flat[0])
    if not np.all(npix == sigma2):
        raise ValueError("closed form needs uniform white noise")
    S = np.asarray(problem.s_k, dtype=np.float64)
    N = np.full_like(S, sigma2)
    if problem.p_oof is not None:
        N = N + np.asarray(problem.p_oof, dtype=np.float64)
    if problem.p_stripe is not None:
        N[:, 0] += nx * np.asarray(problem.p_stripe, dtype=np.float64)
    dk = np.fft.rfft2(np.asarray(problem.d, dtype=np.float64), norm="ortho")
    return np.fft.irfft2(S / (S + N) * dk, s=(ny, nx), norm="ortho")


def inverse_noise_dense(problem) -> np.ndarray:
    """N^-1 d with N^-1 zero on masked pixels: P^T (P N P^T)^-1 P d (the map
    that Section 4's small-alpha Wiener filter approximates)."""
    _, N = dense_covariances(problem)
    P = observed_index(problem)
    b = np.asarray(problem.d, dtype=np.float64).ravel()[P]
    cf = sla.cho_factor(N[np.ix_(P, P)], lower=True)
    out = np.zeros(problem.d.size)
    out[P] = sla.cho_solve(cf, b)
    return out.reshape(problem.d.shape)
