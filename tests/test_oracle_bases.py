"""Pins of the oracle's basis operators against definitions written out
independently (explicit DFT matrices, explicit exponential sums)."""

import numpy as np
import pytest

from oracle import bases, direct


@pytest.mark.parametrize("n", [8, 16, 64])
def test_dft_matrix_matches_fft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    F = bases.dft_matrix(n)
    np.testing.assert_allclose(F @ x, np.fft.fft(x, norm="ortho"), rtol=0, atol=1e-13)
    np.testing.assert_allclose(F.conj().T @ F, np.eye(n), atol=1e-13)


@pytest.mark.parametrize("shape", [(8, 8), (16, 8), (64, 64)])
def test_rfft2u_is_unitary_dft(shape):
    ny, nx = shape
    rng = np.random.default_rng(1)
    u = rng.standard_normal(shape)
    full = bases.dft_matrix(ny) @ u @ bases.dft_matrix(nx).T
    half = bases.rfft2u(u)
    np.testing.assert_allclose(half, full[:, : nx // 2 + 1], atol=1e-12)
    np.testing.assert_allclose(bases.irfft2u(half, shape), u, atol=1e-13)


def test_full_from_half_hermitian_map():
    ny, nx = 6, 8
    rng = np.random.default_rng(2)
    u = rng.standard_normal((ny, nx))
    spec = np.abs(np.fft.fft2(u)) ** 2  # symmetric under k -> -k
    half = spec[:, : nx // 2 + 1]
    np.testing.assert_allclose(bases.full_from_half(half, nx), spec, rtol=1e-14)


def _hermitian_positive(ny, nx, rng):
    v = np.abs(np.fft.fft2(rng.standard_normal((ny, nx)))) ** 2 + 0.5
    return v[:, : nx // 2 + 1]


def test_fourier_operator_matches_dense_circulant():
    ny, nx = 8, 6
    rng = np.random.default_rng(3)
    eig = _hermitian_positive(ny, nx, rng)
    op = bases.FourierDiag(eig, (ny, nx))
    M = direct.stationary_cov_dense(eig, nx)
    u = rng.standard_normal((ny, nx))
    np.testing.assert_allclose(op.apply(u).ravel(), M @ u.ravel(), rtol=1e-12, atol=1e-12)
    inv = op.apply_fn(lambda e: 1.0 / e, u)
    np.testing.assert_allclose(inv.ravel(), np.linalg.solve(M, u.ravel()), rtol=1e-10, atol=1e-12)
    assert op.inv_quad(u) == pytest.approx(u.ravel() @ np.linalg.solve(M, u.ravel()), rel=1e-11)


def test_stripe_operator_matches_dense_row_covariance():
    ny, nx = 8, 5
    rng = np.random.default_rng(4)
    p = rng.uniform(0.5, 3.0, ny)
    p = 0.5 * (p + p[(-np.arange(ny)) % ny])  # P(k) = P(-k): real stripes
    c = 0.7
    op = bases.StripeDiag(p, c, (ny, nx))
    M = direct.stripe_cov_dense(p, nx) + c * np.eye(ny * nx)
    u = rng.standard_normal((ny, nx))
    np.testing.assert_allclose(op.apply(u).ravel(), M @ u.ravel(), rtol=1e-12, atol=1e-12)
    f = op.apply_fn(lambda e: 1.0 / (e + 2.0), u)
    np.testing.assert_allclose(f.ravel(), np.linalg.solve(M + 2.0 * np.eye(ny * nx), u.ravel()),
                               rtol=1e-11, atol=1e-12)
    assert op.inv_quad(u) == pytest.approx(u.ravel() @ np.linalg.solve(M, u.ravel()), rel=1e-11)


def test_stripe_term_is_kx0_column_of_2d_spectrum():
    """Row-constant noise has unitary 2-D modes only on k_x = 0, with variance
    nx P(k_y): the dense stripe covariance diagonalised by the 2-D DFT."""
    ny, nx = 8, 4
    rng = np.random.default_rng(5)
    p = rng.uniform(0.5, 3.0, ny)
    p = 0.5 * (p + p[(-np.arange(ny)) % ny])
    M = direct.stripe_cov_dense(p, nx)
    F = np.kron(bases.dft_matrix(ny), bases.dft_matrix(nx))
    D = F @ M @ F.conj().T
    expect = np.zeros((ny, nx))
    expect[:, 0] = nx * p
    np.testing.assert_allclose(D, np.diag(expect.ravel()), atol=1e-12)
