"""The library's own 2-D FFT kernels (the transforms every sweep uses) against
numpy, in both precisions."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SHAPES = [(64, 64), (128, 64), (64, 256), (512, 512), (1024, 1024), (2048, 2048), (256, 4096),
          (4096, 256), (384, 384), (768, 256), (128, 1536), (1536, 768)]


def _tol(prec, n):
    return 2e-6 * np.log2(n) if prec == "f32" else 1e-14 * np.log2(n)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("shape", SHAPES)
def test_rfft2_matches_numpy(gpu_lib, prec, shape):
    import torch
    ny, nx = shape
    if not gpu_lib.load().wf_supported(ny, nx, 0 if prec == "f32" else 1):
        pytest.skip("size not built for this precision")
    print(f"rfft2 {prec} {shape}", flush=True)
    rng = np.random.default_rng(ny * 7 + nx)
    x = rng.standard_normal((ny, nx))
    dt = torch.float32 if prec == "f32" else torch.float64
    xt = torch.tensor(x, dtype=dt, device="cuda")
    ctx = gpu_lib.Context(ny, nx, prec)
    X = ctx.rfft2(xt).cpu().numpy()
    ref = np.fft.rfft2(xt.cpu().numpy().astype(np.float64))
    err = np.linalg.norm(X - ref) / np.linalg.norm(ref)
    assert err < _tol(prec, ny * nx), err
    back = ctx.irfft2(torch.tensor(ref, device="cuda",
                                   dtype=torch.complex64 if prec == "f32" else torch.complex128))
    back = back.cpu().numpy()
    ref_back = np.fft.irfft2(ref.astype(np.complex128), s=shape)
    err2 = np.linalg.norm(back - ref_back) / np.linalg.norm(ref_back)
    assert err2 < _tol(prec, ny * nx), err2


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_irfft2_ignores_imaginary_dc_and_nyquist_like_numpy(gpu_lib, prec):
    import torch
    ny, nx = 64, 128
    rng = np.random.default_rng(3)
    X = rng.standard_normal((ny, nx // 2 + 1)) + 1j * rng.standard_normal((ny, nx // 2 + 1))
    ctx = gpu_lib.Context(ny, nx, prec)
    cd = torch.complex64 if prec == "f32" else torch.complex128
    Xt = torch.tensor(X, dtype=cd, device="cuda")
    got = ctx.irfft2(Xt).cpu().numpy()
    ref = np.fft.irfft2(Xt.cpu().numpy().astype(np.complex128), s=(ny, nx))
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < _tol(prec, ny * nx)
