"""Element-wise comparison of a GPU field with the oracle's, shared by the
GPU parity tests."""

import numpy as np

# relative L2 bars of the two precision paths
TOL = {"f32": 1e-5, "f64": 1e-10}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def assert_parity(s_gpu, ref, prec):
    """Relative L2 error within the path's bar; the largest single-pixel
    error within 5 bars of the largest value; and the two real columns of
    the half spectrum (k_x = 0 and nx/2, which the sweep packs into one
    complex column and updates on half of k_y) within 10 bars of their own
    norm, or of the share of the whole field's bar that falls on one column
    where the column is nearly empty."""
    tol = TOL[prec]
    err = rel(s_gpu, ref)
    emax = float(np.max(np.abs(s_gpu - ref)) / np.max(np.abs(ref)))
    G, R = np.fft.rfft2(s_gpu), np.fft.rfft2(ref)
    nh = R.shape[1]
    cols = []
    for kx in (0, nh - 1):
        col_err = float(np.linalg.norm(G[:, kx] - R[:, kx]))
        bound = max(10 * tol * np.linalg.norm(R[:, kx]), 10 * tol * np.linalg.norm(R) / np.sqrt(nh))
        cols.append((kx, col_err, bound))
    print(f"  rel L2 {err:.2e}, max {emax:.2e}, columns " +
          ", ".join(f"k_x={kx}: {e:.2e} (bound {b:.2e})" for kx, e, b in cols), flush=True)
    assert err < tol
    assert emax < 5 * tol
    for kx, e, b in cols:
        assert e < b, kx
