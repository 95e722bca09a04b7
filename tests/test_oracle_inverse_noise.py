"""Section 4's second use of the solver: a small flat signal covariance
S = alpha I turns the Wiener filter into approximate inverse-noise weighting,
N^-1 d ~= alpha^-1 S (S + N)^-1 d."""

import numpy as np
import pytest

import oracle
import synth
from oracle import direct


def _problem(mask):
    p = synth.make_problem(16, 16, 3, pix_arcmin=8.0, stripe_rms=3.0, white_contrast=0.2)
    if mask:
        m = np.ones((16, 16), np.uint8)
        m[4:7, 9:12] = 0
        p.mask = m
    return p


@pytest.mark.parametrize("mask", [False, True])
def test_small_alpha_wiener_tends_to_inverse_noise_linearly(mask):
    """(alpha I + N)^-1 = N^-1 - alpha N^-2 + ..., so the error of the
    approximation falls in proportion to alpha."""
    p = _problem(mask)
    exact = direct.inverse_noise_dense(p)
    errs = []
    for alpha in (1e-2, 1e-3, 1e-4):
        q = synth.make_problem(16, 16, 3, pix_arcmin=8.0, stripe_rms=3.0, white_contrast=0.2)
        q.mask = p.mask
        q.s_k = np.full_like(p.s_k, alpha)
        approx = direct.wiener_dense(q) / alpha
        errs.append(np.linalg.norm(approx - exact) / np.linalg.norm(exact))
    assert errs[0] < 1e-2
    assert 8.0 < errs[0] / errs[1] < 12.0
    assert 8.0 < errs[1] / errs[2] < 12.0
    if mask:
        assert np.all(exact[p.mask == 0] == 0)


def test_iteration_reaches_the_small_alpha_wiener_filter():
    p = _problem(mask=True)
    alpha = 1e-3
    q = synth.make_problem(16, 16, 3, pix_arcmin=8.0, stripe_rms=3.0, white_contrast=0.2)
    q.mask = p.mask
    q.s_k = np.full_like(p.s_k, alpha)
    target = direct.wiener_dense(q) / alpha
    r = oracle.inverse_noise_weight(p, alpha, oracle.AdaptiveSchedule(lam0=1e3, plateau=1e-3),
                                    settings=oracle.Settings(chain="augmented"),
                                    max_sweeps=40000, monitor_every=4, rtol=1e-12,
                                    full_residual=True)
    assert r.converged
    assert np.linalg.norm(r.s - target) / np.linalg.norm(target) < 1e-9
