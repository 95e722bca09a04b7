"""The joint objective J_lambda (eqn 2mess_prob) summed in float64 on the GPU.

The sweep kernels add up the quadratic terms of the hierarchical model's
-2 log P on the last sweep of every monitor chunk (pixel term in the row
kernel, Fourier-side terms per mode in the column kernel); the controller
reduces the block partials in a fixed order.  Checked against the oracle's
joint_objective on the same state, against Appendix A's monotonicity at fixed
lambda, and at convergence against the minimum of chi^2, d^T (S + N)^-1 d over
the observed pixels (the messengers marginalise out, Appendix A).
"""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth
from oracle import direct

pytestmark = pytest.mark.gpu

# J is a sum of non-negative terms; the float32 path's fields carry about
# 1e-7 relative rounding per value, which the differences between
# neighbouring messengers amplify
JTOL = {"f64": 1e-8, "f32": 1e-4}
BETA = (0.9, 0.9, 0.95)  # every Nbar_i > 0, so the oracle's J is finite


def _tensors(p, prec):
    import torch
    dt = torch.float32 if prec == "f32" else torch.float64

    def t(a):
        return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    mask = None if p.mask is None else torch.tensor(p.mask, dtype=torch.uint8, device="cuda")
    return t(p.d), t(p.s_k), t(p.n_pix), t(p.p_oof), t(p.p_stripe), mask


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("chain", ["three", "merged", "augmented"])
@pytest.mark.parametrize("shape,K,n", [((64, 64), 8, 40), ((128, 64), 5, 23)])
def test_joint_objective_matches_oracle(gpu_lib, prec, chain, shape, K, n):
    """Every trace record's J against the oracle's J of its own state after
    the same sweeps (ragged last chunk in the second shape)."""
    ny, nx = shape
    print(f"joint {prec} {shape} {chain} K={K} n={n}", flush=True)
    p = synth.make_problem(ny, nx, 31, mask_frac=0.08)
    lams = list(oracle.cooling_ramp(n // 2, n, 300.0))
    ctx = gpu_lib.Context(ny, nx, prec)
    sched = gpu_lib.Schedule(lambdas=lams, rtol=0.0, max_sweeps=n, monitor_every=K,
                             beta=BETA, chain=chain)
    _, rep, trace = ctx.solve(*_tensors(p, prec), schedule=sched)
    res = oracle.solve(p, oracle.FixedSchedule(lams),
                       settings=oracle.Settings(beta=BETA, chain=chain), max_sweeps=n,
                       monitor_every=K, record_joint=True)
    assert trace.shape[0] == len(res.trace)
    for g, o in zip(trace, res.trace):
        assert g[0] == o[0]
        assert np.isfinite(g[5]) and g[5] > 0
        assert g[5] == pytest.approx(o[5], rel=JTOL[prec]), (g[0], g[5], o[5])
    assert rep["chi2_joint"] == trace[-1, 5]
    # |(1 - m) x| of the report is the masked part of the residual monitor
    st = oracle.setup(p, oracle.Settings(beta=BETA, chain=chain))
    dg = oracle.diagnostics(st, res.state, lams[-1])
    assert rep["masked_x_norm"] == pytest.approx(dg.masked_x, rel=1e-8 if prec == "f64" else 2e-3)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("chain", ["three", "augmented"])
def test_joint_objective_never_increases_at_fixed_lambda(gpu_lib, prec, chain):
    """Appendix A: each update maximises the joint probability along one
    field, so at fixed lambda J cannot rise from one check to the next."""
    p = synth.make_problem(128, 128, 32, mask_frac=0.1)
    ctx = gpu_lib.Context(128, 128, prec)
    for lam in (30.0, 1.0):
        sched = gpu_lib.Schedule(lambdas=[lam], rtol=0.0, max_sweeps=96, monitor_every=4,
                                 beta=BETA, chain=chain)
        _, rep, trace = ctx.solve(*_tensors(p, prec), schedule=sched)
        J = trace[:, 5]
        slack = 1e-12 if prec == "f64" else 1e-6
        assert np.all(np.diff(J) <= slack * J[:-1]), np.diff(J).max()
        assert J[-1] < J[0]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_joint_objective_with_unit_white_beta_is_finite(gpu_lib, prec):
    """With the default beta_white = 1 one pixel has Nbar_2 = 0; its exact
    update puts t_2 on the data and its link adds nothing."""
    p = synth.make_problem(64, 64, 33, mask_frac=0.05)
    ctx = gpu_lib.Context(64, 64, prec)
    sched = gpu_lib.Schedule(lambdas=list(oracle.cooling_ramp(10, 20, 100.0)), rtol=0.0,
                             max_sweeps=20, monitor_every=5)
    _, rep, trace = ctx.solve(*_tensors(p, prec), schedule=sched)
    assert np.all(np.isfinite(trace[:, 5])) and np.all(trace[:, 5] > 0)


def test_converged_joint_objective_is_min_chi2(gpu_lib):
    """At lambda = 1 the converged J equals min_s chi^2(s) = d^T (S + N)^-1 d
    over the observed pixels (Appendix A: integrating the messengers out of
    the joint probability returns P(s, d)).  A 64^2 map with a disc mask
    (4' pixels, mild white-noise contrast: it converges to 1e-11 in about
    30k sweeps), float64 augmented chain, against a dense Cholesky solve."""
    p = synth.make_problem(64, 64, 7, pix_arcmin=4.0, stripe_rms=3.0, white_contrast=0.2)
    m = np.ones((64, 64), np.uint8)
    yy, xx = np.mgrid[:64, :64]
    m[(yy - 20) ** 2 + (xx - 40) ** 2 <= 36] = 0
    p.mask = m
    ctx = gpu_lib.Context(64, 64, "f64")
    sched = gpu_lib.Schedule(lambda0=1e4, rtol=1e-11, max_sweeps=80000, monitor_every=4,
                             chain="augmented", stop_full=True)
    _, rep, trace = ctx.solve(*_tensors(p, "f64"), schedule=sched)
    assert rep["status"] == "OK" and rep["lam"] == 1.0
    S, N = direct.dense_covariances(p)
    P = direct.observed_index(p)
    dobs = np.asarray(p.d, dtype=np.float64).ravel()[P]
    cf = sla.cho_factor((S + N)[np.ix_(P, P)], lower=True)
    chi2_min = float(dobs @ sla.cho_solve(cf, dobs))
    assert rep["chi2_joint"] == pytest.approx(chi2_min, rel=1e-9)
