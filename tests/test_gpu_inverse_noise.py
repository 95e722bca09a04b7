"""wf_inverse_noise_weight (Section 4, S = alpha I) against the oracle."""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

from parity_checks import TOL, assert_parity


def _t(a, prec, torch):
    dt = torch.float32 if prec == "f32" else torch.float64
    return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("chain", ["three", "augmented"])
def test_inverse_noise_weight_parity(gpu_lib, prec, chain):
    import torch
    p = synth.make_problem(64, 128, 12, mask_frac=0.06)
    alpha = 0.5
    lams = list(oracle.cooling_ramp(20, 30, 1e3))
    print(f"inverse noise {prec} {chain}", flush=True)
    ctx = gpu_lib.Context(64, 128, prec)
    sched = gpu_lib.Schedule(lambdas=lams, rtol=0.0, max_sweeps=len(lams), monitor_every=10,
                             chain=chain)
    out, rep, trace = ctx.inverse_noise_weight(
        _t(p.d, prec, torch), _t(p.n_pix, prec, torch), _t(p.p_oof, prec, torch),
        _t(p.p_stripe, prec, torch), torch.tensor(p.mask, device="cuda"), alpha=alpha,
        schedule=sched)
    ref = oracle.inverse_noise_weight(p, alpha, oracle.FixedSchedule(lams),
                                      settings=oracle.Settings(chain=chain),
                                      max_sweeps=len(lams), monitor_every=10)
    got = out.cpu().numpy().astype(np.float64)
    assert_parity(got, ref.s, prec)


def test_inverse_noise_weight_converges_to_dense(gpu_lib):
    """Float64, augmented chain, run to convergence: equals the dense
    small-alpha Wiener filter, which is within O(alpha) of N^-1 d."""
    import torch
    from oracle import direct
    p = synth.make_problem(64, 64, 13, mask_frac=0.05)
    alpha = 1e-3
    ctx = gpu_lib.Context(64, 64, "f64")
    sched = gpu_lib.Schedule(lambda0=1e4, rtol=1e-12, max_sweeps=20000, monitor_every=8,
                             chain="augmented", stop_full=True)
    out, rep, _ = ctx.inverse_noise_weight(
        _t(p.d, "f64", torch), _t(p.n_pix, "f64", torch), _t(p.p_oof, "f64", torch),
        _t(p.p_stripe, "f64", torch), torch.tensor(p.mask, device="cuda"), alpha=alpha,
        schedule=sched)
    assert rep["status"] == "OK"
    q = synth.make_problem(64, 64, 13, mask_frac=0.05)
    q.s_k = np.full_like(q.s_k, alpha)
    target = direct.wiener_dense(q) / alpha
    got = out.cpu().numpy()
    assert np.linalg.norm(got - target) / np.linalg.norm(target) < 1e-8
    exact = direct.inverse_noise_dense(p)
    assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < 1e-2
