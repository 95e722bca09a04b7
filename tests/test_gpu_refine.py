"""wf_solve_refined: float32 sweeps refined by float64 residuals.

The float32 iteration alone stalls near rho ~ 1e-5 (rounding of its stored
fields, amplified in the residual); each refinement round solves the
float64 residual's right-hand side with float32 sweeps again and adds the
result.  Pinned against the dense Cholesky Wiener solution far below the
float32 floor (unmasked), and against the float64 path's own residual."""

import numpy as np
import pytest

import synth
from oracle import direct

pytestmark = pytest.mark.gpu


def _t(a, torch):
    return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=torch.float64,
                                               device="cuda")


def _refine(gpu_lib, p, rtol, rounds=6, chain="augmented"):
    import torch
    ny, nx = p.d.shape
    c32 = gpu_lib.Context(ny, nx, "f32")
    c64 = gpu_lib.Context(ny, nx, "f64")
    first = gpu_lib.Schedule(lambda0=1e4, shrink=0.9, rtol=1e-4, max_sweeps=20000,
                             monitor_every=8, chain=chain)
    corr = gpu_lib.Schedule(lambda0=100.0, shrink=0.9, rtol=0.05, max_sweeps=20000,
                            monitor_every=8, chain=chain)
    mask = None if p.mask is None else torch.tensor(p.mask, dtype=torch.uint8, device="cuda")
    s, rep, trace = gpu_lib.solve_refined(c32, c64, _t(p.d, torch), _t(p.s_k, torch),
                                          _t(p.n_pix, torch), _t(p.p_oof, torch),
                                          _t(p.p_stripe, torch), mask, first=first, corr=corr,
                                          max_rounds=rounds, rtol=rtol)
    for row in trace:
        print(f"  round {int(row[0])}: {int(row[1])} sweeps, rho {row[2]:.2e}, "
              f"rho_mask {row[3]:.2e}", flush=True)
    return s.cpu().numpy(), rep


def test_refined_float32_reaches_the_dense_solution(gpu_lib):
    """64^2, three noise terms, no mask: float32 sweeps with float64
    refinement to rho <= 1e-12 equal the dense Cholesky solution to 1e-10,
    far below what float32 fields reach alone (rho ~ 1e-5)."""
    p = synth.make_problem(64, 64, 1)
    s, rep = _refine(gpu_lib, p, 1e-12)
    print(f"  refined: {rep['status']} rounds {rep['refine_rounds']} sweeps {rep['sweeps']} "
          f"rho {rep['rho']:.2e}", flush=True)
    assert rep["status"] == "OK" and rep["rho"] <= 1e-12
    assert rep["refine_rounds"] >= 2
    sd = direct.wiener_dense(p)
    err = float(np.linalg.norm(s - sd) / np.linalg.norm(sd))
    print(f"  vs dense Cholesky: {err:.2e}", flush=True)
    assert err < 1e-10


def test_refined_masked_reaches_a_residual_float32_cannot(gpu_lib):
    """With a mask the refinement drives the observed residual far below
    the float32 floor as well (the masked part of x, which the residual does
    not see, stays at round 0's level)."""
    p = synth.make_problem(128, 128, 3, mask_frac=0.1)
    s, rep = _refine(gpu_lib, p, 1e-10)
    assert rep["status"] == "OK" and rep["rho"] <= 1e-10
    assert rep["refine_rounds"] >= 2
    assert np.all(np.isfinite(s))


def test_refined_reports_not_converged_when_rounds_run_out(gpu_lib):
    p = synth.make_problem(64, 64, 2, mask_frac=0.05)
    s, rep = _refine(gpu_lib, p, 1e-14, rounds=0)
    assert rep["status"] == "NOT_CONVERGED" and rep["refine_rounds"] == 1
    assert np.all(np.isfinite(s))


def test_refined_c3_residual_checked_by_oracle(gpu_lib):
    """The benchmark's fastest route to rho <= 1e-6 on the masked 2048^2 map
    (float32 sweeps cooled by lambda^0.8 with checks every 8 sweeps, float64
    refinement): the oracle evaluates Section 2's residual of the returned
    chain field u = S_chain x itself and finds rho <= 1e-6, equal to the
    library's own float64 figure."""
    import torch
    import oracle
    p = synth.named_config("c3")
    n = p.d.shape[0]
    print("refined c3, oracle residual", flush=True)
    c32 = gpu_lib.Context(n, n, "f32")
    c64 = gpu_lib.Context(n, n, "f64")
    first = gpu_lib.Schedule(lambda0=1e4, shrink=0.8, rtol=1e-3, max_sweeps=30000,
                             monitor_every=8, chain="augmented", chain_field=True)
    corr = gpu_lib.Schedule(lambda0=300.0, shrink=0.8, rtol=0.1, max_sweeps=30000,
                            monitor_every=8, chain="augmented")
    mask = torch.tensor(p.mask, dtype=torch.uint8, device="cuda")
    u, rep, trace = gpu_lib.solve_refined(c32, c64, _t(p.d, torch), _t(p.s_k, torch),
                                          _t(p.n_pix, torch), _t(p.p_oof, torch),
                                          _t(p.p_stripe, torch), mask, first=first, corr=corr,
                                          max_rounds=4, rtol=1e-6)
    print(f"  {rep['status']} rounds {rep['refine_rounds']} sweeps {rep['sweeps']} "
          f"rho {rep['rho']:.2e} rho_mask {rep['rho_mask']:.2e}", flush=True)
    assert rep["status"] == "OK"
    st = oracle.setup(p, oracle.Settings(chain="augmented"))
    dg = oracle.diagnostics_of_field(st, u.cpu().numpy())
    print(f"  oracle: rho {dg.rho:.3e} rho_mask {dg.rho_mask:.3e}", flush=True)
    assert dg.rho <= 1e-6
    assert dg.rho == pytest.approx(rep["rho"], rel=1e-6)
    assert dg.rho_mask == pytest.approx(rep["rho_mask"], rel=1e-6)


def test_refined_output_modes_agree(gpu_lib):
    """s = S x and u = S_chain x from the same refined solve: u's signal part
    S (S + N_F)^-1 u equals s (64^2, three terms, mask)."""
    import torch
    p = synth.make_problem(64, 64, 7, mask_frac=0.1)
    outs = []
    for cf in (False, True):
        c32 = gpu_lib.Context(64, 64, "f32")
        c64 = gpu_lib.Context(64, 64, "f64")
        first = gpu_lib.Schedule(lambda0=1e4, shrink=0.9, rtol=1e-4, max_sweeps=20000,
                                 monitor_every=8, chain="augmented", chain_field=cf)
        corr = gpu_lib.Schedule(lambda0=100.0, shrink=0.9, rtol=0.05, max_sweeps=20000,
                                monitor_every=8, chain="augmented")
        mask = torch.tensor(p.mask, dtype=torch.uint8, device="cuda")
        s, rep, _ = gpu_lib.solve_refined(c32, c64, _t(p.d, torch), _t(p.s_k, torch),
                                          _t(p.n_pix, torch), _t(p.p_oof, torch),
                                          _t(p.p_stripe, torch), mask, first=first, corr=corr,
                                          max_rounds=3, rtol=1e-9)
        outs.append((s.cpu().numpy(), rep))
    (s, r0), (u, r1) = outs
    assert r0["rho"] == r1["rho"] and r0["sweeps"] == r1["sweeps"]
    # s = S S_chain^-1 u, mode by mode (unitary transforms of the oracle)
    import oracle
    from oracle.bases import irfft2u, rfft2u
    st = oracle.setup(p, oracle.Settings(chain="augmented"))
    s_from_u = irfft2u(rfft2u(u) * (st.S.eig / st.S_chain.eig), u.shape)
    assert np.linalg.norm(s_from_u - s) / np.linalg.norm(s) < 1e-12


def test_refined_warm_start_from_the_solution_needs_one_round(gpu_lib):
    """Round 0 warm-started (field mode 1) from the refined solution's own
    chain field: the float32 solve starts at its fixed point, so the float64
    residual is at the float32 rounding level after one check, and the
    refinement from there ends where the first one did."""
    import torch
    p = synth.make_problem(128, 128, 8, mask_frac=0.1)
    c32 = gpu_lib.Context(128, 128, "f32")
    c64 = gpu_lib.Context(128, 128, "f64")
    mask = torch.tensor(p.mask, dtype=torch.uint8, device="cuda")
    args = (_t(p.d, torch), _t(p.s_k, torch), _t(p.n_pix, torch), _t(p.p_oof, torch),
            _t(p.p_stripe, torch), mask)

    def sched(lam0, cf):
        return gpu_lib.Schedule(lambda0=lam0, shrink=0.8, rtol=1e-3, max_sweeps=20000,
                                monitor_every=8, chain="augmented", chain_field=cf)
    corr = gpu_lib.Schedule(lambda0=300.0, shrink=0.8, rtol=0.1, max_sweeps=20000,
                            monitor_every=8, chain="augmented")
    u, rep0, _ = gpu_lib.solve_refined(c32, c64, *args, first=sched(1e4, True), corr=corr,
                                       max_rounds=4, rtol=1e-8)
    assert rep0["status"] == "OK"
    u1, rep1, tr1 = gpu_lib.solve_refined(c32, c64, *args, first=sched(1.0, True), corr=corr,
                                          max_rounds=4, rtol=1e-8, s_init=u)
    print(f"  from zero: {rep0['sweeps']} sweeps; from its own solution: {rep1['sweeps']} "
          f"sweeps, rho after round 0 {tr1[0][2]:.2e}", flush=True)
    assert rep1["status"] == "OK"
    assert tr1[0][1] <= 16 and tr1[0][2] < 1e-4
    assert rep1["sweeps"] < rep0["sweeps"]
    u_np, u1_np = u.cpu().numpy(), u1.cpu().numpy()
    assert np.linalg.norm(u1_np - u_np) / np.linalg.norm(u_np) < 1e-4
