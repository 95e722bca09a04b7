"""GPU messenger iteration against the CPU float64 oracle on identical inputs.

Iterate parity: both sides run the same fixed lambda sequence for the same
number of sweeps and the signal estimates are compared element by element
(relative L2): <= 1e-10 for the float64 path, <= 1e-5 for the float32 path.
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

from parity_checks import TOL
from parity_checks import assert_parity as _assert_parity


def _tensors(p, prec, device="cuda"):
    import torch
    dt = torch.float32 if prec == "f32" else torch.float64

    def t(a):
        return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=dt, device=device)
    mask = None if p.mask is None else torch.tensor(p.mask, dtype=torch.uint8, device=device)
    return t(p.d), t(p.s_k), t(p.n_pix), t(p.p_oof), t(p.p_stripe), mask


def _run_both(gpu_lib, p, prec, lams, *, chain="three", beta=(0.9, 0.9, 1.0), floor_frac=0.5,
              monitor_every=8, s_init=None, chain_field=False):
    import torch
    ny, nx = p.d.shape
    print(f"parity {prec} {ny}x{nx} chain={chain} sweeps={len(lams)} "
          f"mask={p.mask is not None} oof={p.p_oof is not None} "
          f"stripe={p.p_stripe is not None} warm={s_init is not None}", flush=True)
    ctx = gpu_lib.Context(ny, nx, prec)
    sched = gpu_lib.Schedule(lambdas=list(lams), rtol=0.0, max_sweeps=len(lams),
                             monitor_every=monitor_every, beta=beta, floor_frac=floor_frac,
                             chain=chain, chain_field=chain_field)
    args = _tensors(p, prec)
    si = None
    if s_init is not None:
        si = torch.tensor(s_init, dtype=args[0].dtype, device="cuda")
    s_gpu, rep, trace = ctx.solve(*args, schedule=sched, s_init=si)
    s_gpu = s_gpu.cpu().numpy().astype(np.float64)
    si_np = None if si is None else si.cpu().numpy().astype(np.float64)
    res = oracle.solve(p, oracle.FixedSchedule(list(lams)),
                       settings=oracle.Settings(beta=beta, floor_frac=floor_frac, chain=chain),
                       s_init=si_np, max_sweeps=len(lams), monitor_every=monitor_every,
                       chain_field=chain_field)
    return s_gpu, rep, trace, res


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _ramp(n_cool, n, lam0=1e3):
    return oracle.cooling_ramp(n_cool, n, lam0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("chain", ["three", "merged", "augmented"])
def test_iterate_parity_c1_shape(gpu_lib, prec, chain):
    p = synth.make_problem(64, 64, 1)
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, prec, _ramp(40, 60), chain=chain)
    assert rep["sweeps"] == 60 and rep["status"] == "NOT_CONVERGED"
    _assert_parity(s_gpu, res.s, prec)
    # monitor trace: same sweeps, lambdas and residuals
    assert trace.shape[0] == len(res.trace)
    for g, o in zip(trace, res.trace):
        assert g[0] == o[0] and g[1] == o[1]
        rt = 1e-8 if prec == "f64" else 2e-3
        assert g[2] == pytest.approx(o[2], rel=rt)
        assert g[4] == pytest.approx(o[4], rel=rt, abs=1e-12)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(128, 64), (64, 256), (256, 256)])
def test_iterate_parity_masked_nonsquare(gpu_lib, prec, shape):
    ny, nx = shape
    p = synth.make_problem(ny, nx, 21, mask_frac=0.08)
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, prec, _ramp(20, 40), monitor_every=16)
    _assert_parity(s_gpu, res.s, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(384, 128), (128, 768), (768, 384), (1536, 64)])
def test_iterate_parity_radix3_lengths(gpu_lib, prec, shape):
    """Lengths 3 x 2^k use a radix-3 pass (384, 768, 1536)."""
    ny, nx = shape
    p = synth.make_problem(ny, nx, 23, mask_frac=0.05)
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, prec, _ramp(10, 20), monitor_every=8)
    _assert_parity(s_gpu, res.s, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("terms", [("oof",), ("stripe",), (), ("oof", "stripe")])
@pytest.mark.parametrize("chain", ["three", "merged", "augmented"])
def test_iterate_parity_term_subsets(gpu_lib, prec, terms, chain):
    p = synth.make_problem(64, 128, 5, mask_frac=0.05,
                           oof_level=10.0 if "oof" in terms else None,
                           stripe_rms=10.0 if "stripe" in terms else None)
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, prec, _ramp(12, 24), chain=chain,
                                       monitor_every=5)
    _assert_parity(s_gpu, res.s, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("chain", ["three", "augmented"])
def test_warm_start_parity(gpu_lib, prec, chain):
    p = synth.make_problem(64, 64, 9, mask_frac=0.1)
    s_init = np.asarray(p.s_true, dtype=np.float32 if prec == "f32" else np.float64)
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, prec, _ramp(10, 20, 50.0), chain=chain,
                                       s_init=s_init)
    _assert_parity(s_gpu, res.s, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("chain", ["three", "augmented"])
@pytest.mark.parametrize("warm", [False, True])
def test_chain_field_mode_parity(gpu_lib, prec, chain, warm):
    """field_mode 1: warm start and output are the chain's signal-end field."""
    p = synth.make_problem(64, 128, 10, mask_frac=0.1)
    s_init = None
    if warm:
        s_init = np.asarray(1.1 * p.s_true, dtype=np.float32 if prec == "f32" else np.float64)
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, prec, _ramp(10, 20, 20.0), chain=chain,
                                       s_init=s_init, chain_field=True)
    _assert_parity(s_gpu, res.s, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("chain", ["three", "merged", "augmented"])
def test_projected_modes_parity(gpu_lib, prec, chain):
    """A 1/f variance of +inf projects a Fourier mode out of the data."""
    import dataclasses
    p = synth.make_problem(64, 64, 12, mask_frac=0.1)
    po = np.array(p.p_oof)
    for ky, kx in [(0, 0), (1, 0), (63, 0), (0, 1), (1, 1), (63, 1)]:
        po[ky, kx] = np.inf
    p = dataclasses.replace(p, p_oof=po)
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, prec, _ramp(20, 40), chain=chain,
                                       monitor_every=8)
    assert np.all(np.isfinite(s_gpu))
    _assert_parity(s_gpu, res.s, prec)


def test_projected_every_mode_is_rejected(gpu_lib):
    import torch
    p = synth.make_problem(64, 64, 13)
    args = list(_tensors(p, "f64"))
    args[3] = torch.full_like(args[3], float("inf"))
    ctx = gpu_lib.Context(64, 64, "f64")
    with pytest.raises(gpu_lib.WFError) as e:
        ctx.solve(*args, schedule=gpu_lib.Schedule(lambdas=[1.0], max_sweeps=1, rtol=0.0))
    assert e.value.status == -1


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_sweep_and_ragged_chunk(gpu_lib, prec):
    """max_sweeps = 1, and a budget that is not a multiple of the monitor
    interval (the last chunk is partial)."""
    p = synth.make_problem(64, 64, 2)
    for lams, K in (([30.0], 4), (list(_ramp(7, 13, 100.0)), 5)):
        s_gpu, rep, trace, res = _run_both(gpu_lib, p, prec, lams, monitor_every=K)
        assert rep["sweeps"] == len(lams)
        _assert_parity(s_gpu, res.s, prec)
        assert trace[-1][0] == len(lams) - 1


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adaptive_schedule_replayed_by_oracle(gpu_lib, prec):
    """The adaptive lambda trajectory depends on rounding, so the oracle
    replays the lambdas the GPU recorded (constant within a monitor chunk)."""
    import torch  # noqa: F401
    p = synth.make_problem(64, 64, 4)
    ctx = gpu_lib.Context(64, 64, prec)
    K = 4
    sched = gpu_lib.Schedule(lambda0=1e3, rtol=0.0, max_sweeps=80, monitor_every=K,
                             chain="augmented")
    s_gpu, rep, trace = ctx.solve(*_tensors(p, prec), schedule=sched)
    lams = np.repeat(trace[:, 1], K)[: rep["sweeps"]]
    assert trace[0, 1] == 1e3 and lams[-1] < 1e3  # it did cool
    res = oracle.solve(p, oracle.FixedSchedule(list(lams)),
                       settings=oracle.Settings(chain="augmented"), max_sweeps=len(lams),
                       monitor_every=K)
    _assert_parity(s_gpu.cpu().numpy().astype(np.float64), res.s, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adaptive_decisions_follow_the_section_3_3_rule(gpu_lib, prec):
    """The device controller's cooling decisions, replayed on the host from
    the residuals the GPU itself recorded through oracle.next_lambda (the
    rule pinned on hand-built sequences): every lambda in the trace is the
    rule's output after the previous check."""
    p = synth.make_problem(128, 128, 14, mask_frac=0.05)
    ctx = gpu_lib.Context(128, 128, prec)
    K = 4
    sched = gpu_lib.Schedule(lambda0=1e4, shrink=0.7, plateau=3e-2, rtol=0.0, max_sweeps=600,
                             monitor_every=K, chain="augmented")
    _, rep, trace = ctx.solve(*_tensors(p, prec), schedule=sched)
    rule = oracle.AdaptiveSchedule(lam0=1e4, shrink=0.7, plateau=3e-2, snap=1e-3)
    lam, prev = 1e4, None
    shrinks = 0
    for i, row in enumerate(trace):
        assert row[1] == pytest.approx(lam, rel=1e-14), i
        new, prev = oracle.next_lambda(rule, lam, prev, int(row[0]), row[3])
        shrinks += new < lam
        lam = new
    assert shrinks >= 5


@pytest.mark.parametrize("chain", ["merged", "three"])
def test_projected_modes_float32_full_size(gpu_lib, chain):
    """Projected modes (1/f variance +inf, carried as 1e30) on the 2048^2 map
    in float32: the sweep forms normalised weights before touching a field,
    so no product overflows (unnormalised low-k coefficients reach 2e8)."""
    import dataclasses
    oracle.bases.set_workers(16)
    p = synth.named_config("c3")
    po = np.array(p.p_oof)
    for ky in (0, 1, 2, 2046, 2047):
        po[ky, :3] = np.inf
    p = dataclasses.replace(p, p_oof=po)
    lams = [1e4, 3e3, 1e3]
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, "f32", lams, chain=chain, monitor_every=3)
    assert np.all(np.isfinite(s_gpu))
    _assert_parity(s_gpu, res.s, "f32")


def test_converges_to_dense_wiener_solution_f64(gpu_lib):
    """C1 workload (64x64, three terms) on the float64 path with the
    augmented chain, run to rho <= 1e-12 and compared with the dense
    4096x4096 Cholesky solve."""
    from oracle import direct
    p = synth.named_config("c1")
    ctx = gpu_lib.Context(64, 64, "f64")
    sched = gpu_lib.Schedule(lambda0=1e4, rtol=1e-12, max_sweeps=5000, monitor_every=4,
                             chain="augmented")
    s_gpu, rep, trace = ctx.solve(*_tensors(p, "f64"), schedule=sched)
    assert rep["status"] == "OK"
    sd = direct.wiener_dense(p)
    _assert_parity(s_gpu.cpu().numpy(), sd, "f64")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_stationary_closed_form_one_sweep(gpu_lib, prec):
    """Uniform white noise with beta_white = 1 and the augmented chain: the
    single messenger takes all the pixel noise and one sweep at lambda = 1 is
    the exact per-mode filter (Section 3.1), at a bench-sized map."""
    from oracle import direct
    n = 1024 if prec == "f64" else 2048
    p = synth.make_stationary_problem(n, n, 8)
    ctx = gpu_lib.Context(n, n, prec)
    sched = gpu_lib.Schedule(lambdas=[1.0], rtol=0.0, max_sweeps=1, monitor_every=1,
                             chain="augmented")
    s_gpu, rep, trace = ctx.solve(*_tensors(p, prec), schedule=sched)
    sc = direct.wiener_stationary(p)
    _assert_parity(s_gpu.cpu().numpy().astype(np.float64), sc, prec)
    assert rep["rho"] < (1e-12 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("n", [1024, 2048])
def test_full_size_parity_float64_three_levels(gpu_lib, n):
    """The float64 three-level kernels at 1024^2 and 2048^2 (16 values per
    thread; the 2048-point column kernel spills) for 50 sweeps of cooling
    from 1e4, masked C3 recipe, against the oracle at 1e-10."""
    oracle.bases.set_workers(16)
    p = synth.named_config("c3") if n == 2048 else synth.make_problem(n, n, 3, mask_frac=0.10)
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, "f64", _ramp(40, 50, 1e4), monitor_every=16)
    _assert_parity(s_gpu, res.s, "f64")
    for g, o in zip(trace, res.trace):
        assert g[2] == pytest.approx(o[2], rel=1e-8)


def test_full_size_parity_float32_1024(gpu_lib):
    """The float32 8-value row and column kernels at 1024^2 (C3 recipe)."""
    oracle.bases.set_workers(16)
    p = synth.make_problem(1024, 1024, 3, mask_frac=0.10)
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, "f32", _ramp(40, 50, 1e4), monitor_every=16)
    _assert_parity(s_gpu, res.s, "f32")


@pytest.mark.parametrize("chain", ["three", "merged", "augmented"])
@pytest.mark.parametrize("shape", [(4096, 128), (128, 4096)])
def test_parity_float32_4096_point_kernels(gpu_lib, shape, chain):
    """The float32 kernels at the longest supported length: 4096-point
    column transforms (16 values per thread, per-mode state four modes at a
    time) and 4096-point row transforms, masked, every chain."""
    ny, nx = shape
    p = synth.make_problem(ny, nx, 27, mask_frac=0.05)
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, "f32", _ramp(8, 12), monitor_every=4,
                                       chain=chain)
    assert rep["sweeps"] == 12
    _assert_parity(s_gpu, res.s, "f32")


@pytest.mark.parametrize("prec,n,tile", [("f32", 1536, 1), ("f32", 1536, 5), ("f32", 768, 3),
                                         ("f64", 1536, 1)])
def test_full_size_parity_radix3(gpu_lib, prec, n, tile):
    """The 12-value kernels (five-pass 1536-point plan, four-pass 768-point
    plan) at the batch's full sizes, in the default tiling and in the ones
    the batch's autotuner picks (float32), masked C3 recipe, against the
    oracle; the residual trace too."""
    oracle.bases.set_workers(16)
    p = synth.make_problem(n, n, 3, mask_frac=0.10)
    lams = list(_ramp(40, 50, 1e4))
    print(f"parity {prec} {n}x{n} tiling {tile}", flush=True)
    ctx = gpu_lib.Context(n, n, prec)
    assert ctx.set_tile(tile)
    sched = gpu_lib.Schedule(lambdas=lams, rtol=0.0, max_sweeps=len(lams), monitor_every=16)
    s_gpu, rep, trace = ctx.solve(*_tensors(p, prec), schedule=sched)
    res = oracle.solve(p, oracle.FixedSchedule(lams), max_sweeps=len(lams), monitor_every=16)
    _assert_parity(s_gpu.cpu().numpy().astype(np.float64), res.s, prec)
    for g, o in zip(trace, res.trace):
        assert g[2] == pytest.approx(o[2], rel=1e-8 if prec == "f64" else 2e-3)


def test_c3_benchmark_run_parity(gpu_lib):
    """The benchmark's step exactly: the 2048^2 masked map, three-level
    float32 chain, 500 sweeps of lambda_k = 1e4^(1 - k/400) then 1, residual
    every 16 sweeps, in the tiling the benchmark's autotuner picks (8 x 2
    tiles, 4 rows per row block), against the float64 oracle."""
    oracle.bases.set_workers(16)
    p = synth.named_config("c3")
    lams = list(oracle.cooling_ramp(400, 500, 1e4))
    ctx = gpu_lib.Context(2048, 2048, "f32")
    assert ctx.set_tile(3)
    sched = gpu_lib.Schedule(lambdas=lams, rtol=0.0, max_sweeps=500, monitor_every=16)
    s_gpu, rep, trace = ctx.solve(*_tensors(p, "f32"), schedule=sched)
    s_gpu = s_gpu.cpu().numpy().astype(np.float64)
    print("  oracle: 500 sweeps at 2048^2", flush=True)
    res = oracle.solve(p, oracle.FixedSchedule(lams), max_sweeps=500, monitor_every=16)
    _assert_parity(s_gpu, res.s, "f32")
    assert trace.shape[0] == len(res.trace)
    for g, o in zip(trace, res.trace):
        assert g[0] == o[0] and g[1] == o[1]
        assert g[2] == pytest.approx(o[2], rel=2e-3)


def test_full_size_iterate_parity_c3(gpu_lib):
    """The 2048x2048 masked workload in the launch configuration the
    benchmark times (float32, three levels): a few sweeps against the oracle."""
    oracle.bases.set_workers(16)
    p = synth.named_config("c3")
    lams = [1e4, 5e3, 2e3, 1e3]
    s_gpu, rep, trace, res = _run_both(gpu_lib, p, "f32", lams, monitor_every=2)
    _assert_parity(s_gpu, res.s, "f32")
    for g, o in zip(trace, res.trace):
        assert g[2] == pytest.approx(o[2], rel=2e-3)


# ---------------------------------------------------------------------------
# error handling
# ---------------------------------------------------------------------------

def _expect(gpu_lib, status, p, prec="f32", **kw):
    ctx = gpu_lib.Context(*p.d.shape, prec)
    sched = gpu_lib.Schedule(lambdas=[10.0, 1.0], rtol=0.0, max_sweeps=4, monitor_every=2, **kw)
    with pytest.raises(gpu_lib.WFError) as ei:
        ctx.solve(*_tensors(p, prec), schedule=sched)
    assert gpu_lib.STATUS[ei.value.status] == status


def test_error_codes(gpu_lib):
    p = synth.make_problem(64, 64, 1)
    q = synth.make_problem(64, 64, 1)
    q.d = q.d.copy()
    q.d[3, 4] = np.nan
    _expect(gpu_lib, "ENONFINITE", q)
    q = synth.make_problem(64, 64, 1)
    q.p_oof = np.zeros_like(q.p_oof)
    _expect(gpu_lib, "ENOTPD", q)
    q = synth.make_problem(64, 64, 1)
    q.mask = np.zeros((64, 64), np.uint8)
    _expect(gpu_lib, "EINVAL", q)
    _expect(gpu_lib, "ENOTPD", p, floor_frac=0.0)
    q = synth.make_problem(64, 64, 1)
    q.n_pix = q.n_pix.copy()
    q.n_pix[0, 0] = -1.0
    _expect(gpu_lib, "ENOTPD", q)
    q = synth.make_problem(64, 64, 1)
    q.s_k = q.s_k.copy()
    q.s_k[1, 1] = -1.0
    _expect(gpu_lib, "EINVAL", q)
    # spectra of real fields are even in k: k_y and -k_y of the real columns
    # k_x = 0 and nx/2 must agree, and the stripe spectrum must be even
    q = synth.make_problem(64, 64, 1)
    q.s_k = q.s_k.copy()
    q.s_k[3, 0] *= 1.5
    _expect(gpu_lib, "EINVAL", q)
    q = synth.make_problem(64, 64, 1)
    q.p_oof = q.p_oof.copy()
    q.p_oof[61, 32] *= 1.5
    _expect(gpu_lib, "EINVAL", q)
    q = synth.make_problem(64, 64, 1)
    q.p_stripe = q.p_stripe.copy()
    q.p_stripe[5] *= 2.0
    _expect(gpu_lib, "EINVAL", q)
    q = synth.make_problem(64, 64, 1)
    q.s_k = q.s_k.copy()
    q.s_k[3, 1] *= 1.5  # k_x = 1 is complex: no constraint
    s_ok, _, _, res = _run_both(gpu_lib, q, "f32", [10.0, 3.0, 1.0, 1.0], monitor_every=2)
    _assert_parity(s_ok, res.s, "f32")
    ctx = gpu_lib.Context(64, 64, "f32")
    with pytest.raises(gpu_lib.WFError):
        ctx.solve(*_tensors(p, "f32"), schedule=gpu_lib.Schedule(max_sweeps=0))
    with pytest.raises(gpu_lib.WFError) as ei:
        gpu_lib.Context(100, 64, "f32")
    assert gpu_lib.STATUS[ei.value.status] == "EUNSUPPORTED"


def test_masked_pixel_values_are_ignored(gpu_lib):
    p = synth.make_problem(64, 64, 6, mask_frac=0.1)
    ctx = gpu_lib.Context(64, 64, "f32")
    sched = gpu_lib.Schedule(lambdas=list(_ramp(10, 20)), rtol=0.0, max_sweeps=20, monitor_every=5)
    a, _, _ = ctx.solve(*_tensors(p, "f32"), schedule=sched)
    a = a.cpu().numpy().copy()
    q = synth.make_problem(64, 64, 6, mask_frac=0.1)
    q.d = np.where(q.mask == 0, np.nan, q.d)
    q.n_pix = np.where(q.mask == 0, -3.0, q.n_pix)
    b, _, _ = ctx.solve(*_tensors(q, "f32"), schedule=sched)
    np.testing.assert_array_equal(a, b.cpu().numpy())


def test_bitwise_deterministic(gpu_lib):
    p = synth.make_problem(256, 256, 3, mask_frac=0.1)
    ctx = gpu_lib.Context(256, 256, "f32")
    sched = gpu_lib.Schedule(lambda0=1e3, rtol=0.0, max_sweeps=64, monitor_every=8)
    a, ra, ta = ctx.solve(*_tensors(p, "f32"), schedule=sched)
    a = a.cpu().numpy().copy()
    b, rb, tb = ctx.solve(*_tensors(p, "f32"), schedule=sched)
    np.testing.assert_array_equal(a, b.cpu().numpy())
    np.testing.assert_array_equal(ta, tb)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_unaligned_inputs_give_identical_results(gpu_lib, prec):
    """The set-up passes read the caller's per-pixel arrays four values at a
    time with vector loads when the pointers allow it, else one by one in the
    same order: d and N_pix one element, and the mask one byte, past an
    aligned address give the same solve bit for bit."""
    import torch
    p = synth.make_problem(256, 128, 5, mask_frac=0.1)
    args = _tensors(p, prec)
    d, sk, npix, poof, pst, mask = args

    def shifted(t):
        buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=t.device)
        v = buf[1:].view(t.shape)
        v.copy_(t)
        return v
    un = (shifted(d), sk, shifted(npix), poof, pst, shifted(mask))
    esz = 4 if prec == "f32" else 8
    assert un[0].data_ptr() % (4 * esz) != 0 and un[5].data_ptr() % 4 != 0
    ctx = gpu_lib.Context(256, 128, prec)
    sched = gpu_lib.Schedule(lambdas=[1e3, 300.0, 100.0, 30.0, 10.0, 3.0, 1.0, 1.0], rtol=0.0,
                             max_sweeps=8, monitor_every=4)
    a, ra, ta = ctx.solve(*args, schedule=sched)
    a = a.cpu().numpy().copy()
    b, rb, tb = ctx.solve(*un, schedule=sched)
    np.testing.assert_array_equal(a, b.cpu().numpy())
    np.testing.assert_array_equal(ta, tb)
    assert ra["d2"] == rb["d2"]


@pytest.mark.parametrize("shape", [(2048, 2048), (1536, 768), (256, 256)])
def test_tilings_give_identical_results(gpu_lib, shape):
    """Every transit-buffer tiling only moves data differently, so all of
    them must give bit-identical sweeps (float32; the tuned lengths)."""
    ny, nx = shape
    p = synth.named_config("c3") if shape == (2048, 2048) else synth.make_problem(ny, nx, 24,
                                                                                   mask_frac=0.1)
    ctx = gpu_lib.Context(ny, nx, "f32")
    args = _tensors(p, "f32")
    sched = gpu_lib.Schedule(lambdas=[1e4, 3e3, 1e3, 300.0, 100.0, 30.0], rtol=0.0,
                             max_sweeps=6, monitor_every=3)
    ref = None
    n_built = 0
    for tile in range(gpu_lib.load().wf_tile_count()):
        if not ctx.set_tile(tile):
            continue
        n_built += 1
        print(f"tiling {tile}", flush=True)
        s, rep, trace = ctx.solve(*args, schedule=sched)
        s = s.cpu().numpy().copy()
        if ref is None:
            ref = (s, trace)
        else:
            np.testing.assert_array_equal(s, ref[0])
            np.testing.assert_array_equal(trace[:, :5], ref[1][:, :5])
            # the joint objective's block partials follow the tiling, so
            # only their summation order differs
            np.testing.assert_allclose(trace[:, 5], ref[1][:, 5], rtol=1e-12)
    assert n_built >= 2


def test_autotuner_times_every_built_tiling_and_keeps_the_fastest(gpu_lib):
    p = synth.make_problem(768, 1536, 25, mask_frac=0.1)
    ctx = gpu_lib.Context(768, 1536, "f32")
    args = _tensors(p, "f32")
    times = ctx.autotune(*args, sweeps=16)
    print("  tilings:", {k: round(v, 3) for k, v in times.items()}, flush=True)
    assert len(times) == gpu_lib.load().wf_tile_count()  # all built at these lengths
    assert ctx.tile == min(times, key=times.get)
    ctx64 = gpu_lib.Context(256, 256, "f64")
    q = synth.make_problem(256, 256, 26)
    t64 = ctx64.autotune(*_tensors(q, "f64"), sweeps=8)
    assert list(t64) == [1] and ctx64.tile == 1  # float64: the default tiling only
    # the tuned context still matches the oracle
    lams = list(_ramp(10, 20))
    s_gpu, rep, trace = ctx.solve(*args, schedule=gpu_lib.Schedule(
        lambdas=lams, rtol=0.0, max_sweeps=20, monitor_every=8))
    res = oracle.solve(p, oracle.FixedSchedule(lams), max_sweeps=20, monitor_every=8)
    _assert_parity(s_gpu.cpu().numpy().astype(np.float64), res.s, "f32")


def test_converged_c2_field_matches_converged_oracle(gpu_lib):
    """C2 (512^2, three terms, no mask): the GPU's float64 augmented solve
    and the oracle's, each from zero with the same adaptive schedule
    (lambda^0.97 from 1e4) to rho <= 1e-9, element by element.  The bar is
    the oracle's own distance from its 1e-11 solution on this map (9.2e-10
    relative L2, 2.3e-8 of the largest value), with headroom."""
    oracle.bases.set_workers(16)
    p = synth.named_config("c2")
    ctx = gpu_lib.Context(512, 512, "f64")
    sched = gpu_lib.Schedule(lambda0=1e4, shrink=0.97, rtol=1e-9, max_sweeps=60000,
                             monitor_every=16, chain="augmented")
    s_gpu, rep, trace = ctx.solve(*_tensors(p, "f64"), schedule=sched)
    assert rep["status"] == "OK"
    s_gpu = s_gpu.cpu().numpy()
    print(f"  GPU: {rep['sweeps']} sweeps, rho {rep['rho']:.3e}; oracle solve", flush=True)
    res = oracle.solve(p, oracle.AdaptiveSchedule(lam0=1e4, shrink=0.97),
                       settings=oracle.Settings(chain="augmented"), max_sweeps=60000,
                       monitor_every=16, rtol=1e-9)
    assert res.converged
    err = _rel(s_gpu, res.s)
    emax = float(np.max(np.abs(s_gpu - res.s)) / np.max(np.abs(res.s)))
    print(f"  oracle {res.sweeps} sweeps; rel L2 {err:.2e}, max {emax:.2e}", flush=True)
    assert err < 3e-9
    assert emax < 6e-8


@pytest.mark.parametrize("cfg,prec,bound", [("c2", "f64", 1.0e-6), ("c3", "f64", 1.0e-6),
                                            ("c2", "f32", 3.0e-5)])
def test_converged_residual_checked_by_oracle(gpu_lib, cfg, prec, bound):
    """Full-size zero-start solves (C2 512^2; C3 2048^2 with its mask): the
    oracle evaluates Section 2's residual of the GPU's converged field itself
    (augmented chain, field mode 1: u = (S + N_F) x, so x follows without
    dividing by the signal spectrum).  float64 meets rho <= 1e-6; float32
    stops at its rounding floor (about 1e-5 here)."""
    import torch
    p = synth.named_config(cfg)
    ny, nx = p.d.shape
    print(f"converged residual {cfg} {prec}", flush=True)
    ctx = gpu_lib.Context(ny, nx, prec)
    sched = gpu_lib.Schedule(lambda0=1e6, rtol=1e-6, max_sweeps=60000 if prec == "f64" else 20000,
                             monitor_every=16, chain="augmented", chain_field=True)
    u, rep, _ = ctx.solve(*_tensors(p, prec), schedule=sched)
    if prec == "f64":
        assert rep["status"] == "OK"
    st = oracle.setup(p, oracle.Settings(chain="augmented"))
    dg = oracle.diagnostics_of_field(st, u.cpu().numpy().astype(np.float64))
    assert dg.rho <= bound * (1 + 1e-6)
    if prec == "f64":
        assert dg.rho == pytest.approx(rep["rho"], rel=1e-6)
        assert dg.rho_mask == pytest.approx(rep["rho_mask"], rel=1e-6, abs=1e-15)
