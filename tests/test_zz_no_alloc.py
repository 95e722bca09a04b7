"""wf_solve_noalloc (workspace in the library's static device scratch)
against wf_solve with a context of the default tiling: same kernels, so the
results, reports and traces must agree bit for bit.  Two calls in a row on
one GPU, the second on a smaller map, so the second runs on what the first
left in the scratch."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _tensors(p, prec):
    import torch
    dt = torch.float32 if prec == "f32" else torch.float64

    def t(a):
        return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    mask = None if p.mask is None else torch.tensor(p.mask, dtype=torch.uint8, device="cuda")
    return t(p.d), t(p.s_k), t(p.n_pix), t(p.p_oof), t(p.p_stripe), mask


def _both(gpu_lib, p, prec, sched, s_init=None):
    ny, nx = p.d.shape
    print(f"no-alloc {prec} {ny}x{nx} chain={sched.chain} sweeps<={sched.max_sweeps}", flush=True)
    args = _tensors(p, prec)
    a, ra, ta = gpu_lib.solve_noalloc(*args, schedule=sched, s_init=s_init)
    ctx = gpu_lib.Context(ny, nx, prec)
    b, rb, tb = ctx.solve(*args, schedule=sched, s_init=s_init)
    ctx.close()
    return a.cpu().numpy(), ra, ta, b.cpu().numpy(), rb, tb


def _same(ra, rb):
    for key in ("status", "sweeps", "n_records", "lam", "rho", "rho_mask", "dd2", "d2",
                "chi2_joint", "masked_x_norm", "tau", "phi"):
        assert ra[key] == rb[key], key


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_solve_two_calls_second_smaller(gpu_lib, prec):
    lams = [1e3 * 0.8 ** k for k in range(30)] + [1.0] * 10
    big = synth.make_problem(256, 256, 41, mask_frac=0.08)
    sched = gpu_lib.Schedule(lambdas=lams, rtol=0.0, max_sweeps=len(lams), monitor_every=8)
    a, ra, ta, b, rb, tb = _both(gpu_lib, big, prec, sched)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ta, tb)
    _same(ra, rb)
    # second call, smaller map, adaptive schedule with an early stop (the
    # host checks the device schedule every few chunks); float32 fields
    # settle at a residual of about 1e-5, hence its looser target
    small = synth.make_problem(128, 256, 42, mask_frac=0.05)
    sched = gpu_lib.Schedule(lambda0=1e3, shrink=0.9, rtol=1e-4 if prec == "f32" else 1e-6,
                             max_sweeps=20000, monitor_every=8, chain="augmented")
    a, ra, ta, b, rb, tb = _both(gpu_lib, small, prec, sched)
    assert ra["status"] == "OK" and ra["sweeps"] < 20000
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ta, tb)
    _same(ra, rb)


def test_noalloc_warm_start_and_limit(gpu_lib):
    import torch
    p = synth.make_problem(64, 128, 43, mask_frac=0.1)
    s0 = torch.tensor(p.s_true, dtype=torch.float32, device="cuda")
    sched = gpu_lib.Schedule(lambdas=[50.0, 20.0, 5.0, 1.0], rtol=0.0, max_sweeps=9,
                             monitor_every=4)
    a, ra, ta, b, rb, tb = _both(gpu_lib, p, "f32", sched, s_init=s0)
    np.testing.assert_array_equal(a, b)
    _same(ra, rb)
    q = synth.make_problem(1024, 1024, 44)
    with pytest.raises(gpu_lib.WFError) as e:
        gpu_lib.solve_noalloc(*_tensors(q, "f32"), schedule=sched)
    assert e.value.status == -7
