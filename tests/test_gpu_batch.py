"""Batched solves (many maps, shared launches, one chunk replayed as a HIP
graph) against per-map solves and the CPU float64 oracle.

A map in a batch runs the same kernels with the same arguments as a map solved
alone, so its result must be bitwise identical to the single solve; the single
solves are themselves held to the oracle by the parity tests, and a few batch
members are compared with the oracle directly here as well.
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

from parity_checks import TOL, assert_parity


def _dict(p, prec):
    import torch
    dt = torch.float32 if prec == "f32" else torch.float64

    def t(a):
        return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    out = dict(d=t(p.d), s_k=t(p.s_k), n_pix=t(p.n_pix), p_oof=t(p.p_oof),
               p_stripe=t(p.p_stripe))
    if p.mask is not None:
        out["mask"] = torch.tensor(p.mask, dtype=torch.uint8, device="cuda")
    return out


def _single(gpu_lib, p, prec, sched):
    ny, nx = p.d.shape
    ctx = gpu_lib.Context(ny, nx, prec)
    pb = _dict(p, prec)
    s, rep, _ = ctx.solve(pb["d"], pb["s_k"], pb["n_pix"], pb["p_oof"], pb["p_stripe"],
                          pb.get("mask"), schedule=sched)
    return s.cpu().numpy(), rep


def _batch(gpu_lib, probs, prec, sched):
    ctxs = [gpu_lib.Context(p.d.shape[0], p.d.shape[1], prec) for p in probs]
    outs, reps = gpu_lib.solve_batch(ctxs, [_dict(p, prec) for p in probs], schedule=sched)
    return [o.cpu().numpy() for o in outs], reps


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _mixed_problems():
    # three shapes (one with a factor 3), mixed masks and noise terms, so the
    # batch has several shape classes and several chain kinds per shape
    return [
        synth.make_problem(64, 64, 31),
        synth.make_problem(64, 64, 32, mask_frac=0.1),
        synth.make_problem(64, 64, 33, stripe_rms=None),
        synth.make_problem(128, 64, 34, mask_frac=0.05),
        synth.make_problem(384, 128, 35, oof_level=None),
        synth.make_problem(64, 64, 36, oof_level=None, stripe_rms=None),
        synth.make_problem(128, 64, 37),
    ]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("chain", ["three", "augmented"])
def test_batch_fixed_schedule_matches_single_and_oracle(gpu_lib, prec, chain):
    probs = _mixed_problems()
    lams = list(oracle.cooling_ramp(14, 27, 300.0))
    print(f"batch fixed {prec} {chain} maps={len(probs)}", flush=True)
    sched = gpu_lib.Schedule(lambdas=lams, rtol=0.0, max_sweeps=len(lams), monitor_every=4,
                             chain=chain)
    outs, reps = _batch(gpu_lib, probs, prec, sched)
    for i, p in enumerate(probs):
        s1, rep1 = _single(gpu_lib, p, prec, sched)
        assert reps[i]["sweeps"] == len(lams) and rep1["sweeps"] == len(lams)
        assert np.array_equal(outs[i], s1), i
        assert reps[i]["rho"] == rep1["rho"]
    for i in (1, 4):
        res = oracle.solve(probs[i], oracle.FixedSchedule(lams),
                           settings=oracle.Settings(chain=chain), max_sweeps=len(lams),
                           monitor_every=4)
        assert_parity(outs[i].astype(np.float64), res.s, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_adaptive_each_map_stops_on_its_own(gpu_lib, prec):
    """Adaptive schedule with a residual target: every map keeps its own
    controller, so sweeps, final lambda and result equal its single solve."""
    probs = [synth.make_problem(64, 64, 41),
             synth.make_problem(64, 64, 42, white_sigma=3.0),
             synth.make_problem(128, 64, 43, mask_frac=0.1)]
    print(f"batch adaptive {prec}", flush=True)
    sched = gpu_lib.Schedule(lambda0=1e3, rtol=3e-4,
                             max_sweeps=4000, monitor_every=8, chain="augmented")
    outs, reps = _batch(gpu_lib, probs, prec, sched)
    sweeps = []
    for i, p in enumerate(probs):
        s1, rep1 = _single(gpu_lib, p, prec, sched)
        assert reps[i]["status"] == rep1["status"] == "OK"
        assert reps[i]["sweeps"] == rep1["sweeps"]
        assert reps[i]["lam"] == rep1["lam"]
        assert np.array_equal(outs[i], s1), i
        sweeps.append(reps[i]["sweeps"])
    assert len(set(sweeps)) > 1  # the maps did stop at different sweeps


def test_batch_of_one_equals_solve(gpu_lib):
    p = synth.make_problem(64, 128, 51, mask_frac=0.05)
    sched = gpu_lib.Schedule(lambdas=list(oracle.cooling_ramp(6, 11, 100.0)), rtol=0.0,
                             max_sweeps=11, monitor_every=3)
    outs, reps = _batch(gpu_lib, [p], "f64", sched)
    s1, rep1 = _single(gpu_lib, p, "f64", sched)
    assert np.array_equal(outs[0], s1)
    assert reps[0]["sweeps"] == 11 and reps[0]["n_records"] == rep1["n_records"]


def test_batch_errors(gpu_lib):
    import torch
    p = synth.make_problem(64, 64, 61)
    q = synth.make_problem(64, 64, 62)
    sched = gpu_lib.Schedule(lambdas=[10.0, 1.0], rtol=0.0, max_sweeps=2, monitor_every=1)
    c1 = gpu_lib.Context(64, 64, "f32")
    c2 = gpu_lib.Context(64, 64, "f32")
    c3 = gpu_lib.Context(64, 64, "f64")
    # the same context twice
    with pytest.raises(gpu_lib.WFError) as e:
        gpu_lib.solve_batch([c1, c1], [_dict(p, "f32"), _dict(q, "f32")], schedule=sched)
    assert e.value.status == -1
    # mixed precision
    with pytest.raises(gpu_lib.WFError) as e:
        gpu_lib.solve_batch([c1, c3], [_dict(p, "f32"), _dict(q, "f64")], schedule=sched)
    assert e.value.status == -1
    # a non-finite observed pixel in the second map
    bad = _dict(q, "f32")
    bad["d"][3, 5] = float("nan")
    with pytest.raises(gpu_lib.WFError) as e:
        gpu_lib.solve_batch([c1, c2], [_dict(p, "f32"), bad], schedule=sched)
    assert e.value.status == -3
    # contexts are still usable afterwards
    outs, reps = gpu_lib.solve_batch([c1, c2], [_dict(p, "f32"), _dict(q, "f32")],
                                     schedule=sched)
    assert all(r["sweeps"] == 2 for r in reps)
    torch.cuda.synchronize()


def test_uneven_batch_shapes(gpu_lib):
    """48 maps of three sizes (16 each of 256^2, 768^2, 1536^2) in one batch:
    every map equals its single solve bit for bit (sampled), and a 256^2 map
    matches the oracle."""
    sizes = [256] * 16 + [768] * 16 + [1536] * 16
    probs = [synth.make_problem(n, n, 700 + i, mask_frac=0.05) for i, n in enumerate(sizes)]
    lams = list(oracle.cooling_ramp(8, 16, 300.0))
    sched = gpu_lib.Schedule(lambdas=lams, rtol=0.0, max_sweeps=len(lams), monitor_every=8)
    print("uneven batch 48 maps", flush=True)
    outs, reps = _batch(gpu_lib, probs, "f32", sched)
    assert all(r["sweeps"] == len(lams) for r in reps)
    for i in (0, 15, 16, 31, 32, 47):
        s1, _ = _single(gpu_lib, probs[i], "f32", sched)
        assert np.array_equal(outs[i], s1), i
    res = oracle.solve(probs[3], oracle.FixedSchedule(lams), max_sweeps=len(lams),
                       monitor_every=8)
    assert_parity(outs[3].astype(np.float64), res.s, "f32")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_warm_starts_match_single(gpu_lib, prec):
    """Per-map warm starts (one entry None) give the single solves' results."""
    import torch
    probs = [synth.make_problem(64, 64, 81, mask_frac=0.1), synth.make_problem(64, 64, 82),
             synth.make_problem(128, 64, 83)]
    dt = torch.float32 if prec == "f32" else torch.float64
    inits = [torch.tensor(probs[0].s_true, dtype=dt, device="cuda"), None,
             torch.tensor(0.5 * probs[2].s_true, dtype=dt, device="cuda")]
    sched = gpu_lib.Schedule(lambdas=list(oracle.cooling_ramp(6, 12, 50.0)), rtol=0.0,
                             max_sweeps=12, monitor_every=4, chain="augmented")
    ctxs = [gpu_lib.Context(p.d.shape[0], p.d.shape[1], prec) for p in probs]
    outs, reps = gpu_lib.solve_batch(ctxs, [_dict(p, prec) for p in probs], schedule=sched,
                                     s_inits=inits)
    for i, p in enumerate(probs):
        ny, nx = p.d.shape
        ctx = gpu_lib.Context(ny, nx, prec)
        pb = _dict(p, prec)
        s1, _, _ = ctx.solve(pb["d"], pb["s_k"], pb["n_pix"], pb["p_oof"], pb["p_stripe"],
                             pb.get("mask"), schedule=sched, s_init=inits[i])
        assert torch.equal(outs[i], s1), i


def test_batch_autotuner_tunes_each_shape_on_its_batch(gpu_lib):
    """wf_autotune_batch: for each shape, every built tiling is timed on a
    batched probe of that shape's maps and their contexts keep the fastest;
    the batch solved afterwards equals the same batch in the default tiling
    bit for bit (a tiling moves data, it does not change the arithmetic)."""
    import torch
    sizes = [256, 256, 256, 768, 768]
    probs = [synth.make_problem(n, n, 900 + i, mask_frac=0.05) for i, n in enumerate(sizes)]
    pbs = [_dict(p, "f32") for p in probs]
    ctxs = [gpu_lib.Context(n, n, "f32") for n in sizes]
    print("batch autotune 3 x 256^2 + 2 x 768^2", flush=True)
    res = gpu_lib.autotune_batch(ctxs, pbs, sweeps=16)
    nt = gpu_lib.load().wf_tile_count()
    assert set(res) == {(256, 256), (768, 768)}
    for (ny, nx), (chosen, times) in res.items():
        print(f"  {ny}x{nx}: tiling {chosen}", {k: round(v, 3) for k, v in times.items()},
              flush=True)
        assert len(times) == nt  # every tiling is built at these lengths
        assert chosen == min(times, key=times.get)
        assert all(c.tile == chosen for c in ctxs if (c.ny, c.nx) == (ny, nx))
    sched = gpu_lib.Schedule(lambdas=list(oracle.cooling_ramp(6, 12, 300.0)), rtol=0.0,
                             max_sweeps=12, monitor_every=4)
    outs, _ = gpu_lib.solve_batch(ctxs, pbs, schedule=sched)
    ref_ctxs = [gpu_lib.Context(n, n, "f32") for n in sizes]
    ref, _ = gpu_lib.solve_batch(ref_ctxs, pbs, schedule=sched)
    for i, (a, b) in enumerate(zip(outs, ref)):
        assert torch.equal(a, b), i
    # float64 contexts: the default tiling is the only one built
    c64 = [gpu_lib.Context(64, 64, "f64") for _ in range(2)]
    q = [_dict(synth.make_problem(64, 64, 910 + i), "f64") for i in range(2)]
    r64 = gpu_lib.autotune_batch(c64, q, sweeps=4)
    assert list(r64) == [(64, 64)] and r64[(64, 64)][0] == 1 and list(r64[(64, 64)][1]) == [1]


def test_batch_autotuner_error_keeps_tilings(gpu_lib):
    """A map whose data hold a NaN on an observed pixel: wf_autotune_batch
    returns the solve's error (WF_ENONFINITE) and the group's contexts keep
    the tiling they had."""
    import torch
    probs = [synth.make_problem(256, 256, 920 + i) for i in range(2)]
    pbs = [_dict(p, "f32") for p in probs]
    pbs[1]["d"][7, 9] = float("nan")
    ctxs = [gpu_lib.Context(256, 256, "f32") for _ in probs]
    for c in ctxs:
        assert c.set_tile(6)
    with pytest.raises(gpu_lib.WFError) as e:
        gpu_lib.autotune_batch(ctxs, pbs, sweeps=4)
    assert e.value.status == -3
    assert all(c.tile == 6 for c in ctxs)
    torch.cuda.synchronize()
