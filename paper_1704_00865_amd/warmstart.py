"""Learned warm start: training data from the solver, training, and the
sweeps-to-residual comparison with the zero start.

The network predicts the chain's signal-end field of the augmented chain,
u = (S + N_F) x with x = S^-1 s (the signal plus the Fourier-diagonal noise
the filter attributes to the data), and the solve starts from it with
field_mode 1: the messenger then starts consistent with u, which a signal
estimate alone cannot give (a start from s leaves the messenger's noise part
to be rebuilt over many sweeps).

Orchestration only (Python loops over batches); the solves, the network's
forward and backward passes and the optimiser run in the library's kernels.
"""

from __future__ import annotations

import time
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from . import Context, Schedule, solve_batch
from .nn import WarmNet, init_params


@dataclass
class MapSet:
    """Stacked maps of one size on the device: d, n_pix, mask [n, h, w] and,
    for training, the solver's Wiener solutions s."""
    d: object
    n_pix: object
    mask: object
    s: object = None

    @property
    def n(self) -> int:
        return int(self.d.shape[0])


def stack_problems(problems, precision: str = "f64", device="cuda") -> MapSet:
    import torch
    dt = torch.float64 if precision == "f64" else torch.float32
    d = torch.tensor(np.stack([p.d for p in problems]), dtype=dt, device=device)
    npix = torch.tensor(np.stack([p.n_pix for p in problems]), dtype=dt, device=device)
    h, w = problems[0].d.shape
    m = np.stack([p.mask if p.mask is not None else np.ones((h, w), np.uint8) for p in problems])
    mask = torch.tensor(m, dtype=torch.uint8, device=device)
    return MapSet(d, npix, mask)


def _inputs(problems, ms: MapSet, i: int):
    import torch
    p = problems[i]
    dt = ms.d.dtype
    dev = ms.d.device

    def t(a):
        return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    return dict(d=ms.d[i], s_k=t(p.s_k), n_pix=ms.n_pix[i], p_oof=t(p.p_oof),
                p_stripe=t(p.p_stripe), mask=ms.mask[i])


def solve_set(problems, ms: MapSet, schedule: Schedule, s_init=None, group: int = 64, log=None):
    """Solve every map of the set with one schedule in batches of ``group``
    maps, from zero or from the warm starts s_init [n, h, w].  Each map
    stops on its own.  Returns (solutions [n, h, w], list of reports)."""
    import torch
    n = ms.n
    h, w = ms.d.shape[1:]
    prec = "f64" if ms.d.dtype == torch.float64 else "f32"
    out = torch.empty_like(ms.d)
    reps = []
    ctxs = [Context(h, w, prec, device=ms.d.device) for _ in range(min(group, n))]
    for g0 in range(0, n, group):
        idx = list(range(g0, min(n, g0 + group)))
        _, r = solve_batch(ctxs[:len(idx)], [_inputs(problems, ms, i) for i in idx],
                           schedule=schedule, outs=[out[i] for i in idx],
                           s_inits=None if s_init is None else [s_init[i] for i in idx])
        reps += r
        if log and n > group:
            log(f"solved {len(reps)}/{n} maps")
    for c in ctxs:
        c.close()
    return out, reps


def train(net: WarmNet, data: MapSet, *, epochs: int, batch: int, lr: float, seed: int = 0,
          lr_final: float | None = None, log=None) -> List[float]:
    """Adam over shuffled mini-batches; the learning rate decays
    geometrically from lr to lr_final over the run.  Returns the mean loss
    of each epoch."""
    import torch
    rng = np.random.default_rng(seed)
    n = data.n
    steps = epochs * (n // batch)
    lr_final = lr if lr_final is None else lr_final
    k = 0
    hist = []
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(n), device=data.d.device)
        tot = 0.0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            cur = lr * (lr_final / lr) ** (k / max(steps - 1, 1))
            tot += net.train_step(data.d[idx].contiguous(), data.n_pix[idx].contiguous(),
                                  data.mask[idx].contiguous(), data.s[idx].contiguous(), cur)
            k += 1
        hist.append(tot / max(n // batch, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.4e}")
    return hist


def conv_flops_per_step(h: int, w: int, batch: int) -> dict:
    """Multiply-add work of one training step (forward, input adjoint and
    weight gradient of every convolution; the first layer's input adjoint is
    not needed), counting 2 flops per multiply-add.  'executed' uses the
    stored channel counts (input 4 -> 32, output 1 -> 32), 'useful' the real
    ones."""
    from .nn import CHANNELS, layer_shapes
    shapes = layer_shapes()
    L = len(CHANNELS)
    levels = [0, 0]
    for l in range(1, L):
        levels += [l, l]
    for l in range(L - 2, -1, -1):
        levels += [l, l]
    levels.append(0)
    ex = us = 0.0
    for i, ((ci, co), lev) in enumerate(zip(shapes, levels)):
        P = batch * (h >> lev) * (w >> lev)
        cr = 4 if i == 0 else ci
        orr = 1 if i == len(shapes) - 1 else co
        passes = 2 if i == 0 else 3
        ex += passes * 2.0 * 9 * ci * co * P
        us += passes * 2.0 * 9 * cr * orr * P
    return {"executed": ex, "useful": us}


def predict(net: WarmNet, data: MapSet, batch: int):
    import torch
    out = torch.empty_like(data.d)
    for b0 in range(0, data.n, batch):
        sl = slice(b0, min(data.n, b0 + batch))
        net.predict(data.d[sl].contiguous(), data.n_pix[sl].contiguous(), data.mask[sl].contiguous(),
                    out=out[sl])
    return out


def rel_error(a, b) -> np.ndarray:
    """Per-map relative L2 error |a - b| / |b|."""
    import torch
    num = torch.linalg.vector_norm((a - b).double(), dim=(1, 2))
    den = torch.linalg.vector_norm(b.double(), dim=(1, 2))
    return (num / den).cpu().numpy()


def _seeds(problems):
    return [p.meta.get("seed") for p in problems if getattr(p, "meta", None)]


def _seed_range(problems):
    sd = _seeds(problems)
    return [min(sd), max(sd)] if sd else None


def experiment(train_problems: Sequence, test_problems: Sequence, *, precision: str = "f64",
               target_rtol: float = 1e-5, eval_rtol: float = 1e-6, lam0: float = 1e4,
               shrink: float = 0.97, warm_lam0: Sequence[float] = (1e3, 1e2, 10.0),
               epochs: int = 20, batch: int = 16,
               lr: float = 2e-3, seed: int = 0, max_sweeps: int = 200000,
               target_precision: str | None = None, target_lam0: float | None = None,
               target_shrink: float | None = None, log=None) -> dict:
    """Train on solver solutions (chain fields u) of train_problems and
    compare sweeps to rho <= eval_rtol on test_problems from the zero start
    and from the network's prediction (for each lambda0 in warm_lam0), with
    the converged field as a warm start for reference.  Augmented chain.

    The training targets may be solved in another precision and schedule
    (target_*; the network is then trained and run in that precision and its
    prediction converted).  The test maps must be held out: a seed shared
    with the training maps raises ValueError."""
    import torch
    shared = set(_seeds(train_problems)) & set(_seeds(test_problems))
    if shared:
        raise ValueError(f"test maps share seeds with the training maps: {sorted(shared)[:8]}")
    tprec = precision if target_precision is None else target_precision
    h, w = train_problems[0].d.shape
    t0 = time.perf_counter()
    tr = stack_problems(train_problems, tprec)
    te = stack_problems(test_problems, precision)
    tsched = Schedule(lambda0=lam0 if target_lam0 is None else target_lam0,
                      shrink=shrink if target_shrink is None else target_shrink,
                      rtol=target_rtol, max_sweeps=max_sweeps,
                      monitor_every=16, chain="augmented", chain_field=True)
    tr.s, rtr = solve_set(train_problems, tr, tsched, log=log)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    if log:
        log(f"training targets: {tr.n} solves in {t_gen:.1f} s, "
            f"{np.mean([r['sweeps'] for r in rtr]):.0f} sweeps each")
    net = WarmNet(h, w, batch_max=max(batch, 8), precision=tprec)
    net.set_params(init_params(seed))
    t1 = time.perf_counter()
    hist = train(net, tr, epochs=epochs, batch=batch, lr=lr, lr_final=lr * 0.05, seed=seed, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    steps = epochs * (tr.n // batch)
    tr = None  # the training set is no longer needed
    # reference solutions of the test maps and the predictions
    esched = Schedule(lambda0=lam0, shrink=shrink, rtol=eval_rtol, max_sweeps=max_sweeps,
                      monitor_every=16, chain="augmented", chain_field=True)
    t2 = time.perf_counter()
    s_ref, rzero = solve_set(test_problems, te, esched, log=log)
    torch.cuda.synchronize()
    t_zero = time.perf_counter() - t2
    t_p = time.perf_counter()
    if tprec == precision:
        pred = predict(net, te, max(batch, 8))
    else:
        nd = torch.float32 if tprec == "f32" else torch.float64
        pred = predict(net, MapSet(te.d.to(nd), te.n_pix.to(nd), te.mask), max(batch, 8))
        pred = pred.to(te.d.dtype)
    torch.cuda.synchronize()
    t_pred = time.perf_counter() - t_p
    err_pred = rel_error(pred, s_ref)
    err_zero = np.ones(te.n)
    e = (pred - s_ref).double()
    row = e.mean(dim=2, keepdim=True).expand_as(e)
    frac_rows = float((row.pow(2).sum() / e.pow(2).sum()).item())
    res = {"maps_train": len(train_problems), "maps_test": te.n, "map": [h, w],
           "dtype": precision, "target_dtype": tprec,
           "held_out": {"train_seeds": _seed_range(train_problems),
                        "test_seeds": _seed_range(test_problems), "shared_seeds": 0},
           "chain": "augmented", "eval_rtol": eval_rtol, "target_rtol": target_rtol,
           "target_sweeps_mean": float(np.mean([r["sweeps"] for r in rtr])),
           "gen_seconds": round(t_gen, 2), "train_seconds": round(t_train, 2), "train_steps": steps,
           "train_batch": batch, "epochs": epochs, "loss_first_epoch": hist[0],
           "train_step_ms": round(1e3 * t_train / max(steps, 1), 3),
           "train_tflops_executed": round(conv_flops_per_step(h, w, batch)["executed"] * steps
                                          / t_train / 1e12, 2),
           "train_mfma_frac_bf16": round(conv_flops_per_step(h, w, batch)["executed"] * steps
                                         / t_train / 2.5e15, 4),
           "loss_last_epoch": hist[-1],
           "pred_rel_error_median": float(np.median(err_pred)),
           "pred_error_energy_in_row_means": frac_rows,
           "shrink": shrink,
           "zero": {"lambda0": lam0, "sweeps_mean": float(np.mean([r["sweeps"] for r in rzero])),
                    "seconds": round(t_zero, 2),
                    "converged": int(sum(r["status"] == "OK" for r in rzero)),
                    "rel_error_start_median": float(np.median(err_zero))},
           "warm": []}
    for l0 in warm_lam0:
        sch = Schedule(lambda0=l0, shrink=shrink, rtol=eval_rtol, max_sweeps=max_sweeps,
                       monitor_every=16, chain="augmented", chain_field=True)
        t3 = time.perf_counter()
        _, rw = solve_set(test_problems, te, sch, s_init=pred, log=log)
        torch.cuda.synchronize()
        ratio = [a["sweeps"] / max(b["sweeps"], 1) for a, b in zip(rzero, rw)]
        res["warm"].append({"lambda0": l0,
                            "sweeps_mean": float(np.mean([r["sweeps"] for r in rw])),
                            "converged": int(sum(r["status"] == "OK" for r in rw)),
                            "seconds": round(time.perf_counter() - t3, 2),
                            "sweeps_ratio_per_map_median": float(np.median(ratio))})
        if log:
            log(f"warm lambda0={l0:g}: network {res['warm'][-1]['sweeps_mean']:.0f} sweeps, "
                f"zero start {res['zero']['sweeps_mean']:.0f}")
    # reference: the converged field itself as the start, at lambda = 1
    sch = Schedule(lambda0=1.0, shrink=shrink, rtol=eval_rtol, max_sweeps=max_sweeps,
                   monitor_every=16, chain="augmented", chain_field=True)
    _, rx = solve_set(test_problems, te, sch, s_init=s_ref, log=log)
    res["exact_start"] = {"lambda0": 1.0, "sweeps_mean": float(np.mean([r["sweeps"] for r in rx]))}
    best = min(res["warm"], key=lambda r: (-r["converged"], r["sweeps_mean"]))
    res["best_warm_lambda0"] = best["lambda0"]
    res["speedup_sweeps"] = res["zero"]["sweeps_mean"] / max(best["sweeps_mean"], 1.0)
    # wall time of the test set from either start, the network's inference
    # counted on its side
    res["predict_seconds"] = round(t_pred, 4)
    res["speedup_wall"] = res["zero"]["seconds"] / max(res["predict_seconds"] + best["seconds"],
                                                       1e-9)
    res["default_start"] = "network" if res["speedup_wall"] > 1.0 else "zero"
    net.close()
    return res
