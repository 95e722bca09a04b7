"""Warm-start network kernels (bfloat16 matrix-core convolutions, float32
accumulation) against the float64 oracle (oracle.warmnet) on identical
bfloat16-representable inputs.

Tolerances follow from the arithmetic: a bfloat16 result carries a relative
rounding error of at most 2^-9 per element, products of bfloat16 values are
exact in float32 and float32 sums over at most ~10^5 terms add ~1e-6.
  * one convolution with a bfloat16 output: relative L2 <= 4e-3 (2^-8);
  * the weight gradient (float32 output): relative L2 <= 1e-5;
  * the whole network: 14 rounded intermediate activations, <= 14 * 2^-9,
    so 3e-2; its gradient passes ~3 rounded tensors per layer, bound 5e-2.
"""

import numpy as np
import pytest

from oracle import warmnet as wn

pytestmark = pytest.mark.gpu

CH = (32, 64, 96, 128)


def _bf16(shape, seed, scale=1.0):
    import torch
    g = torch.Generator().manual_seed(seed)
    return (torch.randn(shape, generator=g) * scale).to(torch.bfloat16).cuda()


def _np(t):
    import torch
    return t.to(torch.float64).cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("ci,co", [(32, 32), (64, 96), (96, 128), (128, 64)])
@pytest.mark.parametrize("relu", [False, True])
def test_conv_forward(gpu_lib, ci, co, relu):
    import torch
    from paper_1704_00865_amd import nn
    print(f"conv fwd {ci}->{co} relu={relu}", flush=True)
    x = _bf16((2, 16, 32, ci), 1)
    w = _bf16((3, 3, ci, co), 2, 0.1)
    b = torch.randn(co, generator=torch.Generator().manual_seed(3)).float().cuda()
    out = nn.conv3x3(1 if relu else 0, x, w, b, ci=ci, co=co)
    ref = wn.conv3x3(_np(x), _np(w), b.double().cpu().numpy())
    if relu:
        ref = np.maximum(ref, 0)
    got = _np(out)
    assert _rel(got, ref) < 4e-3
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-3 * np.sqrt(np.mean(ref ** 2)))


@pytest.mark.parametrize("ci,co", [(32, 64), (96, 32), (128, 128)])
def test_conv_input_adjoint(gpu_lib, ci, co):
    from paper_1704_00865_amd import nn
    print(f"conv dgrad {ci}<-{co}", flush=True)
    g = _bf16((2, 8, 16, co), 4)
    w = _bf16((3, 3, ci, co), 5, 0.1)
    out = nn.conv3x3(2, g, w, ci=ci, co=co)
    ref = wn.conv3x3_grad_input(_np(g), _np(w))
    assert _rel(_np(out), ref) < 4e-3


@pytest.mark.parametrize("ci,co", [(32, 32), (64, 96), (128, 128)])
@pytest.mark.parametrize("shape", [(2, 16, 32), (3, 64, 64)])
def test_conv_weight_gradient(gpu_lib, ci, co, shape):
    from paper_1704_00865_amd import nn
    print(f"conv wgrad {ci}x{co} {shape}", flush=True)
    x = _bf16(shape + (ci,), 6)
    g = _bf16(shape + (co,), 7)
    out = nn.conv3x3(3, x, g=g, ci=ci, co=co)
    ref = wn.conv3x3_grad_weight(_np(x), _np(g))
    assert _rel(out.double().cpu().numpy(), ref) < 1e-5


def _params(seed):
    """He-initialised parameters with a non-zero output layer and biases,
    rounded so that every weight is a bfloat16 value."""
    import torch
    from paper_1704_00865_amd import nn
    rng = np.random.default_rng(seed)
    p = nn.init_params(seed)
    offs = nn.layer_offsets()
    ci, co, wo, bo = offs[-1]
    w = np.zeros((3, 3, ci, co))
    w[..., 0] = rng.standard_normal((3, 3, ci)) * 0.05
    p[wo:wo + w.size] = w.ravel()
    for i, (ci, co, wo, bo) in enumerate(offs):
        nreal = 1 if i == len(offs) - 1 else co
        p[bo:bo + nreal] = rng.standard_normal(nreal) * 0.05
    pt = torch.tensor(p).to(torch.bfloat16).float()
    for _, co, _, bo in offs:  # biases stay float32
        pt[bo:bo + co] = torch.tensor(p[bo:bo + co])
    return pt.numpy().astype(np.float32)


def _to_oracle(p):
    """Flat padded parameter vector -> oracle Params with the real channels."""
    from paper_1704_00865_amd import nn
    ws, bs = [], []
    offs = nn.layer_offsets()
    for i, (ci, co, wo, bo) in enumerate(offs):
        w = p[wo:wo + 9 * ci * co].astype(np.float64).reshape(3, 3, ci, co)
        b = p[bo:bo + co].astype(np.float64)
        if i == 0:
            w = w[:, :, :4, :]
        if i == len(offs) - 1:
            w, b = w[..., :1], b[:1]
        ws.append(w)
        bs.append(b)
    return wn.Params(ws, bs)


def _features(n, h, w, seed):
    import torch
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, h, w, 4))
    x[..., 2] = (rng.random((n, h, w)) > 0.1)
    xt = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).float()
    return xt.numpy().astype(np.float64), xt.cuda()


def test_network_forward(gpu_lib):
    from paper_1704_00865_amd import nn
    print("net forward", flush=True)
    p = _params(11)
    net = nn.WarmNet(64, 64, batch_max=2)
    net.set_params(p)
    xn, xt = _features(2, 64, 64, 12)
    y = net.forward_features(xt).double().cpu().numpy()
    ref = wn.forward(_to_oracle(p), xn, CH).y
    assert _rel(y, ref) < 3e-2


def test_network_gradient(gpu_lib):
    import torch
    from paper_1704_00865_amd import nn
    print("net gradient", flush=True)
    p = _params(13)
    net = nn.WarmNet(64, 64, batch_max=2)
    net.set_params(p)
    xn, xt = _features(2, 64, 64, 14)
    tgt = np.random.default_rng(15).standard_normal((2, 64, 64)).astype(np.float32)
    g, loss = net.gradient_features(xt, torch.tensor(tgt).cuda())
    g = g.double().cpu().numpy()
    po = _to_oracle(p)
    tp = wn.forward(po, xn, CH)
    ref = wn.backward(po, tp, tgt.astype(np.float64), CH)
    assert loss == pytest.approx(wn.loss(tp.y, tgt), rel=3e-2)
    go = _to_oracle(g)
    for i in range(len(ref.w)):
        assert _rel(go.w[i], ref.w[i]) < 5e-2, i
        assert _rel(go.b[i], ref.b[i]) < 5e-2, i
    # padded entries receive no gradient
    offs = nn.layer_offsets()
    ci, co, wo, bo = offs[0]
    assert np.all(g[wo:wo + 9 * ci * co].reshape(3, 3, ci, co)[:, :, 4:, :] == 0)
    ci, co, wo, bo = offs[-1]
    assert np.all(g[wo:wo + 9 * ci * co].reshape(3, 3, ci, co)[..., 1:] == 0)
    assert np.all(g[bo + 1:bo + co] == 0)


def test_features_and_prediction_scale(gpu_lib):
    """predict = sigma * network(features): with the oracle's features fed
    to forward_features, predict must return sigma times that output."""
    import torch
    from paper_1704_00865_amd import nn
    import synth
    p = _params(17)
    pb = synth.make_problem(64, 64, 18, mask_frac=0.1)
    net = nn.WarmNet(64, 64, batch_max=1)
    net.set_params(p)
    d = torch.tensor(pb.d[None], dtype=torch.float32).cuda()
    npix = torch.tensor(pb.n_pix[None], dtype=torch.float32).cuda()
    mask = torch.tensor(pb.mask[None], dtype=torch.uint8).cuda()
    s = net.predict(d, npix, mask).double().cpu().numpy()[0]
    f, sig = wn.features(pb.d, pb.n_pix, pb.mask)
    y = net.forward_features(torch.tensor(f[None], dtype=torch.float32).cuda()).double().cpu().numpy()[0]
    assert _rel(s, sig * y) < 1e-2


def test_training_reduces_the_loss_and_adam_matches(gpu_lib):
    """Two Adam steps on a fixed batch: each equals the oracle's Adam
    (oracle.warmnet.Adam, float64, carrying its moments from step to step)
    applied to the GPU's own gradient at the current parameters, computed
    from the oracle's features of the same maps; thirty more steps lower
    the loss."""
    import torch
    from paper_1704_00865_amd import nn
    import synth
    probs = [synth.make_problem(64, 64, 30 + i, mask_frac=0.05) for i in range(2)]
    d = torch.tensor(np.stack([q.d for q in probs]), dtype=torch.float32).cuda()
    npix = torch.tensor(np.stack([q.n_pix for q in probs]), dtype=torch.float32).cuda()
    mask = torch.tensor(np.stack([q.mask for q in probs]), dtype=torch.uint8).cuda()
    tgt = torch.tensor(np.stack([q.s_true for q in probs]), dtype=torch.float32).cuda()
    # the network's inputs and scaled targets, as the training step forms them
    feats, sigs = zip(*[wn.features(q.d, q.n_pix, q.mask) for q in probs])
    x = torch.tensor(np.stack(feats), dtype=torch.float32).cuda()
    t_sc = torch.tensor(np.stack([q.s_true / sg for q, sg in zip(probs, sigs)]),
                        dtype=torch.float32).cuda()
    net = nn.WarmNet(64, 64, batch_max=2)
    p0 = _params(19)
    net.set_params(p0)
    lr = 1e-3
    adam = wn.Adam(lr=lr)
    cur = p0.astype(np.float64)
    losses = []
    for step in range(2):
        g, _ = net.gradient_features(x, t_sc)
        ref = adam.step(wn.Params([cur], []), wn.Params([g.double().cpu().numpy()], [])).w[0]
        losses.append(net.train_step(d, npix, mask, tgt, lr))
        got = net.get_params().double().cpu().numpy()
        diff = np.abs(got - ref)
        print(f"  Adam step {step + 1}: max |gpu - oracle| {diff.max():.2e}, "
              f"99.9% {np.quantile(diff, 0.999):.2e}", flush=True)
        # float32 parameters and moments against float64 (observed: 3e-8)
        assert diff.max() <= 1e-6
        cur = got
    for _ in range(30):
        losses.append(net.train_step(d, npix, mask, tgt, lr))
    assert losses[-1] < 0.5 * losses[0]


def test_network_is_translation_equivariant_at_1024(gpu_lib):
    """At the 1024^2 warm-start size, where the float64 reference would take
    minutes: the periodic network commutes with translations by multiples of
    8 pixels (the pooling grid of three levels), and the loss gradient of a
    translated input and target equals the original one (float32 sums over
    the pixels in another order)."""
    import torch
    from paper_1704_00865_amd import nn
    print("net 1024 equivariance", flush=True)
    p = _params(23)
    net = nn.WarmNet(1024, 1024, batch_max=1)
    net.set_params(p)
    _, x = _features(1, 1024, 1024, 24)
    sh = (64, 200)
    y = net.forward_features(x)
    yr = net.forward_features(torch.roll(x, shifts=sh, dims=(1, 2)).contiguous())
    ref = torch.roll(y, shifts=sh, dims=(1, 2))
    assert float((yr - ref).abs().max()) <= 1e-5 * float(ref.abs().max())
    tgt = torch.tensor(np.random.default_rng(25).standard_normal((1, 1024, 1024)),
                       dtype=torch.float32, device="cuda")
    g0, l0 = net.gradient_features(x, tgt)
    g1, l1 = net.gradient_features(torch.roll(x, shifts=sh, dims=(1, 2)).contiguous(),
                                   torch.roll(tgt, shifts=sh, dims=(1, 2)).contiguous())
    assert l1 == pytest.approx(l0, rel=1e-5)
    g0, g1 = g0.double().cpu().numpy(), g1.double().cpu().numpy()
    assert np.linalg.norm(g1 - g0) <= 1e-3 * np.linalg.norm(g0)


def test_warm_start_pipeline(gpu_lib):
    """End to end on small maps: solver targets (chain field), a short
    training run, then the solve from the prediction reaches the same
    solution as the zero start; the prediction beats the zero prediction, and
    the exact field as a start converges at once."""
    import torch
    import synth
    from paper_1704_00865_amd import warmstart
    trp = [synth.make_problem(64, 64, 300 + i, mask_frac=0.1) for i in range(48)]
    tep = [synth.make_problem(64, 64, 400 + i, mask_frac=0.1) for i in range(4)]
    print("warm start pipeline", flush=True)
    res = warmstart.experiment(trp, tep, epochs=6, batch=8, lr=2e-3, warm_lam0=(1e3,),
                               eval_rtol=1e-6, target_rtol=1e-6)
    assert res["zero"]["converged"] == 4 and res["warm"][0]["converged"] == 4
    assert res["pred_rel_error_median"] < 0.9
    assert res["loss_last_epoch"] < res["loss_first_epoch"]
    assert res["exact_start"]["sweeps_mean"] <= 32
    # same solution from either start
    te = warmstart.stack_problems(tep)
    sched = gpu_lib.Schedule(lambda0=1e4, shrink=0.97, rtol=1e-9, max_sweeps=200000,
                             monitor_every=16, chain="augmented", chain_field=True)
    s0, _ = warmstart.solve_set(tep, te, sched)
    s1, _ = warmstart.solve_set(tep, te, sched, s_init=torch.zeros_like(te.d) + 1.0)
    assert float(warmstart.rel_error(s1, s0).max()) < 1e-6


def test_warm_start_float32_targets_on_held_out_maps(gpu_lib):
    """The configuration the benchmark runs, scaled down: float32 training
    targets, float64 evaluation, one warm lambda0.  The sweeps ratio is taken
    over the held-out maps only (disjoint seeds), map by map."""
    import synth
    from paper_1704_00865_amd import warmstart
    trp = [synth.make_problem(64, 64, 500 + i, mask_frac=0.1) for i in range(32)]
    tep = [synth.make_problem(64, 64, 600 + i, mask_frac=0.1) for i in range(4)]
    print("warm start, float32 targets", flush=True)
    res = warmstart.experiment(trp, tep, epochs=2, batch=8, lr=2e-3, warm_lam0=(1e4,),
                               target_precision="f32", target_rtol=1e-4, target_lam0=1e4,
                               target_shrink=0.9)
    assert res["target_dtype"] == "f32" and res["dtype"] == "f64"
    assert res["maps_train"] == 32 and res["maps_test"] == 4
    assert res["held_out"] == {"train_seeds": [500, 531], "test_seeds": [600, 603],
                               "shared_seeds": 0}
    assert res["zero"]["converged"] == 4 and res["warm"][0]["converged"] == 4
    assert res["warm"][0]["sweeps_ratio_per_map_median"] > 0
    assert res["speedup_sweeps"] == pytest.approx(
        res["zero"]["sweeps_mean"] / res["warm"][0]["sweeps_mean"])
    # the wall-time comparison charges the network's inference to its side
    assert res["predict_seconds"] > 0
    assert res["speedup_wall"] == pytest.approx(
        res["zero"]["seconds"] / (res["predict_seconds"] + res["warm"][0]["seconds"]))
    assert res["default_start"] == ("network" if res["speedup_wall"] > 1.0 else "zero")
    assert 0 < res["target_sweeps_mean"] < 200000
