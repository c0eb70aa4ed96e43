"""GPU parity of the learned warm-start kernels (include/cg_net.h) against
the FP64 reference network (oracle/unet.py), through the C ABI.

The GPU stores weights and activations in bfloat16 and accumulates in
float32; the reference runs in float64 on the same bfloat16-rounded conv
weights and input.  Each bfloat16 rounding of an activation perturbs it by
at most 2^-9 relatively; through the ReLU masks and the sums of the
backward pass these add up to about 1% in norm, so tensors are compared by
relative norm error within 2e-2.  The first convolution's weight gradient
is reached last by the backward pass and collects the most: rounding only
the forward activations of the float64 reference to bfloat16 already moves
it by about 2% (L = 3, three input channels), so it gets 3e-2.
"""
import os
import tempfile

import numpy as np
import pytest

from oracle import unet

pytestmark = pytest.mark.gpu

C_BASE, SCALE = 32, 0.1


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_13880_amd import binding as B
    c = B.Context(0)
    yield c
    c.close()


def _round_convs(p, c, L, cin=1):
    """The parameter vector as the GPU computes with it: conv weights in
    bfloat16, biases and the head in float32."""
    layers, hw, hb, n = unet.layer_table(c, L, cin)
    q = np.asarray(p, dtype=np.float32).astype(np.float64)
    for ly in layers:
        s = slice(ly.w_off, ly.w_off + ly.cout * 9 * ly.cin)
        q[s] = unet.bf16_round(q[s])
    return q


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _setup(ctx, L, H, W, B, seed, cin=1, gain=0.0):
    import torch
    from paper_2604_13880_amd import binding as Bd
    net = Bd.Net(ctx, base_channels=C_BASE, levels=L, height=H, width=W, max_batch=B, out_scale=SCALE, seed=seed,
                 in_channels=cin, residual_gain=gain)
    rng = np.random.default_rng(seed)
    p = unet.init_params(C_BASE, L, seed, cin0=cin)
    p += 0.02 * rng.standard_normal(p.size)      # non-zero biases
    net.set_params(torch.from_numpy(p.astype(np.float32)))
    x = unet.bf16_round(rng.standard_normal((B, H, W) if cin == 1 else (B, H, W, cin)))
    tgt = 0.05 * rng.standard_normal((B, H, W, 2))
    return net, p, x, tgt


@pytest.mark.parametrize("L,H,W,B,cin,gain", [(2, 32, 32, 2, 1, 0.0), (3, 32, 48, 2, 1, 0.0), (4, 64, 64, 1, 1, 0.0),
                                              (3, 32, 32, 2, 3, 0.5)])
def test_forward_and_gradients_match_reference(ctx, L, H, W, B, cin, gain):
    import torch
    print(f"net L={L} H={H} W={W} B={B} cin={cin} gain={gain}", flush=True)
    net, p, x, tgt = _setup(ctx, L, H, W, B, seed=100 + L, cin=cin, gain=gain)
    q = _round_convs(p, C_BASE, L, cin)
    want, cache = unet.forward(q, x, C_BASE, L, SCALE, gain)
    loss_ref, g_ref = unet.backward(q, cache, tgt, C_BASE, L, SCALE)
    got = net.forward(torch.from_numpy(x.astype(np.float32)))
    net.zero_grads()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    net.backward(torch.from_numpy(tgt.astype(np.float32)), loss)
    g = net.grads().cpu().numpy()
    torch.cuda.synchronize()
    assert _rel(got.cpu().numpy(), want) < 2e-2
    assert abs(float(loss.cpu()) - loss_ref) < 2e-2 * loss_ref
    layers, hw, hb, n = unet.layer_table(C_BASE, L, cin)
    for k, ly in enumerate(layers):
        tol = 3e-2 if k == 0 else 2e-2
        sw = slice(ly.w_off, ly.w_off + ly.cout * 9 * ly.cin)
        sb = slice(ly.b_off, ly.b_off + ly.cout)
        assert _rel(g[sw], g_ref[sw]) < tol, (k, _rel(g[sw], g_ref[sw]))
        assert _rel(g[sb], g_ref[sb]) < tol, (k, "bias", _rel(g[sb], g_ref[sb]))
    assert _rel(g[hw:hw + 2 * C_BASE], g_ref[hw:hw + 2 * C_BASE]) < 2e-2
    assert _rel(g[hb:hb + 2], g_ref[hb:hb + 2]) < 2e-2
    net.close()


def _maxrel(a, b):
    """max |a - b| over the tensor's scale max |b| (element-wise check)."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def test_product_shape_elementwise(ctx):
    """The shipped configuration: 4 levels, 32 base channels, 3 input
    channels (log-density and a two-channel field), 128^2 grid, residual
    head gain 2.4; batch 8 (the reference's float64 CPU pass stays within
    seconds).

    Bound, per tensor (output, every layer's weight and bias gradient, the
    head), in relative norm and element-wise (max abs error over the
    tensor's largest magnitude): the GPU may be no farther from the float64
    net than the same float64 net with bfloat16 storage between layers
    (unet.forward / backward with store=bf16_round) is, times 2, and never
    beyond 3e-2 in norm / 6e-2 element-wise.  The storage roundings flip
    ReLU masks near zero, and the gradients follow the masks
    discontinuously, so two bfloat16 realisations differ from each other
    about as much as either differs from float64 (measured: up to 2.5% in
    norm at this shape).  A wrong element is off by the order of the
    tensor's scale and fails the element-wise bound."""
    import torch
    from paper_2604_13880_amd import learned as Lr
    cfg = Lr.NET_CFG
    L, H, W, cin, gain = cfg["levels"], cfg["height"], cfg["width"], cfg["in_channels"], cfg["residual_gain"]
    net, p, x, tgt = _setup(ctx, L, H, W, 8, seed=321, cin=cin, gain=gain)
    q = _round_convs(p, C_BASE, L, cin)
    got = net.forward(torch.from_numpy(x.astype(np.float32))).cpu().numpy()
    net.zero_grads()
    net.backward(torch.from_numpy(tgt.astype(np.float32)))
    g = net.grads().cpu().numpy()
    want, cache = unet.forward(q, x, C_BASE, L, SCALE, gain)
    _, g_ref = unet.backward(q, cache, tgt, C_BASE, L, SCALE)
    want16, cache16 = unet.forward(q, x, C_BASE, L, SCALE, gain, store=unet.bf16_round)
    _, g16 = unet.backward(q, cache16, tgt, C_BASE, L, SCALE, store=unet.bf16_round)
    layers, hw, hb, n = unet.layer_table(C_BASE, L, cin)
    tensors = [("output", got, want, want16)]
    for k, ly in enumerate(layers):
        sw = slice(ly.w_off, ly.w_off + ly.cout * 9 * ly.cin)
        sb = slice(ly.b_off, ly.b_off + ly.cout)
        tensors.append((f"layer {k:2d} w ({ly.cin}->{ly.cout})", g[sw], g_ref[sw], g16[sw]))
        tensors.append((f"layer {k:2d} b", g[sb], g_ref[sb], g16[sb]))
    tensors.append(("head", g[hw:hb + 2], g_ref[hw:hb + 2], g16[hw:hb + 2]))
    for name, a, ref, r16 in tensors:
        en, ee = _rel(a, ref), _maxrel(a, ref)
        sn, se = _rel(r16, ref), _maxrel(r16, ref)
        print(f"{name:22s} gpu: norm {en:.2e} elem {ee:.2e} | bf16-storage net: norm {sn:.2e} elem {se:.2e}",
              flush=True)
        assert en <= min(3e-2, max(2 * sn, 5e-3)), name
        assert ee <= min(6e-2, max(2 * se, 1e-2)), name
    net.close()


def test_backward_is_deterministic(ctx):
    """Gradient shares are summed in a fixed order: two backward passes of
    the same batch give the same bits (loss included)."""
    import torch
    net, p, x, tgt = _setup(ctx, 3, 64, 64, 4, seed=11, cin=3, gain=1.0)
    xt = torch.from_numpy(x.astype(np.float32))
    tt = torch.from_numpy(tgt.astype(np.float32))
    out = []
    for _ in range(2):
        net.forward(xt)
        net.zero_grads()
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        net.backward(tt, loss)
        out.append((net.grads().clone(), loss.clone()))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    net.close()


def test_gradients_accumulate_and_reset(ctx):
    import torch
    net, p, x, tgt = _setup(ctx, 2, 32, 32, 1, seed=7)
    xt = torch.from_numpy(x.astype(np.float32))
    tt = torch.from_numpy(tgt.astype(np.float32))
    net.zero_grads()
    net.forward(xt)
    net.backward(tt)
    g1 = net.grads().cpu().numpy()
    net.forward(xt)
    net.backward(tt)
    g2 = net.grads().cpu().numpy()
    assert _rel(g2, 2 * g1) < 1e-5
    net.zero_grads()
    assert not net.grads().abs().max().item()
    net.close()


def test_adam_step_matches_reference(ctx):
    import torch
    net, p, x, tgt = _setup(ctx, 2, 32, 32, 2, seed=9)
    p32 = np.asarray(p, np.float32).astype(np.float64)
    net.zero_grads()
    net.forward(torch.from_numpy(x.astype(np.float32)))
    net.backward(torch.from_numpy(tgt.astype(np.float32)))
    g = net.grads().cpu().numpy().astype(np.float64)
    m = np.zeros_like(p32)
    v = np.zeros_like(p32)
    want = p32
    for step in (1, 2):
        net.adam_step(1e-3)
        want, m, v = unet.adam(want, g, m, v, step, lr=1e-3)
    got = net.params().cpu().numpy()
    assert np.max(np.abs(got - want)) < 1e-6
    net.close()


def test_copy_weights_give_closed_forms_on_gpu(ctx):
    import torch
    from paper_2604_13880_amd import binding as Bd
    L, H, W = 3, 32, 32
    from test_oracle_unet import _copy_net
    p = _copy_net(C_BASE, L, False)
    net = Bd.Net(ctx, base_channels=C_BASE, levels=L, height=H, width=W, max_batch=2, out_scale=0.5)
    net.set_params(torch.from_numpy(p.astype(np.float32)))
    x = unet.bf16_round(np.random.default_rng(2).random((2, H, W)))
    got = net.forward(torch.from_numpy(x.astype(np.float32))).cpu().numpy()
    q = 4
    blk = x.reshape(2, H // q, q, W // q, q).mean(axis=(2, 4))
    want = np.repeat(np.repeat(blk, q, axis=1), q, axis=2)
    assert np.max(np.abs(got[..., 0] - 0.5 * want)) < 0.5 * 2 ** -7
    assert np.max(np.abs(got[..., 1] - 0.5 * (2 * want + 0.25))) < 2 ** -6
    net.close()


def test_save_load_roundtrip(ctx):
    import torch
    from paper_2604_13880_amd import binding as Bd
    net, p, x, tgt = _setup(ctx, 2, 32, 32, 1, seed=13)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "w.bin")
        net.save(path)
        other = Bd.Net(ctx, base_channels=C_BASE, levels=2, height=32, width=32, max_batch=1, out_scale=SCALE,
                       seed=99)
        other.load(path)
        assert torch.equal(other.params(), net.params())
        xt = torch.from_numpy(x.astype(np.float32))
        assert torch.equal(other.forward(xt), net.forward(xt))
        wrong = Bd.Net(ctx, base_channels=C_BASE, levels=3, height=32, width=32, max_batch=1)
        with pytest.raises(Bd.CartogramError):
            wrong.load(path)
        other.close()
        wrong.close()
    net.close()


def test_training_fits_a_fixed_batch(ctx):
    import torch
    net, p, x, tgt = _setup(ctx, 3, 32, 32, 4, seed=21)
    xt = torch.from_numpy(x.astype(np.float32))
    # a smooth target the net can represent
    yy, xx = np.meshgrid(np.linspace(0, 1, 32), np.linspace(0, 1, 32), indexing="ij")
    tgt = np.stack([0.05 * np.sin(3 * xx) * np.ones((4, 1, 1)), 0.03 * np.cos(2 * yy) * np.ones((4, 1, 1))], -1)
    tt = torch.from_numpy(tgt.astype(np.float32))
    losses = []
    for it in range(150):
        net.zero_grads()
        net.forward(xt)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        net.backward(tt, loss)
        net.adam_step(2e-3)
        losses.append(float(loss.cpu()))
    assert losses[-1] < 0.1 * losses[0], (losses[0], losses[-1])
    net.close()


def test_net_argument_checks(ctx):
    from paper_2604_13880_amd import binding as Bd
    with pytest.raises(Bd.CartogramError):
        Bd.Net(ctx, base_channels=16, levels=2, height=32, width=32)
    with pytest.raises(Bd.CartogramError):
        Bd.Net(ctx, base_channels=32, levels=3, height=30, width=32)
    with pytest.raises(Bd.CartogramError):   # 2^24 pixels per batch
        Bd.Net(ctx, base_channels=32, levels=2, height=1024, width=1024, max_batch=16)
    net = Bd.Net(ctx, base_channels=32, levels=2, height=32, width=32, max_batch=1)
    import torch
    with pytest.raises(Bd.CartogramError):
        net.forward(torch.zeros((2, 32, 32), device="cuda"))
    net.close()
