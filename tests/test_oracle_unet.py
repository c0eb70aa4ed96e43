"""Pins of the FP64 reference network (oracle/unet.py): parameter count
derived by hand from the architecture, finite-difference gradients, and
hand-built weights that turn the net into closed-form functions (which
fixes the layer order, the concatenation order, pooling, upsampling and
the head layout)."""
import numpy as np
import pytest

from oracle import unet


def test_parameter_count_of_the_warm_start_net():
    # 4 levels, 32/64/128/256 channels, decoder inputs 384/192/96 channels:
    # sum of 9*cin*cout + cout over the 14 conv layers + the 1x1 head (66)
    by_hand = (9 * 1 * 32 + 32) + (9 * 32 * 32 + 32) + (9 * 32 * 64 + 64) + (9 * 64 * 64 + 64) \
        + (9 * 64 * 128 + 128) + (9 * 128 * 128 + 128) + (9 * 128 * 256 + 256) + (9 * 256 * 256 + 256) \
        + (9 * 384 * 128 + 128) + (9 * 128 * 128 + 128) + (9 * 192 * 64 + 64) + (9 * 64 * 64 + 64) \
        + (9 * 96 * 32 + 32) + (9 * 32 * 32 + 32) + 66
    assert by_hand == 1946338
    assert unet.layer_table(32, 4)[3] == by_hand


@pytest.mark.parametrize("L,cin,gain", [(2, 1, 0.0), (3, 1, 0.0), (2, 3, 0.4)])
def test_gradients_vs_finite_differences(L, cin, gain):
    c, H, W, B, scale = 2, 8, 8, 2, 0.7
    rng = np.random.default_rng(11 + L)
    p = unet.init_params(c, L, seed=5, cin0=cin)
    p += 0.05 * rng.standard_normal(p.size)          # non-zero biases, generic kinks
    x = rng.standard_normal((B, H, W, cin))
    tgt = rng.standard_normal((B, H, W, 2))

    def loss_at(q):
        out, cache = unet.forward(q, x, c, L, scale, gain)
        return float(((out - tgt) ** 2).mean())

    out, cache = unet.forward(p, x, c, L, scale, gain)
    loss, g = unet.backward(p, cache, tgt, c, L, scale)
    assert abs(loss - loss_at(p)) < 1e-14
    h = 1e-6
    idx = rng.choice(p.size, 60, replace=False)
    for i in idx:
        q1, q2 = p.copy(), p.copy()
        q1[i] += h
        q2[i] -= h
        fd = (loss_at(q1) - loss_at(q2)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])
    d = rng.standard_normal(p.size)
    fd = (loss_at(p + h * d) - loss_at(p - h * d)) / (2 * h)
    assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(fd))


def _copy_net(c, L, use_skip_at_level0):
    """Weights that copy channel 0 through every level: encoder convs pass
    channel 0 on, decoder convs take channel 0 of the upsampled input, or
    (level 0, if use_skip_at_level0) the first skip channel."""
    layers, hw, hb, n = unet.layer_table(c, L)
    p = np.zeros(n)

    def centre(ly, o, ci):
        p[ly.w_off + ((o * 3 + 1) * 3 + 1) * ly.cin + ci] = 1.0

    for l in range(L):
        centre(layers[2 * l], 0, 0)
        centre(layers[2 * l + 1], 0, 0)
    for l in range(L - 2, -1, -1):
        ia = 2 * L + 2 * (L - 2 - l)
        src = (c << (l + 1)) if (l == 0 and use_skip_at_level0) else 0
        centre(layers[ia], 0, src)
        centre(layers[ia + 1], 0, 0)
    p[hw + 0 * c + 0] = 1.0
    p[hw + 1 * c + 0] = 2.0
    p[hb + 1] = 0.25
    return p


@pytest.mark.parametrize("L", [2, 3])
def test_copy_weights_give_closed_forms(L):
    c, H, W, scale = 2, 16, 16, 0.5
    rng = np.random.default_rng(3)
    x = rng.random((2, H, W))                        # non-negative: ReLU passes it
    out, _ = unet.forward(_copy_net(c, L, True), x, c, L, scale)
    assert np.allclose(out[..., 0], scale * x, rtol=0, atol=1e-15)
    assert np.allclose(out[..., 1], scale * (2 * x + 0.25), rtol=0, atol=1e-15)
    # through the deepest level: block means over 2^(L-1) pixels, repeated
    out, _ = unet.forward(_copy_net(c, L, False), x, c, L, scale)
    q = 2 ** (L - 1)
    blk = x.reshape(2, H // q, q, W // q, q).mean(axis=(2, 4))
    want = np.repeat(np.repeat(blk, q, axis=1), q, axis=2)
    assert np.allclose(out[..., 0], scale * want, rtol=0, atol=1e-14)


def test_residual_head_adds_the_given_field():
    c, L, scale, gain = 2, 2, 0.3, 1.7
    layers, hw, hb, n = unet.layer_table(c, L, 3)
    p = np.zeros(n)
    p[hb:hb + 2] = [0.5, -1.0]                       # zero weights: the net part is scale * bias
    x = np.random.default_rng(1).standard_normal((2, 8, 8, 3))
    out, _ = unet.forward(p, x, c, L, scale, gain)
    assert np.allclose(out, gain * x[..., 1:3] + scale * np.array([0.5, -1.0]), atol=1e-15)


def test_adam_first_step_moves_by_lr_times_sign():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -1e-3, 0.0])
    q, m, v = unet.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=1e-12)
    # after one bias-corrected step m_hat = g, v_hat = g^2: the move is lr * sign(g)
    assert np.allclose(q, [0.9, -1.9, 3.0], atol=1e-9)


def test_storage_rounding_option():
    """store=bf16_round rounds exactly the stored activations (every one a
    bfloat16 value) and the masked gradients entering the products; with
    store=None the pass is the plain float64 one (the finite-difference
    pins above)."""
    c, L = 8, 2
    rng = np.random.default_rng(4)
    p = unet.init_params(c, L, 4, cin0=2) + 0.02 * rng.standard_normal(unet.layer_table(c, L, 2)[3])
    x = unet.bf16_round(rng.standard_normal((2, 8, 8, 2)))
    tgt = 0.1 * rng.standard_normal((2, 8, 8, 2))
    o1, c1 = unet.forward(p, x, c, L, 0.2, 0.5)
    o2, c2 = unet.forward(p, x, c, L, 0.2, 0.5, store=lambda z: z)
    assert np.array_equal(o1, o2)
    o3, c3 = unet.forward(p, x, c, L, 0.2, 0.5, store=unet.bf16_round)
    for key in ("a", "e"):
        for t in c3[key]:
            v = t.numpy()
            assert np.array_equal(v, unet.bf16_round(v))
    assert 0 < np.abs(o3 - o1).max() < 1e-2 * np.abs(o1).max()
    l1, g1 = unet.backward(p, c1, tgt, c, L, 0.2)
    l2, g2 = unet.backward(p, c1, tgt, c, L, 0.2, store=lambda z: z)
    assert l1 == l2 and np.array_equal(g1, g2)
