"""FP64 CPU reference of the learned warm-start network.

TEST INFRASTRUCTURE ONLY.  This module is the plain reference that the
library's bfloat16 training and inference kernels are checked against;
only the tests, the smoke check and the benchmark's CPU-baseline leg may
import it, and it imports nothing from the product package.

The network is not part of the paper (whose warm start is the previous
step of a series, Method: time-varying cartograms); its definition here
is the library's: a U-Net with `levels` resolutions, level l having
c 2^l channels and two 3x3 convolutions (zero padding, bias, ReLU), 2x2
average pooling between encoder levels, nearest x2 upsampling and channel
concatenation [upsampled, skip] in the decoder, and a 1x1 head to two
channels multiplied by out_scale.  The loss is the mean squared error
over all B*H*W*2 outputs.

Parameters are one float vector in the library's order: for each 3x3
layer (enc0a, enc0b, ..., enc{L-1}b, dec{L-2}a, dec{L-2}b, ..., dec0a,
dec0b) W[o][ky][kx][c] then bias[o]; then the head W[2][c] and bias[2].

The backward pass is written out layer by layer (im2col for the weight
gradients, the reversed-tap convolution for the input gradients); it is
pinned by finite differences in the tests.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch
import torch.nn.functional as F


@dataclasses.dataclass
class Layer:
    cin: int
    cout: int
    level: int
    w_off: int
    b_off: int


def layer_table(c: int, L: int, cin0: int = 1):
    """Conv layers in parameter order, head offsets, parameter count
    (cin0 input channels)."""
    layers, off = [], 0

    def add(cin, cout, level):
        nonlocal off
        w = off
        off += cout * 9 * cin
        layers.append(Layer(cin, cout, level, w, off))
        off += cout

    for l in range(L):
        add(cin0 if l == 0 else c << (l - 1), c << l, l)
        add(c << l, c << l, l)
    for l in range(L - 2, -1, -1):
        add((c << (l + 1)) + (c << l), c << l, l)
        add(c << l, c << l, l)
    head_w = off
    off += 2 * c
    head_b = off
    off += 2
    return layers, head_w, head_b, off


def _w(p, ly: Layer):
    """Torch conv weight [o][c][ky][kx] of a layer from the flat vector."""
    w = torch.from_numpy(np.asarray(p[ly.w_off:ly.w_off + ly.cout * 9 * ly.cin], dtype=np.float64))
    return w.reshape(ly.cout, 3, 3, ly.cin).permute(0, 3, 1, 2).contiguous()


def _b(p, ly: Layer):
    return torch.from_numpy(np.asarray(p[ly.b_off:ly.b_off + ly.cout], dtype=np.float64))


def _up(x):
    return x.repeat_interleave(2, dim=2).repeat_interleave(2, dim=3)


def forward(p, x, c: int, L: int, out_scale: float, residual_gain: float = 0.0, store=None):
    """x: [B][H][W] or [B][H][W][C] -> (out [B][H][W][2], cache).  All
    float64.  With a residual gain g the output adds g * x[..., 1:3].

    `store` (e.g. bf16_round) is applied where activations are stored
    between layers: every ReLU output and every pooled input.  Without it
    the pass is plain float64."""
    sto = (lambda z: z) if store is None else (lambda z: torch.from_numpy(store(z.numpy())))
    xa = np.asarray(x, dtype=np.float64)
    if xa.ndim == 3:
        xa = xa[..., None]
    layers, hw, hb, n = layer_table(c, L, xa.shape[-1])
    assert len(p) == n
    t = torch.from_numpy(xa).permute(0, 3, 1, 2).contiguous()
    cache = {"x": t, "in": [], "a": [], "e": [], "cat": [], "da": [], "d": []}
    li = 0
    src = t
    for l in range(L):
        if l > 0:
            src = sto(F.avg_pool2d(cache["e"][l - 1], 2))
        cache["in"].append(src)
        a = sto(torch.relu(F.conv2d(src, _w(p, layers[li]), _b(p, layers[li]), padding=1)))
        e = sto(torch.relu(F.conv2d(a, _w(p, layers[li + 1]), _b(p, layers[li + 1]), padding=1)))
        li += 2
        cache["a"].append(a)
        cache["e"].append(e)
    deep = cache["e"][L - 1]
    cache["cat"] = [None] * L
    cache["da"] = [None] * L
    cache["d"] = [None] * L
    for l in range(L - 2, -1, -1):
        cat = torch.cat([_up(deep), cache["e"][l]], dim=1)
        da = sto(torch.relu(F.conv2d(cat, _w(p, layers[li]), _b(p, layers[li]), padding=1)))
        d = sto(torch.relu(F.conv2d(da, _w(p, layers[li + 1]), _b(p, layers[li + 1]), padding=1)))
        li += 2
        cache["cat"][l], cache["da"][l], cache["d"][l] = cat, da, d
        deep = d
    Wh = torch.from_numpy(np.asarray(p[hw:hw + 2 * c], dtype=np.float64)).reshape(2, c)
    bh = torch.from_numpy(np.asarray(p[hb:hb + 2], dtype=np.float64))
    out = out_scale * (torch.einsum("jc,bchw->bhwj", Wh, deep) + bh)
    if residual_gain:
        out = out + residual_gain * torch.from_numpy(xa[..., 1:3])
    cache["d0"] = deep
    cache["resid"] = residual_gain * xa[..., 1:3] if residual_gain else 0.0
    return out.numpy(), cache


def _conv_backward(g, inp, w):
    """Gradients of y = conv3x3(inp, w) (padding 1) for output gradient g:
    (d inp, d w [o][c][ky][kx], d bias)."""
    B, C, H, W = inp.shape
    cols = F.unfold(inp, 3, padding=1)                      # [B][C*9][H*W], index c*9 + ky*3 + kx
    gg = g.reshape(B, g.shape[1], H * W)                     # [B][O][H*W]
    dw = torch.einsum("bop,bkp->ok", gg, cols).reshape(g.shape[1], C, 3, 3)
    db = g.sum(dim=(0, 2, 3))
    w_rev = w.flip(2, 3).transpose(0, 1).contiguous()        # [c][o][2-ky][2-kx]
    dinp = F.conv2d(g, w_rev, padding=1)
    return dinp, dw, db


def backward(p, cache, target, c: int, L: int, out_scale: float, store=None):
    """Loss (mean squared error) and the flat gradient, float64.

    `store` (e.g. bf16_round) is applied to the ReLU-masked output gradient
    of every 3x3 layer before it enters the weight-gradient and
    input-gradient products (the bias gradient sums it unrounded).  Without
    it the pass is plain float64."""
    sto = (lambda z: z) if store is None else (lambda z: torch.from_numpy(store(z.numpy())))
    layers, hw, hb, n = layer_table(c, L, cache["x"].shape[1])
    grads = np.zeros(n, dtype=np.float64)
    Wh = torch.from_numpy(np.asarray(p[hw:hw + 2 * c], dtype=np.float64)).reshape(2, c)
    bh = torch.from_numpy(np.asarray(p[hb:hb + 2], dtype=np.float64))
    d0 = cache["d0"]
    out = out_scale * (torch.einsum("jc,bchw->bhwj", Wh, d0) + bh)
    if not isinstance(cache["resid"], float):
        out = out + torch.from_numpy(cache["resid"])
    tgt = torch.from_numpy(np.asarray(target, dtype=np.float64))
    diff = out - tgt
    loss = float((diff ** 2).mean())
    g_out = 2.0 * diff / diff.numel()                          # [B][H][W][2]
    g_pre = out_scale * g_out
    grads[hw:hw + 2 * c] = torch.einsum("bhwj,bchw->jc", g_pre, d0).reshape(-1).numpy()
    grads[hb:hb + 2] = g_pre.sum(dim=(0, 1, 2)).numpy()
    g = torch.einsum("bhwj,jc->bchw", g_pre, Wh)

    def put(ly, dw, db):
        grads[ly.w_off:ly.w_off + ly.cout * 9 * ly.cin] = dw.permute(0, 2, 3, 1).reshape(-1).numpy()
        grads[ly.b_off:ly.b_off + ly.cout] = db.numpy()

    def conv_pair(g, ia, ib, inp, a, out_act):
        """Backward through out_act = relu(conv_b(a)), a = relu(conv_a(inp))."""
        g = g * (out_act > 0)
        ga, dw, _ = _conv_backward(sto(g), a, _w(p, layers[ib]))
        put(layers[ib], dw, g.sum(dim=(0, 2, 3)))
        ga = ga * (a > 0)
        gi, dw, _ = _conv_backward(sto(ga), inp, _w(p, layers[ia]))
        put(layers[ia], dw, ga.sum(dim=(0, 2, 3)))
        return gi

    g_skip = [None] * L
    for l in range(L - 1):                      # decoder levels from the output upwards
        ia = 2 * L + 2 * (L - 2 - l)
        gcat = conv_pair(g, ia, ia + 1, cache["cat"][l], cache["da"][l], cache["d"][l])
        cd = c << (l + 1)
        g_skip[l] = gcat[:, cd:]
        gu = gcat[:, :cd]
        B, C, H, W = gu.shape
        g = gu.reshape(B, C, H // 2, 2, W // 2, 2).sum(dim=(3, 5))
    for l in range(L - 1, -1, -1):              # encoder levels, deepest first
        if l < L - 1:
            g = g_skip[l] + _up(g_in) / 4.0
        g_in = conv_pair(g, 2 * l, 2 * l + 1, cache["in"][l], cache["a"][l], cache["e"][l])
    return loss, grads


def init_params(c: int, L: int, seed: int, cin0: int = 1):
    """He-normal weights and zero biases (numpy generator; the library's
    own initialisation uses its own seeded generator)."""
    layers, hw, hb, n = layer_table(c, L, cin0)
    rng = np.random.default_rng(seed)
    p = np.zeros(n, dtype=np.float64)
    for ly in layers:
        p[ly.w_off:ly.w_off + ly.cout * 9 * ly.cin] = rng.standard_normal(ly.cout * 9 * ly.cin) * np.sqrt(2.0 / (9 * ly.cin))
    p[hw:hw + 2 * c] = rng.standard_normal(2 * c) * np.sqrt(1.0 / c)
    return p


def adam(p, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step with bias correction (Kingma and Ba); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a):
    """Round float values to bfloat16 (nearest even), returned as float64."""
    t = torch.from_numpy(np.asarray(a, dtype=np.float32).copy())
    return t.to(torch.bfloat16).to(torch.float64).numpy()
