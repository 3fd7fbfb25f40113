"""FP64 reference of the learned warm start (a U-Net that predicts the initial
image of the step-2 minor cycle).  TEST INFRASTRUCTURE ONLY, like the rest of
this package.  The network is not part of the paper: the paper starts every
minor cycle from zero (Algorithm 1); the network only changes where step 2
starts, never what it converges to.

Definition (the same network the library documents in its header):
* input: two channels (i_H / s, l / s) with s = max|l| (1 if l = 0), padded
  with zero channels to 8;
* encoder level j = 0 .. L-1: x -> relu(conv3x3(x)) -> relu(conv3x3(.)),
  width w 2^j; levels are joined by a 2x2 average pool;
* decoder level j = L-2 .. 0: concatenate [nearest 2x upsampling of the level
  below, encoder output of level j], then two relu(conv3x3(.)) of width w 2^j;
* head: a 1x1 convolution to one channel; warm start s * max(head, 0);
* training loss: mean over pixels of (head - target / s)^2.

conv3x3 is a "same" zero-padded cross-correlation,
    y[b, i, j, o] = bias[o] + sum_{dy, dx in -1..1} sum_c x[b, i+dy, j+dx, c] W[o, dy+1, dx+1, c],
with weights stored as rows W[o][k], k = (3 (dy+1) + (dx+1)) cin + c, padded to
a multiple of 32.  The backward pass is written out by the chain rule.

`rnd` (optional) rounds the tensors the library stores in bfloat16 --
input, weights, activations, and the output gradients fed to the matrix
products -- so that the comparison with the GPU measures accumulation order
only.  All arithmetic here is float64.
"""
from __future__ import annotations

import numpy as np


def layer_table(width=32, levels=4, cin0=8):
    """(cin, cout, c1, c2, up, level) of each 3x3 convolution in parameter order."""
    out, prev = [], cin0
    for j in range(levels):
        w = width << j
        out.append((prev, w, prev, 0, 0, j))
        out.append((w, w, w, 0, 0, j))
        prev = w
    for j in range(levels - 2, -1, -1):
        w = width << j
        out.append((prev + w, w, prev, w, 1, j))
        out.append((w, w, w, 0, 0, j))
        prev = w
    return out


def unpack(params, width=32, levels=4):
    """Parameter vector -> list of (W[cout, 3, 3, cin], b[cout]) and the head (w, b)."""
    params = np.asarray(params, np.float64)
    convs, off = [], 0
    for cin, cout, *_ in layer_table(width, levels):
        kpad = (9 * cin + 31) // 32 * 32
        rows = params[off:off + cout * kpad].reshape(cout, kpad)
        off += cout * kpad
        convs.append((rows[:, :9 * cin].reshape(cout, 3, 3, cin), params[off:off + cout]))
        off += cout
    head = (params[off:off + width], params[off + width])
    assert off + width + 1 == params.size
    return convs, head


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) and back to float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x, W, b):
    B, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((B, H, Wd, W.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + H, kx:kx + Wd, :] @ W[:, ky, kx, :].T
    return y


def conv3x3_back(x, W, g, gq=None):
    """Gradients of conv3x3 with respect to its input, weights and bias; gq
    (default g) is the output gradient as the input and weight gradients use
    it, the bias gradient sums g itself."""
    gq = g if gq is None else gq
    B, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    g2 = gq.reshape(-1, gq.shape[-1])
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + H, kx:kx + Wd, :] += gq @ W[:, ky, kx, :]
            dW[:, ky, kx, :] = g2.T @ xp[:, ky:ky + H, kx:kx + Wd, :].reshape(-1, x.shape[-1])
    return dxp[:, 1:H + 1, 1:Wd + 1, :], dW, g.reshape(-1, g.shape[-1]).sum(0)


def pool(x):
    return 0.25 * (x[:, 0::2, 0::2] + x[:, 1::2, 0::2] + x[:, 0::2, 1::2] + x[:, 1::2, 1::2])


def pool_back(g):
    return 0.25 * np.repeat(np.repeat(g, 2, 1), 2, 2)


def up(x):
    return np.repeat(np.repeat(x, 2, 1), 2, 2)


def up_back(g):
    return g[:, 0::2, 0::2] + g[:, 1::2, 0::2] + g[:, 0::2, 1::2] + g[:, 1::2, 1::2]


def _inputs(dirty_h, low, rnd):
    dirty_h = np.asarray(dirty_h, np.float64)
    low = np.asarray(low, np.float64)
    if dirty_h.ndim == 2:
        dirty_h, low = dirty_h[None], low[None]
    s = np.abs(low).reshape(low.shape[0], -1).max(1)
    s = np.where(s > 0, s, 1.0)
    x = np.zeros(dirty_h.shape + (8,))
    x[..., 0] = dirty_h / s[:, None, None]
    x[..., 1] = low / s[:, None, None]
    return rnd(x), s


def forward(params, dirty_h, low, width=32, levels=4, rnd=None):
    """All activations (a dict) of the network on a batch (or one image)."""
    rnd = rnd or (lambda v: v)
    convs, (hw, hb) = unpack(params, width, levels)
    convs = [(rnd(W), b) for W, b in convs]
    x, s = _inputs(dirty_h, low, rnd)
    act = {"in": x, "s": s}
    h = x
    for j in range(levels):
        if j > 0:
            h = rnd(pool(act[("e", j - 1, 1)]))
            act[("pin", j)] = h
        for t in (0, 1):
            W, b = convs[2 * j + t]
            h = rnd(np.maximum(conv3x3(h, W, b), 0.0))
            act[("e", j, t)] = h
    k = 2 * levels
    for j in range(levels - 2, -1, -1):
        cat = np.concatenate([up(h), act[("e", j, 1)]], axis=-1)
        act[("cat", j)] = cat
        for t in (0, 1):
            W, b = convs[k]
            k += 1
            h = rnd(np.maximum(conv3x3(cat if t == 0 else h, W, b), 0.0))
            act[("d", j, t)] = h
    act["out"] = h @ hw + hb
    return act


def warm_start(params, dirty_h, low, width=32, levels=4, rnd=None):
    act = forward(params, dirty_h, low, width, levels, rnd)
    return act["s"][:, None, None] * np.maximum(act["out"], 0.0)


def loss_grad(params, dirty_h, low, target, width=32, levels=4, rnd=None):
    """(loss, gradient vector in the parameter layout)."""
    rnd_g = rnd or (lambda v: v)
    act = forward(params, dirty_h, low, width, levels, rnd)
    convs, (hw, hb) = unpack(params, width, levels)
    convs = [(rnd_g(W), b) for W, b in convs]
    target = np.asarray(target, np.float64)
    if target.ndim == 2:
        target = target[None]
    t = target / act["s"][:, None, None]
    n = t.size
    d = act["out"] - t
    loss = float(np.sum(d * d) / n)
    gout = 2.0 * d / n
    grads = [None] * len(convs)
    top = act[("d", 0, 1)]
    g_hw = np.tensordot(gout, top, axes=([0, 1, 2], [0, 1, 2]))
    g_hb = gout.sum()
    g = (gout[..., None] * hw) * (top > 0)

    def back(i, xin, g):
        dx, dW, db = conv3x3_back(xin, convs[i][0], g, rnd_g(g))
        grads[i] = (dW, db)
        return dx

    k_of = {}
    k = 2 * levels
    for j in range(levels - 2, -1, -1):
        k_of[j] = k
        k += 2
    dskip = {}
    for j in range(0, levels - 1):
        k = k_of[j]
        dx = back(k + 1, act[("d", j, 0)], g)
        g = dx * (act[("d", j, 0)] > 0)
        dx = back(k, act[("cat", j)], g)
        c1 = act[("cat", j)].shape[-1] - act[("e", j, 1)].shape[-1]
        dskip[j] = dx[..., c1:]
        below = act[("e", j + 1, 1)] if j + 1 == levels - 1 else act[("d", j + 1, 1)]
        g = up_back(dx[..., :c1]) * (below > 0)
    dpin = None
    for j in range(levels - 1, -1, -1):
        if j < levels - 1:
            g = (pool_back(dpin) + dskip[j]) * (act[("e", j, 1)] > 0)
        dx = back(2 * j + 1, act[("e", j, 0)], g)
        g = dx * (act[("e", j, 0)] > 0)
        xin = act["in"] if j == 0 else act[("pin", j)]
        dpin = back(2 * j, xin, g)
    parts = []
    for (cin, cout, *_), (dW, db) in zip(layer_table(width, levels), grads):
        kpad = (9 * cin + 31) // 32 * 32
        rows = np.zeros((cout, kpad))
        rows[:, :9 * cin] = dW.reshape(cout, 9 * cin)
        parts += [rows.ravel(), db]
    parts += [g_hw, [g_hb]]
    return loss, np.concatenate([np.ravel(p) for p in parts])
