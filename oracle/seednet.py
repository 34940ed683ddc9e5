"""CPU oracle of the plane-seed network -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  It shares no code with the GPU library.

The network maps a range image to one normal seed and one planarity logit
per 4x8 tile (learned plane seeding of the key-frame fit).  Four 3x3
convolutions with zero padding 1 and strides (2,2), (2,2), (1,2), (1,1),
channels 4 -> 16 -> 32 -> 32 -> 4, ReLU after the first three; the input
channels are (r, x, y, z) / 16 with (x, y, z) = r d, d the FP32 pixel
direction.  Numerics: inputs, weights and stored activations are rounded to
bfloat16 (round to nearest even); products and sums are exact here (FP64),
FP32 on the GPU.

Parameters are one flat FP32 vector: for each layer its weights
``W[out][in][ky][kx]`` then its biases ``b[out]``.

Training pieces: the loss per labelled tile is the binary cross-entropy of
the planarity logit plus, on planar tiles, ``1 - |cos|`` between the seed
and the label normal (mean over labelled tiles); Adam as published by
Kingma and Ba (2015).
"""
from __future__ import annotations

import numpy as np

LAYERS = ((4, 16, (2, 2)), (16, 32, (2, 2)), (32, 32, (1, 2)), (32, 4, (1, 1)))
IN_SCALE = 1.0 / 16.0


def n_params() -> int:
    return sum(o * i * 9 + o for i, o, _ in LAYERS)


def unpack(params: np.ndarray):
    """[(W (o, i, 3, 3), b (o,), stride)] views of the flat parameter vector."""
    out, at = [], 0
    for i, o, st in LAYERS:
        W = params[at: at + o * i * 9].reshape(o, i, 3, 3)
        at += o * i * 9
        b = params[at: at + o]
        at += o
        out.append((W, b, st))
    return out


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest even), returned as FP32 values."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def net_input(range_img: np.ndarray, directions: np.ndarray) -> np.ndarray:
    """Input channels (4, H, W): (r, r d_x, r d_y, r d_z) / 16, FP32 products."""
    r = np.ascontiguousarray(range_img, dtype=np.float32)
    d = np.ascontiguousarray(directions, dtype=np.float32)
    ch = np.stack([r, r * d[..., 0], r * d[..., 1], r * d[..., 2]])
    return (ch * np.float32(IN_SCALE)).astype(np.float32)


def out_size(n: int, stride: int) -> int:
    return (n - 1) // stride + 1


def conv2d(x: np.ndarray, W: np.ndarray, b: np.ndarray, stride) -> np.ndarray:
    """out[o, y, x] = b[o] + sum_{c, ky, kx} W[o, c, ky, kx] xpad[c, y sy + ky, x sx + kx]."""
    sy, sx = stride
    C, H, Wd = x.shape
    Ho, Wo = out_size(H, sy), out_size(Wd, sx)
    xp = np.zeros((C, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((W.shape[0], Ho, Wo)) + np.asarray(b, np.float64)[:, None, None]
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky: ky + sy * (Ho - 1) + 1: sy, kx: kx + sx * (Wo - 1) + 1: sx]
            out += np.einsum("oc,chw->ohw", np.asarray(W[:, :, ky, kx], np.float64), patch)
    return out


def conv2d_backward(x: np.ndarray, W: np.ndarray, dout: np.ndarray, stride):
    """Gradients of conv2d: (dx, dW, db)."""
    sy, sx = stride
    C, H, Wd = x.shape
    _, Ho, Wo = dout.shape
    xp = np.zeros((C, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros(W.shape)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(ky, ky + sy * (Ho - 1) + 1, sy), slice(kx, kx + sx * (Wo - 1) + 1, sx))
            dW[:, :, ky, kx] = np.einsum("ohw,chw->oc", dout, xp[sl])
            dxp[sl] += np.einsum("oc,ohw->chw", np.asarray(W[:, :, ky, kx], np.float64), dout)
    return dxp[:, 1:-1, 1:-1], dW, dout.sum(axis=(1, 2))


def forward(params: np.ndarray, x0: np.ndarray, rounding: bool = True):
    """Seeds (4, H/4, W/8) and the cache for backward.  ``rounding=False``
    skips the bfloat16 roundings (smooth function, for finite differences)."""
    rnd = bf16 if rounding else (lambda a: np.asarray(a, np.float64))
    a = rnd(x0).astype(np.float64)
    cache = []
    layers = unpack(params)
    for li, (W, b, st) in enumerate(layers):
        Wr = rnd(W).astype(np.float64)
        z = conv2d(a, Wr, b, st)
        cache.append((a, Wr, z))
        if li < len(layers) - 1:
            a = rnd(np.maximum(z, 0.0).astype(np.float32) if rounding else np.maximum(z, 0.0)).astype(np.float64)
        else:
            a = z
    return a, cache


def backward(params: np.ndarray, cache, dout: np.ndarray) -> np.ndarray:
    """Gradient of the parameters (flat, FP64) given d(loss)/d(seeds); the
    roundings pass gradients straight through."""
    layers = unpack(params)
    grads = [None] * len(layers)
    g = np.asarray(dout, np.float64)
    for li in range(len(layers) - 1, -1, -1):
        a, Wr, z = cache[li]
        if li < len(layers) - 1:
            g = g * (z > 0)
        dx, dW, db = conv2d_backward(a, Wr, g, layers[li][2])
        grads[li] = (dW, db)
        g = dx
    return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


def loss(seeds: np.ndarray, planar: np.ndarray, normal: np.ndarray, valid: np.ndarray):
    """Mean over valid tiles of BCE(logit, planar) + planar (1 - |cos(seed, normal)|);
    returns (loss, d loss / d seeds).  seeds (4, TR, TC); planar, valid (TR, TC);
    normal (TR, TC, 3) unit."""
    s = np.asarray(seeds, np.float64)
    n = s[:3]
    logit = s[3]
    y = np.asarray(planar, np.float64)
    v = np.asarray(valid, np.float64)
    cnt = max(v.sum(), 1.0)
    bce = np.maximum(logit, 0) - logit * y + np.log1p(np.exp(-np.abs(logit)))
    nn = np.sqrt((n * n).sum(axis=0)) + 1e-12
    lab = np.moveaxis(np.asarray(normal, np.float64), -1, 0)
    cos = (n * lab).sum(axis=0) / nn
    L = (v * (bce + y * (1.0 - np.abs(cos)))).sum() / cnt
    dlogit = v * (1.0 / (1.0 + np.exp(-logit)) - y) / cnt
    dcos_dn = lab / nn - cos * n / (nn * nn)
    dn = -(v * y * np.sign(cos))[None] * dcos_dn / cnt
    return L, np.concatenate([dn, dlogit[None]])


def adam(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases (FP32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o, _ in LAYERS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (i * 9)), o * i * 9))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def labels_from_tiles(status: np.ndarray, axis: np.ndarray, abc: np.ndarray):
    """Training labels from plain fits: planar = accepted; unit normal of the
    stored plane p_k + a p_k1 + b p_k2 = c (sign: dominant component > 0)."""
    status = np.asarray(status)
    k = np.asarray(axis).astype(int)
    a, b = np.asarray(abc)[..., 0], np.asarray(abc)[..., 1]
    n = np.zeros(status.shape + (3,))
    k1 = np.where(k == 0, 1, 0)
    k2 = np.where(k == 2, 1, 2)
    np.put_along_axis(n, k[..., None], 1.0, axis=-1)
    np.put_along_axis(n, k1[..., None], a[..., None], axis=-1)
    np.put_along_axis(n, k2[..., None], b[..., None], axis=-1)
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    planar = (status == 5).astype(np.float64)
    valid = (status >= 2).astype(np.float64)
    return planar, n, valid
