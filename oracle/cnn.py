"""FP64 reference of the surrogate initialiser network (oracle; test infrastructure).

The paper starts each source from an existing catalog's estimate; the build
adds a small convolutional network that maps a source's 5-band 32x32 patch to
its 27 parameters (in standardised unconstrained coordinates).  Architecture:
four 3x3 same-padded convolutions with 32, 64, 64, 128 channels and ReLU, 2x2
max-pooling after the second, third and fourth, then a 2048 -> 256 ReLU layer
and a 256 -> 27 linear layer.  Loss: mean squared error over the batch and the
27 outputs.  Everything here is plain NumPy FP64 with im2col convolutions.

Parity: pinned by central finite differences of the loss (tests).
"""
from __future__ import annotations

import numpy as np

CONV = [(5, 32), (32, 64), (64, 64), (64, 128)]
POOL_AFTER = (1, 2, 3)          # conv indices followed by 2x2 max-pooling
FC = [(2048, 256), (256, 27)]


def param_shapes():
    shp = []
    for ci, co in CONV:
        shp += [(co, ci, 3, 3), (co,)]
    for fi, fo in FC:
        shp += [(fo, fi), (fo,)]
    return shp


def n_params():
    return int(sum(np.prod(s) for s in param_shapes()))


def unpack(flat):
    out, o = [], 0
    for s in param_shapes():
        n = int(np.prod(s))
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def _im2col(x):
    """x (B,C,H,W) -> (B, C*9, H*W) with zero padding, index c*9 + ky*3 + kx."""
    B, C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    cols = np.empty((B, C, 9, H, W))
    for ky in range(3):
        for kx in range(3):
            cols[:, :, ky * 3 + kx] = xp[:, :, ky:ky + H, kx:kx + W]
    return cols.reshape(B, C * 9, H * W)


def _col2im(cols, shape):
    B, C, H, W = shape
    cols = cols.reshape(B, C, 9, H, W)
    xp = np.zeros((B, C, H + 2, W + 2))
    for ky in range(3):
        for kx in range(3):
            xp[:, :, ky:ky + H, kx:kx + W] += cols[:, :, ky * 3 + kx]
    return xp[:, :, 1:H + 1, 1:W + 1]


def conv_forward(x, Wt, b):
    B, C, H, W = x.shape
    cols = _im2col(x)
    y = np.einsum("ok,bkp->bop", Wt.reshape(Wt.shape[0], -1), cols) + b[None, :, None]
    return y.reshape(B, Wt.shape[0], H, W), cols


def conv_backward(dy, x_shape, cols, Wt):
    B, Co, H, W = dy.shape
    d = dy.reshape(B, Co, H * W)
    dW = np.einsum("bop,bkp->ok", d, cols).reshape(Wt.shape)
    db = d.sum(axis=(0, 2))
    dcols = np.einsum("ok,bop->bkp", Wt.reshape(Co, -1), d)
    dx = _col2im(dcols, x_shape)
    return dx, dW, db


def pool_forward(x):
    B, C, H, W = x.shape
    r = x.reshape(B, C, H // 2, 2, W // 2, 2)
    return r.max(axis=(3, 5))


def pool_backward(dy, x):
    """Route each pooled gradient to the first maximal input of its 2x2 window (row-major order)."""
    B, C, H, W = x.shape
    r = x.reshape(B, C, H // 2, 2, W // 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(B, C, H // 2, W // 2, 4)
    idx = np.argmax(r, axis=-1)
    d = np.zeros_like(r)
    np.put_along_axis(d, idx[..., None], dy[..., None], axis=-1)
    return d.reshape(B, C, H // 2, W // 2, 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(B, C, H, W)


def forward(params, x):
    """Returns output (B,27) and a cache for backward."""
    P = unpack(params) if not isinstance(params, list) else params
    cache = []
    a = x
    for i, (ci, co) in enumerate(CONV):
        z, cols = conv_forward(a, P[2 * i], P[2 * i + 1])
        r = np.maximum(z, 0.0)
        cache.append((a.shape, cols, r))
        a = pool_forward(r) if i in POOL_AFTER else r
    B = x.shape[0]
    f = a.reshape(B, -1)
    W1, b1, W2, b2 = P[8], P[9], P[10], P[11]
    h = np.maximum(f @ W1.T + b1, 0.0)
    y = h @ W2.T + b2
    return y, (cache, f, h, P)


def loss_and_grad(params, x, t):
    """Mean squared error (over batch and outputs) and its gradient (flat, like params)."""
    y, (cache, f, h, P) = forward(params, x)
    B = x.shape[0]
    n = y.size
    loss = np.sum((y - t) ** 2) / n
    dy = 2.0 * (y - t) / n
    g = [None] * 12
    g[10] = dy.T @ h
    g[11] = dy.sum(axis=0)
    dh = (dy @ P[10]) * (h > 0)
    g[8] = dh.T @ f
    g[9] = dh.sum(axis=0)
    da = (dh @ P[8]).reshape(B, 128, 4, 4)
    for i in range(len(CONV) - 1, -1, -1):
        x_shape, cols, r = cache[i]
        if i in POOL_AFTER:
            da = pool_backward(da, r)
        dz = da * (r > 0)
        dx, dW, db = conv_backward(dz, x_shape, cols, P[2 * i])
        g[2 * i], g[2 * i + 1] = dW, db
        da = dx
    return loss, np.concatenate([a.ravel() for a in g])
