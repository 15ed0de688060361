"""FP64 numpy oracle of the 3-D convolutional U-Net surrogate.

TEST INFRASTRUCTURE ONLY: used by tests to check the GPU BF16/MFMA
kernels; never imported by the library.

Tensors are channels-last: activations x[n, z, y, x, c]; weights
w[kz, ky, kx, c_in, c_out].  Operations, written from their definitions:
  conv3:  y[p, o] = b[o] + sum_{d in {-1,0,1}^3, i} w[d+1, i, o] x[p+d, i]   (zero padding)
  down2:  y[q, o] = b[o] + sum_{e in {0,1}^3, i} w[e, i, o] x[2q+e, i]      (stride-2, 2^3 kernel)
  up2:    y[2q+e, o] = b[o] + sum_i w[e, i, o] x[q, i]                        (transposed 2^3, stride 2)
  lrelu:  y = x if x > 0 else a x
Backward passes are the exact adjoints (data) and the outer-product
reductions (weights, biases).  Each matmul below is a library primitive
standing for one kernel offset's sum over input channels.
"""
from __future__ import annotations

import numpy as np

LEAK = 0.1


def _shift(x, dz, dy, dx):
    """x shifted so that out[p] = x[p + d] with zeros outside."""
    n, Z, Y, X, c = x.shape
    out = np.zeros_like(x)
    zs, ze = max(0, -dz), min(Z, Z - dz)
    ys, ye = max(0, -dy), min(Y, Y - dy)
    xs, xe = max(0, -dx), min(X, X - dx)
    out[:, zs:ze, ys:ye, xs:xe] = x[:, zs + dz:ze + dz, ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def conv3(x, w, b=None):
    y = np.zeros(x.shape[:4] + (w.shape[4],))
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                y += _shift(x, kz - 1, ky - 1, kx - 1) @ w[kz, ky, kx]
    if b is not None:
        y += b
    return y


def conv3_bwd(x, w, dy):
    """Gradients of conv3 with respect to x, w and b."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                xs = _shift(x, kz - 1, ky - 1, kx - 1)
                dw[kz, ky, kx] = xs.reshape(-1, x.shape[-1]).T @ dy.reshape(-1, dy.shape[-1])
                dx += _shift(dy @ w[kz, ky, kx].T, -(kz - 1), -(ky - 1), -(kx - 1))
    return dx, dw, dy.sum(axis=(0, 1, 2, 3))


def down2(x, w, b=None):
    n, Z, Y, X, c = x.shape
    y = np.zeros((n, Z // 2, Y // 2, X // 2, w.shape[4]))
    for ez in range(2):
        for ey in range(2):
            for ex in range(2):
                y += x[:, ez::2, ey::2, ex::2] @ w[ez, ey, ex]
    if b is not None:
        y += b
    return y


def down2_bwd(x, w, dy):
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for ez in range(2):
        for ey in range(2):
            for ex in range(2):
                xs = x[:, ez::2, ey::2, ex::2]
                dw[ez, ey, ex] = xs.reshape(-1, x.shape[-1]).T @ dy.reshape(-1, dy.shape[-1])
                dx[:, ez::2, ey::2, ex::2] = dy @ w[ez, ey, ex].T
    return dx, dw, dy.sum(axis=(0, 1, 2, 3))


def up2(x, w, b=None):
    n, Z, Y, X, c = x.shape
    y = np.zeros((n, 2 * Z, 2 * Y, 2 * X, w.shape[4]))
    for ez in range(2):
        for ey in range(2):
            for ex in range(2):
                y[:, ez::2, ey::2, ex::2] = x @ w[ez, ey, ex]
    if b is not None:
        y += b
    return y


def up2_bwd(x, w, dy):
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for ez in range(2):
        for ey in range(2):
            for ex in range(2):
                g = dy[:, ez::2, ey::2, ex::2]
                dw[ez, ey, ex] = x.reshape(-1, x.shape[-1]).T @ g.reshape(-1, g.shape[-1])
                dx += g @ w[ez, ey, ex].T
    return dx, dw, dy.sum(axis=(0, 1, 2, 3))


def lrelu(x):
    return np.where(x > 0, x, LEAK * x)


def lrelu_bwd(x, dy):
    return np.where(x > 0, dy, LEAK * dy)


# ---------------------------------------------------------------- network
def init_params(cin, cout, base, levels, seed):
    """He-normal weights, zero biases.  Level l has base * 2^l channels and
    two 3^3 convolutions; a stride-2 2^3 convolution goes down, a
    transposed 2^3 convolution comes up, and the skip is concatenated
    (skip channels first, then the upsampled ones)."""
    rng = np.random.default_rng(seed)

    def conv(k, ci, co):
        return rng.standard_normal((k, k, k, ci, co)) * np.sqrt(2.0 / (k ** 3 * ci)), np.zeros(co)

    P = {}
    ch = [base << l for l in range(levels)]
    c = cin
    for l in range(levels):
        P[f"e{l}a"] = conv(3, c, ch[l])
        P[f"e{l}b"] = conv(3, ch[l], ch[l])
        c = ch[l]
        if l < levels - 1:
            P[f"d{l}"] = conv(2, ch[l], ch[l + 1])
            c = ch[l + 1]
    for l in range(levels - 2, -1, -1):
        P[f"u{l}"] = conv(2, ch[l + 1], ch[l])
        P[f"q{l}a"] = conv(3, 2 * ch[l], ch[l])
        P[f"q{l}b"] = conv(3, ch[l], ch[l])
    P["out"] = conv(3, ch[0], cout)
    return P


def forward(P, x, levels):
    """Returns (output, cache of every intermediate for backward)."""
    cache = {"x": x}
    h = x
    skips = []
    for l in range(levels):
        for s in "ab":
            z = conv3(h, *P[f"e{l}{s}"])
            cache[f"e{l}{s}_in"], cache[f"e{l}{s}_z"] = h, z
            h = lrelu(z)
        if l < levels - 1:
            skips.append(h)
            z = down2(h, *P[f"d{l}"])
            cache[f"d{l}_in"], cache[f"d{l}_z"] = h, z
            h = lrelu(z)
    for l in range(levels - 2, -1, -1):
        z = up2(h, *P[f"u{l}"])
        cache[f"u{l}_in"], cache[f"u{l}_z"] = h, z
        h = np.concatenate([skips[l], lrelu(z)], axis=-1)
        for s in "ab":
            z = conv3(h, *P[f"q{l}{s}"])
            cache[f"q{l}{s}_in"], cache[f"q{l}{s}_z"] = h, z
            h = lrelu(z)
    y = conv3(h, *P["out"])
    cache["out_in"] = h
    return y, cache


def backward(P, cache, dy, levels):
    """Gradients of sum(dy * output) with respect to every parameter, as a
    dict name -> (dw, db).  Decoder stages are undone from the top (level
    0) down, then the encoder from the bottom up, adding the skip gradient
    of each level to the gradient coming back through its down
    convolution."""
    G = {}
    ch = [P[f"e{l}a"][0].shape[4] for l in range(levels)]
    gx, dw, db = conv3_bwd(cache["out_in"], P["out"][0], dy)
    G["out"] = (dw, db)
    g = gx
    dskip = {}
    for l in range(0, levels - 1):
        for s in "ba":
            gz = lrelu_bwd(cache[f"q{l}{s}_z"], g)
            gx, dw, db = conv3_bwd(cache[f"q{l}{s}_in"], P[f"q{l}{s}"][0], gz)
            G[f"q{l}{s}"] = (dw, db)
            g = gx
        dskip[l] = g[..., :ch[l]]
        gz = lrelu_bwd(cache[f"u{l}_z"], g[..., ch[l]:])
        gx, dw, db = up2_bwd(cache[f"u{l}_in"], P[f"u{l}"][0], gz)
        G[f"u{l}"] = (dw, db)
        g = gx
    for l in range(levels - 1, -1, -1):
        for s in "ba":
            gz = lrelu_bwd(cache[f"e{l}{s}_z"], g)
            gx, dw, db = conv3_bwd(cache[f"e{l}{s}_in"], P[f"e{l}{s}"][0], gz)
            G[f"e{l}{s}"] = (dw, db)
            g = gx
        if l > 0:
            gz = lrelu_bwd(cache[f"d{l - 1}_z"], g)
            gx, dw, db = down2_bwd(cache[f"d{l - 1}_in"], P[f"d{l - 1}"][0], gz)
            G[f"d{l - 1}"] = (dw, db)
            g = gx + dskip[l - 1]
    return G


def mse(y, t):
    """Mean squared error and its gradient."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size
