"""Per-layer, per-element parity checks of the U-Net (test infrastructure).

The checks take a network object with the device network's read hooks
(``read``, ``backward_to``, ``get_grads``) and compare every stored tensor
with the FP64 oracle's layer applied to that network's own stored inputs.
``Bf16StorageNet`` is such an object built on the CPU from the oracle's
layer functions, rounding to BF16 where the device stores a tensor; it
lets the CPU suite confirm that the bounds accept correct rounding and
reject an indexing mistake.
"""
import numpy as np

from oracle import unet_oracle as U


def bf16_round(a):
    """Round FP32/FP64 values to the nearest BF16 (ties to even), as FP64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- per-layer, per-element bounds
# Every stored BF16 tensor is the round-to-nearest BF16 of an FP32 value
# accumulated from exact BF16 x BF16 products, so against the exact (FP64)
# result f of the same layer on the device's own stored inputs
#     |dev - f| <= U_BF16 |f| + GAMMA * sum |terms|,
# where sum |terms| is the layer applied to absolute values (|W| * |x| + |b|)
# and GAMMA allows FP32 accumulation: matrix-core blocks of 16 products, a
# few thousand accumulation steps at most (up to 13 824-term dot products in
# the forward and backward-data passes, split reductions over positions for
# the weight gradients), each rounding at most 2^-24 relative.  The
# weight gradients stay FP32 (no BF16 term).  An indexing mistake (a wrong
# tap, halo row, brick, column tile or channel offset) moves elements by a
# fraction of their own size, far outside these bounds.
U_BF16 = 2.0 ** -8
GAMMA = 2.0 ** -16
TINY = 1e-30


def layer_table(cin, cout, base, levels):
    """(name, kind, cin, cout, level_in, level_out) in parameter order."""
    ch = [base << l for l in range(levels)]
    out, c = [], cin
    for l in range(levels):
        out.append((f"e{l}a", "conv3", c, ch[l], l, l))
        out.append((f"e{l}b", "conv3", ch[l], ch[l], l, l))
        c = ch[l]
        if l < levels - 1:
            out.append((f"d{l}", "down2", ch[l], ch[l + 1], l, l + 1))
            c = ch[l + 1]
    for l in range(levels - 2, -1, -1):
        out.append((f"u{l}", "up2", ch[l + 1], ch[l], l + 1, l))
        out.append((f"q{l}a", "conv3", 2 * ch[l], ch[l], l, l))
        out.append((f"q{l}b", "conv3", ch[l], ch[l], l, l))
    out.append(("out", "conv3", ch[0], cout, 0, 0))
    return out


_FWD = {"conv3": U.conv3, "down2": U.down2, "up2": U.up2}
_BWD = {"conv3": U.conv3_bwd, "down2": U.down2_bwd, "up2": U.up2_bwd}


def _shape_at(shape, level):
    return tuple(v >> level for v in shape)


def _excess(dev, ref, bound):
    """Largest |dev - ref| / bound (> 1 fails) and its flat index."""
    r = np.abs(dev - ref) / (bound + TINY)
    i = int(np.argmax(r))
    return float(r.ravel()[i]), i


def check_forward_layers(net, P, n, shape, cin, cout, base, levels, y_dev, samples=None):
    """Each layer's stored output against the FP64 layer on the device's own
    stored input, element by element.  samples: restrict the comparison to
    these samples (the layers are per-sample maps).  Returns the report."""
    rows = []
    table = layer_table(cin, cout, base, levels)
    sel = slice(None) if samples is None else list(samples)
    for i, (name, kind, ci, co, lin, lout) in enumerate(table):
        sin, sout = _shape_at(shape, lin), _shape_at(shape, lout)
        x = net.read(i, 0, n, int(np.prod(sin)), ci).astype(np.float64).reshape((n,) + sin + (ci,))[sel]
        w, b = P[name]
        z = _FWD[kind](x, w, b)
        mag = _FWD[kind](np.abs(x), np.abs(w), np.abs(b))
        if i == len(table) - 1:   # the FP32 output of the last layer
            dev = np.asarray(y_dev, np.float64)[sel]
            ref, bound = z, GAMMA * mag
        else:
            dev = net.read(i, 1, n, int(np.prod(sout)), co).astype(np.float64).reshape((n,) + sout + (co,))[sel]
            ref = U.lrelu(z)
            bound = U_BF16 * np.abs(ref) + GAMMA * mag
        r, at = _excess(dev, ref, bound)
        rows.append((name, "forward", r, dev.size))
        assert r <= 1.0, (name, "forward", r, at, float(dev.ravel()[at]), float(ref.ravel()[at]), float(bound.ravel()[at]))
    return rows


def check_backward_layers(net, P, dyt, n, shape, cin, cout, base, levels, layers=None, dx_samples=None):
    """For each layer (backward order): run the backward pass up to it, then
    its weight and bias gradients against the FP64 reductions over the
    device's stored input and output-side gradient, and its backward-data
    result against the FP64 adjoint times the leaky-ReLU slope of its
    stored input (plus the stored skip gradient for a down convolution),
    element by element."""
    table = layer_table(cin, cout, base, levels)
    idx = {t[0]: i for i, t in enumerate(table)}
    order = backward_order(levels)
    offs, o = {}, 0
    for k, (w, b) in P.items():
        offs[k] = (o, o + w.size, o + w.size + b.size)
        o += w.size + b.size
    sel = slice(None) if dx_samples is None else list(dx_samples)
    rows = []
    for name in order:
        if layers is not None and name not in layers:
            continue
        i = idx[name]
        _, kind, ci, co, lin, lout = table[i]
        sin, sout = _shape_at(shape, lin), _shape_at(shape, lout)
        net.backward_to(dyt, i)
        x = net.read(i, 0, n, int(np.prod(sin)), ci).astype(np.float64).reshape((n,) + sin + (ci,))
        dy = net.read(i, 2, n, int(np.prod(sout)), co).astype(np.float64).reshape((n,) + sout + (co,))
        g = net.get_grads().astype(np.float64)
        w, b = P[name]
        o0, o1, o2 = offs[name]
        dxr, dw, db = _BWD[kind](x, w, dy)
        dxa, dwa, dba = _BWD[kind](np.abs(x), np.abs(w), np.abs(dy))
        r, at = _excess(g[o0:o1].reshape(w.shape), dw, GAMMA * dwa)
        rows.append((name, "weight grad", r, dw.size))
        assert r <= 1.0, (name, "weight grad", r, at)
        r, at = _excess(g[o1:o2], db, GAMMA * dba)
        rows.append((name, "bias grad", r, db.size))
        assert r <= 1.0, (name, "bias grad", r, at)
        if name == "e0a":
            continue   # the input needs no gradient
        dev = net.read(i, 3, n, int(np.prod(sin)), ci).astype(np.float64).reshape((n,) + sin + (ci,))
        slope = np.where(x > 0, 1.0, U.LEAK)
        ref, mag = slope * dxr, slope * dxa
        if kind == "down2":   # + the skip gradient from the decoder of this level
            l = int(name[1:])
            q = idx[f"q{l}a"]
            gq = net.read(q, 3, n, int(np.prod(sin)), 2 * ci).astype(np.float64).reshape((n,) + sin + (2 * ci,))
            ref, mag = ref + gq[..., :ci], mag + np.abs(gq[..., :ci])
        bound = U_BF16 * np.abs(ref) + GAMMA * mag
        r, at = _excess(dev[sel], ref[sel], bound[sel])
        rows.append((name, "backward-data", r, dev[sel].size))
        assert r <= 1.0, (name, "backward-data", r, at)
    return rows


def print_rows(rows):
    print("\n  layer   pass            max |err|/bound   elements")
    for name, what, r, cnt in rows:
        print(f"  {name:6s}  {what:14s}  {r:10.3e}   {cnt}")

def backward_order(levels):
    """Layer names in the order the backward pass reaches them."""
    order = ["out"]
    for l in range(levels - 1):
        order += [f"q{l}b", f"q{l}a", f"u{l}"]
    for l in range(levels - 1, -1, -1):
        order += [f"e{l}b", f"e{l}a"] + ([f"d{l - 1}"] if l > 0 else [])
    return order


class Bf16StorageNet:
    """CPU stand-in with the device network's hooks: FP64 layers, BF16
    rounding of every stored tensor (layer outputs after the leaky ReLU,
    the input, the output gradient, every backward-data result), FP64
    parameter gradients.  `plant` = (layer name, pass) adds an indexing
    mistake there: 'forward' shifts the output by one row along x,
    'wgrad' drops the centre tap's contribution, 'dx' shifts the
    backward-data result by one row along y."""

    def __init__(self, P, cin, cout, base, levels, shape, plant=None):
        self.P, self.levels, self.shape, self.plant = P, levels, shape, plant
        self.table = layer_table(cin, cout, base, levels)
        self.idx = {t[0]: i for i, t in enumerate(self.table)}
        self.names = [t[0] for t in self.table]

    def _planted(self, name, what):
        return self.plant is not None and self.plant == (name, what)

    def forward(self, x):
        P, L = self.P, self.levels
        ch = [P[f"e{l}a"][0].shape[4] for l in range(L)]
        self.fin, self.fout = {}, {}

        def run(name, kind, h, act=True):
            self.fin[name] = h
            z = _FWD[kind](h, *P[name])
            y = bf16_round(U.lrelu(z)) if act else z
            if self._planted(name, "forward"):
                y = np.roll(y, 1, axis=3)
            self.fout[name] = y
            return y

        h, skips = bf16_round(x), []
        for l in range(L):
            h = run(f"e{l}a", "conv3", h)
            h = run(f"e{l}b", "conv3", h)
            if l < L - 1:
                skips.append(h)
                h = run(f"d{l}", "down2", h)
        for l in range(L - 2, -1, -1):
            u = run(f"u{l}", "up2", h)
            h = np.concatenate([skips[l], u], axis=-1)
            h = run(f"q{l}a", "conv3", h)
            h = run(f"q{l}b", "conv3", h)
        y = run("out", "conv3", h, act=False)
        self.y = y
        return y

    def backward_to(self, dy, layer):
        stop = self.names[layer]
        P = self.P
        ch = [P[f"e{l}a"][0].shape[4] for l in range(self.levels)]
        self.bdy, self.bdx, self.G = {}, {}, dict(getattr(self, "G", {}))
        gskip = {}

        def bwd(name, kind, g, add=None):
            x = self.fin[name]
            self.bdy[name] = g
            dx, dw, db = _BWD[kind](x, P[name][0], g)
            if self._planted(name, "wgrad"):
                dw = dw.copy()
                dw[tuple(k // 2 for k in dw.shape[:3])] = 0.0
            self.G[name] = (dw, db)
            if name == "e0a":
                return None
            dx = dx * np.where(x > 0, 1.0, U.LEAK)
            if add is not None:
                dx = dx + add
            dx = bf16_round(dx)
            if self._planted(name, "dx"):
                dx = np.roll(dx, 1, axis=2)
            self.bdx[name] = dx
            return dx

        g = bwd("out", "conv3", bf16_round(dy))
        if stop == "out":
            return
        for l in range(self.levels - 1):
            g = bwd(f"q{l}b", "conv3", g)
            if stop == f"q{l}b":
                return
            gc = bwd(f"q{l}a", "conv3", g)
            gskip[l] = gc[..., :ch[l]]
            if stop == f"q{l}a":
                return
            g = bwd(f"u{l}", "up2", gc[..., ch[l]:])
            if stop == f"u{l}":
                return
        for l in range(self.levels - 1, -1, -1):
            g = bwd(f"e{l}b", "conv3", g)
            if stop == f"e{l}b":
                return
            g = bwd(f"e{l}a", "conv3", g)
            if stop == f"e{l}a":
                return
            if l > 0:
                g = bwd(f"d{l - 1}", "down2", g, add=gskip[l - 1])
                if stop == f"d{l - 1}":
                    return

    def read(self, layer, which, n, positions, channels):
        name = self.names[layer]
        t = {0: self.fin, 1: self.fout, 2: getattr(self, "bdy", {}), 3: getattr(self, "bdx", {})}[which][name]
        if name == "out" and which == 1:
            raise ValueError("the last layer's output is not stored")
        return np.asarray(t, np.float32).reshape(n * positions, channels)

    def get_grads(self):
        parts = []
        for k, (w, b) in self.P.items():
            dw, db = self.G.get(k, (np.zeros_like(w), np.zeros_like(b)))
            parts += [dw.ravel(), db.ravel()]
        return np.concatenate(parts).astype(np.float32)
