"""GPU parity of the BF16 matrix-core U-Net against the FP64 oracle.

The network's weights and inputs are rounded to BF16 before both sides see
them, so the two compute the same function; what remains is the BF16
rounding of the stored activations and gradients (relative 2^-8 per
rounding) and FP32 summation order.  Two references:

* the FP64 oracle itself;
* a BF16-storage model: the oracle's own FP64 layer functions composed as
  the device composes them, rounding to BF16 exactly where the device
  stores a tensor (layer outputs after the leaky ReLU, the input, the
  output gradient and every backward-data result).

Device and storage model share every rounding point but not the FP32
summation order, so a few roundings go to the other BF16 neighbour and
the deep gradients amplify those differences through cancellation just as
they amplify the storage error itself.  The device must therefore be no
farther from the storage model than the model is from the FP64 oracle,
and its own distance from the oracle at most twice the model's (plus
5e-3 for tensors the model reproduces almost exactly): a layout or
indexing mistake gives O(1) errors and fails both.

Those norms are a diagnostic of the whole network.  The parity bar is per
layer and per element: each layer's stored output, backward-data result
and parameter gradients against the FP64 oracle's layer applied to the
device's own stored inputs, within the rounding bounds derived below."""
import numpy as np
import pytest

from oracle import unet_oracle as U
from tests.unet_parity import bf16_round, check_backward_layers, check_forward_layers, print_rows

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def soc():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1812_06632_amd import soc as m
    return m


def flat(P):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for (w, b) in P.values()])


def unflat(P, v):
    out, o = {}, 0
    for k, (w, b) in P.items():
        out[k] = (v[o:o + w.size].reshape(w.shape), v[o + w.size:o + w.size + b.size])
        o += w.size + b.size
    return out


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _slope(h):
    return np.where(h > 0, 1.0, U.LEAK)


def bf16_model_forward(P, x, levels):
    """Forward pass with the device's BF16 storage points."""
    act = lambda z: bf16_round(U.lrelu(z))
    c = {"x": x}
    h, skips = x, []
    for l in range(levels):
        c[f"e{l}a_in"] = h
        h = act(U.conv3(h, *P[f"e{l}a"]))
        c[f"e{l}b_in"] = h
        h = act(U.conv3(h, *P[f"e{l}b"]))
        if l < levels - 1:
            skips.append(h)
            c[f"d{l}_in"] = h
            h = act(U.down2(h, *P[f"d{l}"]))
    for l in range(levels - 2, -1, -1):
        c[f"u{l}_in"] = h
        u = act(U.up2(h, *P[f"u{l}"]))
        h = np.concatenate([skips[l], u], axis=-1)
        c[f"q{l}a_in"] = h
        h = act(U.conv3(h, *P[f"q{l}a"]))
        c[f"q{l}b_in"] = h
        h = act(U.conv3(h, *P[f"q{l}b"]))
    c["out_in"] = h
    return U.conv3(h, *P["out"]), c


def bf16_model_backward(P, c, dy, levels):
    """Backward pass with the device's BF16 storage points: every
    backward-data result is multiplied by the leaky ReLU slope of the layer
    input (the sign of the stored activation) and rounded."""
    G = {}
    ch = [P[f"e{l}a"][0].shape[4] for l in range(levels)]
    gy = bf16_round(dy)

    def layer(name, fn, g, want_dx=True):
        dx, dw, db = fn(c[f"{name}_in"], P[name][0], g)
        G[name] = (dw, db)
        return dx * _slope(c[f"{name}_in"]) if want_dx else None

    g = bf16_round(layer("out", U.conv3_bwd, gy))
    gskip = {}
    for l in range(levels - 1):
        g = bf16_round(layer(f"q{l}b", U.conv3_bwd, g))
        gc = bf16_round(layer(f"q{l}a", U.conv3_bwd, g))
        gskip[l] = gc[..., :ch[l]]
        g = bf16_round(layer(f"u{l}", U.up2_bwd, gc[..., ch[l]:]))
    for l in range(levels - 1, -1, -1):
        g = bf16_round(layer(f"e{l}b", U.conv3_bwd, g))
        g = layer(f"e{l}a", U.conv3_bwd, g, want_dx=l > 0)
        if l > 0:
            g = bf16_round(g)
            g = bf16_round(layer(f"d{l - 1}", U.down2_bwd, g) + gskip[l - 1])
    return G


def _case(levels, base, n, shape, cin=2, cout=2, seed=0):
    rng = np.random.default_rng(seed)
    P = U.init_params(cin, cout, base, levels, seed)
    P = {k: (bf16_round(w), bf16_round(0.05 * rng.standard_normal(b.shape))) for k, (w, b) in P.items()}
    x = bf16_round(rng.standard_normal((n,) + shape + (cin,)))
    dy = bf16_round(rng.standard_normal((n,) + shape + (cout,)))
    return P, x, dy


@pytest.mark.parametrize("levels,base,n,shape", [
    (1, 16, 2, (8, 8, 8)),          # 3^3 convolutions only
    (2, 16, 2, (8, 12, 16)),        # + down, up, concatenation; non-cubic
    (3, 16, 2, (16, 16, 16)),       # three levels
    (2, 32, 1, (16, 8, 8)),         # 32/64 channels: two column tiles per wave
    (1, 16, 1, (64, 64, 32)),       # enough position bricks that a weight-gradient workgroup reduces several
    (1, 64, 1, (64, 64, 32)),       # 8^3-brick convolution with two column tiles per wave
])
def test_forward_and_gradients_match_oracle(soc, levels, base, n, shape):
    P, x, dy = _case(levels, base, n, shape)
    ctx = soc.Context(0)
    net = soc.UNet(ctx, 2, 2, base, levels, n, shape)
    net.set_params(flat(P).astype(np.float32))
    assert np.array_equal(net.get_params(), flat(P).astype(np.float32))
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    y = net.forward(xt).cpu().numpy().astype(np.float64)
    yo, cache = U.forward(P, x, levels)
    ym, cm = bf16_model_forward(P, x, levels)
    net.backward(torch.from_numpy(dy.astype(np.float32)).cuda())
    G = unflat(P, net.get_grads().astype(np.float64))
    Go = U.backward(P, cache, dy, levels)
    Gm = bf16_model_backward(P, cm, dy, levels)
    rows = [("y", rel(y, ym), rel(y, yo), rel(ym, yo))]
    for k in P:
        for j, part in ((0, "w"), (1, "b")):
            rows.append((f"{k}.{part}", rel(G[k][j], Gm[k][j]), rel(G[k][j], Go[k][j]), rel(Gm[k][j], Go[k][j])))
    print("\n  tensor       dev-vs-model  dev-vs-oracle  model-vs-oracle")
    for name, a, b, c in rows:
        print(f"  {name:10s}   {a:10.2e}   {b:10.2e}   {c:10.2e}")
    bad = [(name, a, b, c) for name, a, b, c in rows if not (a <= c + 5e-3 and b <= 2.0 * c + 5e-3)]
    assert not bad, bad
    assert rows[0][2] < 1e-2   # forward within 1e-2 of the FP64 oracle
    # per layer and per element, on the device's own stored tensors
    dyt = torch.from_numpy(dy.astype(np.float32)).cuda()
    net.forward(xt)
    rep = check_forward_layers(net, P, n, shape, 2, 2, base, levels, y)
    rep += check_backward_layers(net, P, dyt, n, shape, 2, 2, base, levels)
    print_rows(rep)
    ctx.close()


def test_backward_is_deterministic(soc):
    P, x, dy = _case(2, 16, 2, (8, 8, 8), seed=3)
    ctx = soc.Context(0)
    net = soc.UNet(ctx, 2, 2, 16, 2, 2, (8, 8, 8))
    net.set_params(flat(P).astype(np.float32))
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    dyt = torch.from_numpy(dy.astype(np.float32)).cuda()
    out = []
    for _ in range(2):
        y = net.forward(xt)
        net.backward(dyt)
        out.append((y.cpu().numpy(), net.get_grads()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    ctx.close()


def test_mse_and_adam_step(soc):
    """MSE value and gradient, and one Adam step, against numpy."""
    P, x, _ = _case(2, 16, 2, (8, 8, 8), seed=4)
    ctx = soc.Context(0)
    net = soc.UNet(ctx, 2, 2, 16, 2, 2, (8, 8, 8))
    p0 = flat(P).astype(np.float32)
    net.set_params(p0)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    y = net.forward(xt)
    t = torch.randn_like(y)
    loss, dy = net.mse(y, t)
    d = (y - t).double().cpu().numpy()
    assert loss == pytest.approx(float(np.mean(d * d)), rel=1e-12)
    np.testing.assert_allclose(dy.cpu().numpy(), 2 * d / d.size, rtol=1e-6, atol=1e-12)
    net.backward(dy)
    g = net.get_grads().astype(np.float64)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    net.adam(lr, b1, b2, eps, step=1)
    m, v = (1 - b1) * g, (1 - b2) * g * g
    expect = p0 - lr * (m / (1 - b1)) / (np.sqrt(v / (1 - b2)) + eps)
    np.testing.assert_allclose(net.get_params(), expect, rtol=2e-6, atol=2e-9)
    ctx.close()


def test_training_reduces_loss(soc):
    """A few hundred Adam steps on a fixed batch fit a smooth target field."""
    ctx = soc.Context(0)
    shape = (16, 16, 16)
    net = soc.UNet(ctx, 2, 2, 16, 3, 4, shape, seed=7)
    g = torch.Generator(device="cuda").manual_seed(1)
    x = torch.randn((4,) + shape + (2,), device="cuda", generator=g)
    k = torch.ones(1, 1, 3, 3, 3, device="cuda") / 27.0
    sm = torch.nn.functional.conv3d(x[..., :1].permute(0, 4, 1, 2, 3), k, padding=1).permute(0, 2, 3, 4, 1)
    t = torch.cat([sm, 0.5 * x[..., 1:] + sm], dim=-1).contiguous()
    losses = []
    for step in range(300):
        y = net.forward(x)
        loss, dy = net.mse(y, t)
        losses.append(loss)
        net.backward(dy)
        net.adam(lr=2e-3)
    print(f"\nloss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.1 * losses[0]
    ctx.close()


def test_bad_shapes_rejected(soc):
    ctx = soc.Context(0)
    with pytest.raises(soc.SocError) as e:
        soc.UNet(ctx, 2, 2, 24, 2, 1, (8, 8, 8))      # base not a multiple of 16
    assert e.value.status == soc.EINVAL
    with pytest.raises(soc.SocError):
        soc.UNet(ctx, 2, 2, 16, 3, 1, (8, 8, 6))      # 6 not divisible by 4
    net = soc.UNet(ctx, 2, 2, 16, 1, 1, (8, 8, 8))
    with pytest.raises(soc.SocError):
        net.forward(torch.zeros((2, 8, 8, 8, 2), device="cuda"))   # batch above nmax
    with pytest.raises(ValueError):
        net.forward(torch.zeros((1, 8, 8, 4, 2), device="cuda"))
    ctx.close()


def test_forward_at_full_size(soc):
    """The surrogate's network at full size and in the benchmark's launch
    configuration: 4 levels, base 32, the surrogate's input features and
    one output, a batch of 4 samples of 64^3.  One sample, computed alone by
    the oracle, is within 5e-3 of the BF16-storage model and within 1e-2
    of the FP64 oracle (relative L2)."""
    from paper_1812_06632_amd.surrogate import N_FEATURES
    P, x, _ = _case(4, 32, 4, (64, 64, 64), cin=N_FEATURES, cout=1, seed=3)
    ctx = soc.Context(0)
    net = soc.UNet(ctx, N_FEATURES, 1, 32, 4, 4, (64, 64, 64))
    net.set_params(flat(P).astype(np.float32))
    y = net.forward(torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    j = 2
    ym, _ = bf16_model_forward(P, x[j:j + 1], 4)
    yo, _ = U.forward(P, x[j:j + 1], 4)
    a, b = rel(y[j:j + 1], ym), rel(y[j:j + 1], yo)
    print(f"\nfull-size forward, sample {j}: dev-vs-model {a:.2e}, dev-vs-oracle {b:.2e}, model-vs-oracle {rel(ym, yo):.2e}")
    assert a < 5e-3 and b < 1e-2
    # every layer, element by element, on sample j (and the batch offsets of
    # the other samples through the output layer)
    rep = check_forward_layers(net, P, 4, (64, 64, 64), N_FEATURES, 1, 32, 4, y, samples=[j])
    print_rows(rep)
    ctx.close()


def test_backward_at_full_size(soc):
    """The same network and batch: the weight and bias gradients of the
    output layer, the first layer, the first layer of level 1 and the
    level-0 down convolution over the whole batch, and their backward-data
    results on one sample (the down convolution's with the skip gradient
    added), per element against the FP64 reductions over the device's own
    stored tensors."""
    from paper_1812_06632_amd.surrogate import N_FEATURES
    P, x, dy = _case(4, 32, 4, (64, 64, 64), cin=N_FEATURES, cout=1, seed=5)
    ctx = soc.Context(0)
    net = soc.UNet(ctx, N_FEATURES, 1, 32, 4, 4, (64, 64, 64))
    net.set_params(flat(P).astype(np.float32))
    net.forward(torch.from_numpy(x.astype(np.float32)).cuda())
    dyt = torch.from_numpy(dy.astype(np.float32)).cuda()
    rep = check_backward_layers(net, P, dyt, 4, (64, 64, 64), N_FEATURES, 1, 32, 4,
                                layers={"out", "e1a", "d0", "e0a"}, dx_samples=[1])
    print_rows(rep)
    ctx.close()
