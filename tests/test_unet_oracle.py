"""Pins of the FP64 U-Net oracle: each convolution against brute-force
loops written from its definition, backward passes against central finite
differences, the transposed convolution as the adjoint of the strided one,
and the whole network's gradient against finite differences."""
import itertools

import numpy as np
import pytest

from oracle import unet_oracle as U


def _brute_conv3(x, w, b):
    n, Z, Y, X, ci = x.shape
    co = w.shape[4]
    y = np.zeros((n, Z, Y, X, co))
    for (nn, z, yy, xx, o) in itertools.product(range(n), range(Z), range(Y), range(X), range(co)):
        s = b[o]
        for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
            zz, y2, x2 = z + dz, yy + dy, xx + dx
            if 0 <= zz < Z and 0 <= y2 < Y and 0 <= x2 < X:
                s += np.dot(x[nn, zz, y2, x2], w[dz + 1, dy + 1, dx + 1, :, o])
        y[nn, z, yy, xx, o] = s
    return y


def test_conv3_matches_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 4, 5, 3))
    w = rng.standard_normal((3, 3, 3, 3, 4))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(U.conv3(x, w, b), _brute_conv3(x, w, b), rtol=1e-12, atol=1e-12)


def test_down_up_definitions_and_adjoint():
    """down2 against loops; <down2(x), y> = <x, up2'(y)> where up2' uses the
    same weights with input/output channels swapped (the adjoint)."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 4, 6, 2, 3))
    w = rng.standard_normal((2, 2, 2, 3, 5))
    y = U.down2(x, w)
    ref = np.zeros_like(y)
    for z, yy, xx in itertools.product(range(2), range(3), range(1)):
        for ez, ey, ex in itertools.product(range(2), repeat=3):
            ref[0, z, yy, xx] += x[0, 2 * z + ez, 2 * yy + ey, 2 * xx + ex] @ w[ez, ey, ex]
    np.testing.assert_allclose(y, ref, rtol=1e-12)
    g = rng.standard_normal(y.shape)
    lhs = np.sum(y * g)
    rhs = np.sum(x * U.up2(g, np.swapaxes(w, 3, 4)))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def _fd_check(f, args, grads, idx_list, eps=1e-6):
    for which, idx in idx_list:
        a = args[which]
        old = a[idx]
        a[idx] = old + eps
        fp = f()
        a[idx] = old - eps
        fm = f()
        a[idx] = old
        num = (fp - fm) / (2 * eps)
        assert grads[which][idx] == pytest.approx(num, rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("op", ["conv3", "down2", "up2"])
def test_layer_backward_finite_differences(op):
    rng = np.random.default_rng(2)
    if op == "conv3":
        x = rng.standard_normal((1, 3, 3, 4, 2))
        w = rng.standard_normal((3, 3, 3, 2, 3))
        fwd, bwd = U.conv3, U.conv3_bwd
    elif op == "down2":
        x = rng.standard_normal((1, 4, 2, 4, 2))
        w = rng.standard_normal((2, 2, 2, 2, 3))
        fwd, bwd = U.down2, U.down2_bwd
    else:
        x = rng.standard_normal((1, 2, 2, 1, 2))
        w = rng.standard_normal((2, 2, 2, 2, 3))
        fwd, bwd = U.up2, U.up2_bwd
    b = rng.standard_normal(3)
    g = rng.standard_normal(fwd(x, w, b).shape)
    dx, dw, db = bwd(x, w, g)
    args = [x, w, b]
    f = lambda: float(np.sum(fwd(args[0], args[1], args[2]) * g))
    idx = [(0, tuple(rng.integers(0, s) for s in x.shape)) for _ in range(6)]
    idx += [(1, tuple(rng.integers(0, s) for s in w.shape)) for _ in range(6)]
    idx += [(2, (int(rng.integers(0, 3)),)) for _ in range(2)]
    _fd_check(f, args, [dx, dw, db], idx)


def test_lrelu_and_mse():
    x = np.array([-2.0, -0.5, 0.0, 0.3, 4.0])
    assert np.allclose(U.lrelu(x), [-0.2, -0.05, 0.0, 0.3, 4.0])
    assert np.allclose(U.lrelu_bwd(x, np.ones(5)), [0.1, 0.1, 0.1, 1.0, 1.0])
    l, g = U.mse(np.array([1.0, 3.0]), np.array([0.0, 1.0]))
    assert l == pytest.approx(2.5) and np.allclose(g, [1.0, 2.0])


def test_unet_gradient_finite_differences():
    """Whole network (3 levels, base 2 channels, 8^3 input): every parameter
    tensor's analytic gradient agrees with central differences."""
    rng = np.random.default_rng(24)   # inputs whose pre-activations all lie > 1e-4 from the kink
    L = 3
    P = U.init_params(2, 2, 2, L, seed=25)
    x = rng.standard_normal((1, 8, 8, 8, 2))
    t = rng.standard_normal((1, 8, 8, 8, 2))
    y, cache = U.forward(P, x, L)
    loss, dy = U.mse(y, t)
    G = U.backward(P, cache, dy, L)
    assert set(G) == set(P)

    def loss_of():
        return U.mse(U.forward(P, x, L)[0], t)[0]

    # central differences must not straddle a kink of the leaky ReLU
    zmin = min(float(np.abs(v).min()) for k, v in cache.items() if k.endswith("_z"))
    assert zmin > 1e-5
    eps = 1e-6

    for name in sorted(P):
        w, b = P[name]
        for k in range(2):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            old = w[idx]
            w[idx] = old + eps
            lp = loss_of()
            w[idx] = old - eps
            lm = loss_of()
            w[idx] = old
            assert G[name][0][idx] == pytest.approx((lp - lm) / (2 * eps), rel=1e-5, abs=1e-9), name
        j = int(rng.integers(0, b.shape[0]))
        old = b[j]
        b[j] = old + eps
        lp = loss_of()
        b[j] = old - eps
        lm = loss_of()
        b[j] = old
        assert G[name][1][j] == pytest.approx((lp - lm) / (2 * eps), rel=1e-5, abs=1e-9), name


# ---------------------------------------------------------------- the GPU parity checks themselves
def _storage_case(plant=None):
    from tests.unet_parity import Bf16StorageNet, bf16_round
    levels, base, n, shape = 2, 16, 2, (8, 8, 8)
    rng = np.random.default_rng(0)
    P = U.init_params(2, 2, base, levels, 0)
    P = {k: (bf16_round(w), bf16_round(0.05 * rng.standard_normal(b.shape))) for k, (w, b) in P.items()}
    x = bf16_round(rng.standard_normal((n,) + shape + (2,)))
    dy = bf16_round(rng.standard_normal((n,) + shape + (2,)))
    net = Bf16StorageNet(P, 2, 2, base, levels, shape, plant=plant)
    y = net.forward(x)
    return net, P, y, dy, (n, shape, 2, 2, base, levels)


def test_per_element_checks_accept_bf16_storage():
    """The per-layer, per-element bounds the GPU parity tests apply hold for
    a network that rounds exactly where the device stores tensors."""
    from tests.unet_parity import check_backward_layers, check_forward_layers
    net, P, y, dy, (n, shape, ci, co, base, levels) = _storage_case()
    rows = check_forward_layers(net, P, n, shape, ci, co, base, levels, y)
    rows += check_backward_layers(net, P, dy, n, shape, ci, co, base, levels)
    assert len(rows) == 4 * 9 - 1   # 9 layers: forward, weight, bias, backward-data (none for e0a)
    fwd = [r for (_, what, r, _) in rows if what == "forward"]
    assert max(fwd) > 0.05   # the BF16 term is exercised, not vacuous


@pytest.mark.parametrize("plant", [("e0b", "forward"), ("u0", "forward"), ("q0a", "wgrad"), ("e1a", "wgrad"),
                                   ("d0", "dx"), ("q0b", "dx")])
def test_per_element_checks_reject_an_indexing_mistake(plant):
    """A one-row shift of one layer's output or backward-data result, or a
    dropped tap in one weight gradient, fails the check of that layer."""
    from tests.unet_parity import check_backward_layers, check_forward_layers
    net, P, y, dy, (n, shape, ci, co, base, levels) = _storage_case(plant)
    with pytest.raises(AssertionError) as e:
        check_forward_layers(net, P, n, shape, ci, co, base, levels, y)
        check_backward_layers(net, P, dy, n, shape, ci, co, base, levels)
    assert e.value.args[0][0] == plant[0]
