"""Pins of the learned start's oracle (oracle/surrogate_oracle.py), on the
CPU: each check is fixed by something other than the oracle's own
formulas -- a brute-force or library computation, a closed form of grey
dust in a point source's or a diluted black body's field, or a special
case whose answer is known -- and is chosen so that a plausible slip
(swapped axes, a wrong distance scale or softening, 4 pi for 16 pi^2, a
floor applied in the wrong place, the wrong interpolation convention)
fails one of them."""
import math

import numpy as np
import pytest

from oracle import surrogate_oracle as so

SIGMA_SB = 5.670374419e-5   # erg cm^-2 s^-1 K^-4


def _wide_grid(K=600, lo=1e9, hi=3e16):
    """Log-spaced frequencies with trapezoid weights: integrates Planck
    spectra from 2 K to a few 10^4 K to ~1e-5."""
    nu = np.exp(np.linspace(math.log(lo), math.log(hi), K))
    w = np.zeros(K)
    d = np.diff(nu)
    w[:-1] += d / 2
    w[1:] += d / 2
    return nu, w


def _cloud(n, seed=0, empty_frac=0.1):
    rng = np.random.default_rng(seed)
    rho = rng.lognormal(0.0, 1.0, n ** 3) * 1e3
    rho[rng.random(n ** 3) < empty_frac] = 0.0
    return rho


def test_block_mean_against_reshape():
    """The oracle's block loops against numpy's reshaped mean, on an
    anisotropic field (a swapped axis would move values)."""
    rng = np.random.default_rng(1)
    a = rng.standard_normal((12, 12, 12)) + np.arange(12)[None, None, :] * 10.0 + np.arange(12)[:, None, None]
    for S in (1, 2, 3, 4, 6, 12):
        b = 12 // S
        want = a.reshape(S, b, S, b, S, b).mean(axis=(1, 3, 5))
        np.testing.assert_allclose(so._block_mean(a, S), want, rtol=1e-13, atol=1e-12)


def test_grey_dust_point_source_closed_form():
    """Grey dust (the same cross section at every frequency) in the
    unattenuated field of a point source of bolometric luminosity L:
    sigma sum w B(T) = sigma sigma_SB T^4 / pi and sum w sigma J = sigma L /
    (16 pi^2 d^2), so T^4 = L / (16 pi sigma_SB d^2) with d the softened
    block-to-source distance.  A negligible external field only sets the
    flux normalisation."""
    n, S = 16, 4
    nu, w = _wide_grid()
    sig = np.full(nu.shape, 3e-22)
    Tstar = 1e4
    Lnu = so.planck(nu, Tstar) * 4 * math.pi ** 2 * (7e12) ** 2   # black body of 100 R_sun: L = 4 pi R^2 sigma T^4
    L = float(w @ Lnu)
    I_bg = so.planck(nu, 3.0) * 1e-30
    root = 3.0e16
    pos = np.array([[5.3, 9.1, 2.2]])
    rho = np.full(n ** 3, 100.0)
    T1 = np.full(n ** 3, 20.0)
    blocks = [(0, 0, 0), (1, 2, 3), (3, 3, 3), (0, 2, 1)]
    got = so.features(rho, root, S, T1, w, sig, I_bg, 5e-22, pos, Lnu[None, :], nu, w, sig, 2.0, 3000.0,
                      blocks=blocks)
    b = n // S
    s = root * b
    for (z, y, x), row in zip(blocks, got):
        d2 = (((x + 0.5) - pos[0, 0] / b) ** 2 + ((y + 0.5) - pos[0, 1] / b) ** 2
              + ((z + 0.5) - pos[0, 2] / b) ** 2 + 0.25) * s * s
        T = (L / (16 * math.pi * SIGMA_SB * d2)) ** 0.25
        assert 5.0 < T < 2000.0
        assert 10 ** (row[2] * 0.5 + 1.5) == pytest.approx(T, rel=2e-4)


def test_diluted_black_body_external_field():
    """Grey dust in an isotropic field W B(T_bb) with no point sources:
    T_thin = W^(1/4) T_bb; the source-flux channel is exactly 0."""
    n, S = 8, 2
    nu, w = _wide_grid()
    sig = np.full(nu.shape, 1e-22)
    for W, Tbb in ((1e-12, 6000.0), (1e-3, 40.0), (0.5, 1000.0)):
        I_bg = W * so.planck(nu, Tbb)
        rho = np.full(n ** 3, 10.0)
        got = so.features(rho, 1e17, S, np.full(n ** 3, 15.0), w, sig, I_bg, 5e-22, np.zeros((0, 3)),
                          np.zeros((0, nu.size)), nu, w, sig, 2.0, 3000.0, blocks=[(1, 0, 1)])
        assert 10 ** (got[0, 2] * 0.5 + 1.5) == pytest.approx(W ** 0.25 * Tbb, rel=2e-4)
        assert got[0, 1] == 0.0


def test_source_flux_equal_to_external_field():
    """A source whose bolometric flux at a block's softened distance equals
    the external field's 4 pi J gives channel 1 = log10(2) / 4 there."""
    n, S = 8, 4
    nu, w = _wide_grid(K=50)
    I_bg = so.planck(nu, 5000.0) * 1e-13
    F_ext = 4 * math.pi * float(w @ I_bg)
    root = 1e17
    b = n // S
    pos = np.array([[0.5, 0.5, 0.5]])                 # root units: inside block (0, 0, 0)
    z, y, x = 2, 1, 3
    d2 = (((x + 0.5) - 0.25) ** 2 + ((y + 0.5) - 0.25) ** 2 + ((z + 0.5) - 0.25) ** 2 + 0.25) * (root * b) ** 2
    shape = so.planck(nu, 8000.0)
    Lnu = shape * (F_ext * 4 * math.pi * d2 / float(w @ shape))
    got = so.features(np.full(n ** 3, 1.0), root, S, np.full(n ** 3, 10.0), w, np.full(nu.shape, 1e-22), I_bg,
                      5e-22, pos, Lnu[None, :], nu, w, np.full(nu.shape, 1e-22), 2.0, 3000.0, blocks=[(z, y, x)])
    assert got[0, 1] == pytest.approx(math.log10(2.0) / 4, rel=1e-12)


def test_optical_depth_and_T1_channels():
    """Channel 0 of a block of known mean density; channel 3 of a block at
    a uniform 100 K is 1, and a block with some empty cells takes them at
    T_floor (log mean, not mean of T)."""
    n, S = 8, 2
    rho = _cloud(n, seed=3, empty_frac=0.0)
    rho3 = rho.reshape(n, n, n)
    T1 = np.full(n ** 3, 100.0)
    T1.reshape(n, n, n)[4:, 4:, 4:] = 10.0
    rho3[4, 4, 4] = 0.0                               # one empty cell in block (1, 1, 1)
    nu, w = _wide_grid(K=30)
    sig = np.full(nu.shape, 1e-22)
    root = 2e17
    got = so.features(rho3.reshape(-1), root, S, T1, w, sig, so.planck(nu, 5000.0) * 1e-13, 5e-22,
                      np.zeros((0, 3)), np.zeros((0, nu.size)), nu, w, sig, 2.0, 3000.0)
    tau = 5e-22 * rho3[0:4, 0:4, 4:8].mean() * root * 4
    assert got[0, 0, 1, 0] == pytest.approx(math.log10(tau + 1e-4) / 2, rel=1e-12)
    assert got[0, 1, 0, 3] == pytest.approx(1.0, abs=1e-14)
    want = ((63 * math.log10(10.0) + math.log10(2.0)) / 64 - 1.5) / 0.5
    assert got[1, 1, 1, 3] == pytest.approx(want, rel=1e-12)


def test_target_known_ratio_and_empty_cells():
    """T = 10^0.1 T1 everywhere: 0.1 / scale in full blocks; a block with
    k of its b^3 cells empty gives (1 - k / b^3) 0.1 / scale; temperatures
    below the floor are raised to it on both sides."""
    n, S = 8, 4
    rho = np.full(n ** 3, 5.0)
    rho.reshape(n, n, n)[0, 0, 0:2] = 0.0            # two empty cells in block (0, 0, 0)
    rng = np.random.default_rng(4)
    T1 = rng.uniform(5.0, 80.0, n ** 3)
    T = T1 * 10 ** 0.1
    t = so.target(rho, S, T, T1, 2.0, 0.05)
    assert t[0, 0, 0] == pytest.approx((1 - 2 / 8) * 0.1 / 0.05, rel=1e-12)
    assert t[2, 3, 1] == pytest.approx(0.1 / 0.05, rel=1e-12)
    T1b = np.full(n ** 3, 1.0)
    tb = so.target(np.full(n ** 3, 5.0), S, np.full(n ** 3, 4.0), T1b, 2.0, 1.0)
    assert np.allclose(tb, math.log10(2.0))            # 4 K against the 2 K floor, not 1 K


@pytest.mark.parametrize("n,S", [(8, 4), (12, 4), (16, 16), (16, 2), (9, 3)])
def test_upsampling_against_torch_trilinear(n, S):
    """The interpolation is torch's trilinear up-sampling with
    align_corners=False (a library routine, run in FP64 on the CPU)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(n * 100 + S)
    pred = rng.standard_normal((S, S, S))
    want = torch.nn.functional.interpolate(torch.from_numpy(pred)[None, None], size=(n, n, n), mode="trilinear",
                                           align_corners=False)[0, 0].numpy()
    np.testing.assert_allclose(so.upsample(pred, n), want, rtol=1e-12, atol=1e-12)


def test_apply_identity_clamps_and_empty_cells():
    """Zero output and offset: the start is T1 raised to the floor; empty
    cells are 0; a large offset clamps at T_max."""
    n, S = 8, 2
    rho = _cloud(n, seed=5)
    rng = np.random.default_rng(6)
    T1 = rng.uniform(0.5, 90.0, n ** 3)
    T = so.apply(rho, np.zeros((S, S, S)), 0.1, 0.0, T1, 2.0, 3000.0)
    np.testing.assert_array_equal(T[rho == 0], 0.0)
    np.testing.assert_allclose(T[rho > 0], np.maximum(T1[rho > 0], 2.0), rtol=1e-15)
    T = so.apply(rho, np.zeros((S, S, S)), 0.1, 5.0, T1, 2.0, 3000.0)
    assert np.all(T[rho > 0] == 3000.0)
    T = so.apply(rho, np.full((S, S, S), 2.0), 0.1, 0.0, T1, 2.0, 3000.0)
    np.testing.assert_allclose(T[rho > 0], np.maximum(T1[rho > 0], 2.0) * 10 ** 0.2, rtol=1e-13)


def test_absorbed_target_and_apply():
    """A = 10^0.3 A1 gives 0.3 / scale in full blocks; empty cells and
    cells with A1 = 0 count 0; applying a constant output c multiplies A1
    by 10^(c scale) and keeps empty cells at 0; target and apply invert
    each other on a field that is constant over each block's
    interpolation stencil (S = n)."""
    n, S = 8, 4
    rng = np.random.default_rng(7)
    rho = np.full(n ** 3, 3.0)
    rho.reshape(n, n, n)[7, 7, 6:8] = 0.0             # two empty cells in block (3, 3, 3)
    A1 = rng.uniform(1e20, 1e24, n ** 3)
    A1.reshape(n, n, n)[0, 0, 0] = 0.0                # an unhit cell in block (0, 0, 0)
    A = A1 * 10 ** 0.3
    t = so.target_absorbed(rho, S, A, A1, 0.1)
    assert t[1, 2, 3] == pytest.approx(3.0, rel=1e-12)
    assert t[3, 3, 3] == pytest.approx(3.0 * 6 / 8, rel=1e-12)
    assert t[0, 0, 0] == pytest.approx(3.0 * 7 / 8, rel=1e-12)
    out = so.apply_absorbed(rho, np.full((S, S, S), 2.0), 0.1, A1)
    np.testing.assert_allclose(out[rho > 0], A1[rho > 0] * 10 ** 0.2, rtol=1e-13)
    assert np.all(out[rho == 0] == 0.0)
    t8 = so.target_absorbed(np.full(n ** 3, 1.0), n, A, A1, 1.0)
    back = so.apply_absorbed(np.full(n ** 3, 1.0), t8, 1.0, A1)
    ok = A1 > 0
    np.testing.assert_allclose(back[ok], A[ok], rtol=1e-12)
