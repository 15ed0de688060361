"""The learned start's three library maps (soc_surrogate_features,
soc_surrogate_target, soc_surrogate_apply) against the oracle
(oracle/surrogate_oracle.py), element by element, through the C ABI:

  * small clouds at several block sizes b = n / S (1, 2, 4; a ragged
    number of blocks per workgroup), with zero, one and two point
    sources and empty cells;
  * the benchmark cloud's size (128^3 into 64^3 blocks) and the learned
    start's target size (256^3 into 64^3) on sampled blocks and cells;
  * the absorbed-energy channel and channel selection in multi-channel
    arrays (other channels untouched);
  * argument errors.

Tolerances: channels 0, 1, 3 and the target are FP64 sums stored in FP32
(relative 1e-6, absolute 1e-6 near zero); channel 2 inverts the library's
4096-entry temperature table by log-log interpolation, whose error in ln T
is below 1e-6 on these spectra (absolute 2e-5 on the channel, i.e. 1e-5 in
log10 T); the start temperatures interpolate in FP32 (relative 2e-6).
"""
import numpy as np
import pytest

from oracle import surrogate_oracle as so
from paper_1812_06632_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def soc():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1812_06632_amd import soc as m
    return m


@pytest.fixture(scope="module")
def ctx(soc):
    c = soc.Context(0)
    yield c
    c.close()


def _problem(n, n_ps, seed):
    P = W.lognormal_problem(n=n, K=16, sigma_ln=1.2, tau_v_mean=8.0, seed=seed, L_star_lsun=3e5,
                            packages_per_freq=1000,
                            ps_frac=((0.31, 0.52, 0.47), (0.72, 0.2, 0.6))[:n_ps])
    if n_ps == 0:
        P.ps_pos = np.zeros((0, 3))
        P.ps_Lnu = np.zeros((0, P.K))
    return P


def _T1(P, seed):
    rng = np.random.default_rng(seed)
    T = rng.uniform(1.0, 120.0, P.grid.ncells).astype(np.float32)   # some below the 2 K floor
    T[P.grid.density() == 0] = 0.0
    return T


def _lib_features(soc, ctx, P, S, T1):
    g = soc.grid_from_workload(ctx, P.grid)
    table = soc.temp_table_build(ctx, P.emit_nu, P.emit_w, P.emit_sigma_abs, P.T_floor, P.T_max, 4096)
    X = soc.surrogate_features(ctx, g, table, S, P.w, P.sigma_abs, P.I_bg, W.SIGMA_V, P.ps_pos, P.ps_Lnu,
                               torch.from_numpy(T1).cuda())
    return g, table, X.cpu().numpy().astype(np.float64)


def _orc_features(P, S, T1, blocks=None):
    return so.features(P.grid.density(), P.grid.root_cell_cm, S, T1, P.w, P.sigma_abs, P.I_bg, W.SIGMA_V,
                       P.ps_pos, P.ps_Lnu, P.emit_nu, P.emit_w, P.emit_sigma_abs, P.T_floor, P.T_max,
                       blocks=blocks)


def _check_features(got, want):
    for ch in (0, 1, 3):
        np.testing.assert_allclose(got[..., ch], want[..., ch], rtol=1e-6, atol=1e-6, err_msg=f"channel {ch}")
    np.testing.assert_allclose(got[..., 2], want[..., 2], rtol=0, atol=2e-5, err_msg="channel 2")


@pytest.mark.parametrize("n,S,n_ps", [(16, 16, 2), (16, 8, 1), (24, 6, 2), (32, 8, 0), (20, 5, 2)])
def test_features_small(soc, ctx, n, S, n_ps):
    P = _problem(n, n_ps, seed=n + S)
    T1 = _T1(P, seed=S)
    _, _, got = _lib_features(soc, ctx, P, S, T1)
    assert got.shape == (S, S, S, 4)
    _check_features(got, _orc_features(P, S, T1))
    if n_ps:
        assert got[..., 1].max() > 0.05


@pytest.mark.parametrize("n", [128, 256])
def test_features_full_size_sampled(soc, ctx, n):
    """The benchmark cloud (two sources) at 128^3 and a 256^3 cloud, both
    into 64^3 blocks: 300 random blocks plus the corners and the sources'
    blocks."""
    P = W.lognormal_problem(n=n, K=32, sigma_ln=1.5 if n == 256 else 1.0, tau_v_mean=20.0 if n == 256 else 5.0,
                            packages_per_freq=1000)
    S = 64
    T1 = _T1(P, seed=n)
    _, _, got = _lib_features(soc, ctx, P, S, T1)
    rng = np.random.default_rng(n)
    blocks = [tuple(int(v) for v in rng.integers(0, S, 3)) for _ in range(300)]
    blocks += [(0, 0, 0), (S - 1, S - 1, S - 1), (0, S - 1, 0)]
    b = n // S
    blocks += [(int(p[2] // b), int(p[1] // b), int(p[0] // b)) for p in P.ps_pos]
    want = _orc_features(P, S, T1, blocks=blocks)
    got_rows = np.array([got[z, y, x] for z, y, x in blocks])
    _check_features(got_rows, want)


@pytest.mark.parametrize("n,S", [(16, 8), (24, 4), (32, 32)])
def test_target(soc, ctx, n, S):
    P = _problem(n, 2, seed=3)
    T1 = _T1(P, seed=4)
    rng = np.random.default_rng(5)
    T = (T1 * rng.uniform(0.8, 3.0, T1.size)).astype(np.float32)
    g = soc.grid_from_workload(ctx, P.grid)
    table = soc.temp_table_build(ctx, P.emit_nu, P.emit_w, P.emit_sigma_abs, P.T_floor, P.T_max, 4096)
    got = soc.surrogate_target(ctx, g, table, S, torch.from_numpy(T).cuda(), torch.from_numpy(T1).cuda(), 0.1)
    want = so.target(P.grid.density(), S, T, T1, P.T_floor, 0.1)
    np.testing.assert_allclose(got.cpu().numpy()[..., 0], want, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("n,S", [(16, 8), (24, 4), (32, 32), (32, 16), (20, 5)])
def test_apply(soc, ctx, n, S):
    P = _problem(n, 1, seed=6)
    T1 = _T1(P, seed=7)
    rng = np.random.default_rng(8)
    pred = rng.standard_normal((S, S, S)).astype(np.float32)
    g = soc.grid_from_workload(ctx, P.grid)
    table = soc.temp_table_build(ctx, P.emit_nu, P.emit_w, P.emit_sigma_abs, P.T_floor, P.T_max, 4096)
    got = soc.surrogate_apply(ctx, g, table, S, torch.from_numpy(pred).cuda(), 0.2, 0.05,
                              torch.from_numpy(T1).cuda()).cpu().numpy()
    want = so.apply(P.grid.density(), pred.astype(np.float64), 0.2, 0.05, T1, P.T_floor, P.T_max)
    np.testing.assert_array_equal(got[want == 0], 0.0)
    np.testing.assert_allclose(got, want, rtol=2e-6, atol=0)


@pytest.mark.parametrize("n,S", [(16, 8), (24, 4), (20, 20)])
def test_absorbed_target_and_apply_in_channel_1_of_2(soc, ctx, n, S):
    P = _problem(n, 2, seed=12)
    rng = np.random.default_rng(13)
    A1 = rng.uniform(1e18, 1e25, P.grid.ncells)
    A1[rng.random(P.grid.ncells) < 0.05] = 0.0
    A = A1 * rng.uniform(1.0, 6.0, P.grid.ncells)
    g = soc.grid_from_workload(ctx, P.grid)
    out = torch.full((S, S, S, 2), -7.0, dtype=torch.float32, device="cuda")
    soc.surrogate_target_absorbed(ctx, g, S, torch.from_numpy(A).cuda(), torch.from_numpy(A1).cuda(), 0.25,
                                  out=out, channels=2, channel=1)
    got = out.cpu().numpy()
    assert np.all(got[..., 0] == -7.0)
    want = so.target_absorbed(P.grid.density(), S, A, A1, 0.25)
    np.testing.assert_allclose(got[..., 1], want, rtol=1e-6, atol=1e-6)
    pred = rng.standard_normal((S, S, S, 2)).astype(np.float32)
    Ag = soc.surrogate_apply_absorbed(ctx, g, S, torch.from_numpy(pred).cuda(), 0.3, torch.from_numpy(A1).cuda(),
                                      channels=2, channel=1).cpu().numpy()
    want = so.apply_absorbed(P.grid.density(), pred[..., 1].astype(np.float64), 0.3, A1)
    np.testing.assert_array_equal(Ag[want == 0], 0.0)
    np.testing.assert_allclose(Ag, want, rtol=2e-6, atol=0)
    table = soc.temp_table_build(ctx, P.emit_nu, P.emit_w, P.emit_sigma_abs, P.T_floor, P.T_max, 4096)
    T1 = _T1(P, seed=14)
    Tg = soc.surrogate_apply(ctx, g, table, S, torch.from_numpy(pred).cuda(), 0.2, 0.0, torch.from_numpy(T1).cuda(),
                             channels=2, channel=0).cpu().numpy()
    want = so.apply(P.grid.density(), pred[..., 0].astype(np.float64), 0.2, 0.0, T1, P.T_floor, P.T_max)
    np.testing.assert_allclose(Tg, want, rtol=2e-6, atol=0)


def test_apply_full_size_sampled(soc, ctx):
    """256^3 start temperatures from a 64^3 output, on 2000 sampled cells
    (the corners and faces included)."""
    P = W.lognormal_problem(n=256, K=8, sigma_ln=1.5, tau_v_mean=20.0, packages_per_freq=1000)
    n, S = 256, 64
    T1 = _T1(P, seed=9)
    pred = np.random.default_rng(10).standard_normal((S, S, S)).astype(np.float32)
    g = soc.grid_from_workload(ctx, P.grid)
    table = soc.temp_table_build(ctx, P.emit_nu, P.emit_w, P.emit_sigma_abs, P.T_floor, P.T_max, 4096)
    got = soc.surrogate_apply(ctx, g, table, S, torch.from_numpy(pred).cuda(), 0.2, 0.0,
                              torch.from_numpy(T1).cuda()).cpu().numpy()
    rng = np.random.default_rng(11)
    cells = list(rng.integers(0, n ** 3, 2000)) + [0, n - 1, n * n - 1, n ** 3 - 1, n ** 3 - n]
    dens = P.grid.density()
    wts = so._axis_weights(n, S)
    for c in cells:
        x, y, z = c % n, (c // n) % n, c // (n * n)
        if dens[c] == 0:
            assert got[c] == 0.0
            continue
        v = 0.0
        (z0, z1, tz), (y0, y1, ty), (x0, x1, tx) = wts[z], wts[y], wts[x]
        for zi, wz in ((z0, 1 - tz), (z1, tz)):
            for yi, wy in ((y0, 1 - ty), (y1, ty)):
                for xi, wx in ((x0, 1 - tx), (x1, tx)):
                    v += wz * wy * wx * float(pred[zi, yi, xi])
        want = np.clip(max(float(T1[c]), P.T_floor) * 10 ** (0.2 * v), P.T_floor, P.T_max)
        assert got[c] == pytest.approx(want, rel=2e-6)


def test_errors(soc, ctx):
    P = _problem(16, 1, seed=1)
    T1 = torch.from_numpy(_T1(P, seed=1)).cuda()
    g = soc.grid_from_workload(ctx, P.grid)
    table = soc.temp_table_build(ctx, P.emit_nu, P.emit_w, P.emit_sigma_abs, P.T_floor, P.T_max, 4096)
    with pytest.raises(soc.SocError, match="divide"):
        soc.surrogate_features(ctx, g, table, 5, P.w, P.sigma_abs, P.I_bg, W.SIGMA_V, P.ps_pos, P.ps_Lnu, T1)
    with pytest.raises(soc.SocError, match="outside"):
        soc.surrogate_features(ctx, g, table, 8, P.w, P.sigma_abs, P.I_bg, W.SIGMA_V, P.ps_pos + 100.0,
                               P.ps_Lnu, T1)
    with pytest.raises(soc.SocError, match="external field"):
        soc.surrogate_features(ctx, g, table, 8, P.w, P.sigma_abs, 0 * P.I_bg, W.SIGMA_V, P.ps_pos, P.ps_Lnu, T1)
    with pytest.raises(soc.SocError, match="scale"):
        soc.surrogate_target(ctx, g, table, 8, T1, T1, 0.0)
    with pytest.raises(soc.SocError, match="channel"):   # channel 2 of 2: refused before any launch
        ctx.check(soc._lib.soc_surrogate_target(ctx.h, g.h, table.h, 8, soc.C.c_void_p(T1.data_ptr()),
                                                soc.C.c_void_p(T1.data_ptr()), 1.0, soc.C.c_void_p(T1.data_ptr()),
                                                2, 2))
    G = W.octree_from_function(4, 4, 4, 2, 1e17, lambda L, lo, size: lo[:, 0] > 2,
                               lambda lo, size: np.ones(lo.shape[0]))
    go = soc.grid_from_workload(ctx, G)
    To = torch.zeros(G.ncells, dtype=torch.float32, device="cuda")
    with pytest.raises(soc.SocError, match="cubic"):
        soc.surrogate_apply(ctx, go, table, 2, torch.zeros(8, device="cuda"), 1.0, 0.0, To)
