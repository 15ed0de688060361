"""A scattering cloud that (almost) does not absorb, in an isotropic
external field, keeps a uniform isotropic radiance equal to the field's,
whatever its scattering optical depth and phase function.  To first order
in k_abs every cell then absorbs 4 pi k_abs V I w, the optically thin
result: a closed form for the per-cell absorption of a scattering cloud,
tested here on the GPU kernels cell by cell (z-scores over 16 independent
seeds), on a regular grid and on an octree.  The oracle meets the same
closed form in tests/test_oracle_pins.py."""
import math

import numpy as np
import pytest

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


def _check(soc, ctx, grid, dens, vol, s_abs, s_sca, g_hg, area, n_bg):
    g = soc.grid_from_workload(ctx, grid)
    freq = (1e14, 1.0, s_abs, s_sca, g_hg)
    runs = []
    for seed in range(16):
        A = torch.zeros(grid.ncells, dtype=torch.float64, device="cuda")
        st = soc.simulate_frequency(ctx, g, freq, A, I_bg=1.0, n_bg=n_bg, seed=200 + seed, stats=True)
        assert st["e_emitted"] == pytest.approx(math.pi * area, rel=1e-12)
        assert st["scatterings"] > 2 * st["packages"]
        runs.append(A.cpu().numpy())
    R = np.array(runs)
    pred = 4 * math.pi * s_abs * dens * vol
    sel = pred > 0
    z = (R.mean(axis=0)[sel] - pred[sel]) / (R.std(axis=0, ddof=1)[sel] / math.sqrt(len(runs)))
    print(f"\nmax |z| {np.abs(z).max():.2f}, mean z {z.mean():.3f} over {z.size} cells")
    assert np.all(R[:, ~sel] == 0.0)
    assert np.all(np.abs(z) < 6.0)
    tot = R.sum(axis=1)   # the cells share packages: the total has its own spread
    print(f"total / closed form {tot.mean() / pred.sum():.6f} +- {tot.std(ddof=1) / math.sqrt(len(runs)) / pred.sum():.6f}")
    assert abs(tot.mean() - pred.sum()) < 4.5 * tot.std(ddof=1) / math.sqrt(len(runs))


@pytest.mark.parametrize("g_hg", [0.0, 0.6])
def test_regular_grid(soc, ctx, g_hg):
    rng = np.random.default_rng(12)
    rho = np.exp(rng.normal(0.0, 0.8, (6, 8, 10))).astype(np.float32)
    s_sca = 0.6 / float(rho.mean())
    grid = W.regular_grid(rho, 1.0)
    _check(soc, ctx, grid, rho.reshape(-1).astype(np.float64), 1.0, s_sca * 1e-6, s_sca, g_hg,
           2 * (48 + 60 + 80), 400000)


def test_octree(soc, ctx):
    """Refined cells take their level's volume; parents absorb nothing."""
    G = W.octree_lognormal(n_root=8, nlevels=3, sigma_ln=1.0, seed=4)
    dens = G.density().astype(np.float64)
    lv = np.zeros(G.ncells, np.int64)
    for L in range(1, G.nlevels):
        lv[G.level_offset[L]:] = L
    s = G.root_cell_cm
    vol = (s * 0.5 ** lv) ** 3
    nbar = float((dens * vol).sum() / vol[dens > 0].sum())
    s_sca = 0.6 / (nbar * s)   # mean scattering optical depth 0.6 per root cell
    _check(soc, ctx, G, dens, vol, s_sca * 1e-6, s_sca, 0.5, 6 * (8 * s) ** 2, 400000)
