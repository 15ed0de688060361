"""GPU parity of the stochastically heated grain solver (Sect. 2.1.1,
Appendix A) through the C ABI against the FP64 oracle: populations and
emission per cell on regular and octree grids, weak fields (nearly all
grains in the lowest bin) to strong ones (targets above the top bin), the
production-size model, the energy balance of the output, error paths."""
import math

import numpy as np
import pytest

from oracle import shg_oracle as O
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


def _cells(grid, G, rng, lo=-3.0, hi=4.0):
    """Absorbed energy per band [K, ncells] of cells in the synthetic field
    scaled by 10^U(lo, hi) and reddened by a random optical depth."""
    rho = grid.density().astype(np.float64)
    lev = np.zeros(grid.ncells, int)
    for L in range(grid.nlevels):
        lev[grid.level_offset[L]:grid.level_offset[L + 1]] = L
    V = (grid.root_cell_cm * 0.5 ** lev) ** 3
    scale = 10 ** rng.uniform(lo, hi, grid.ncells)
    tau = rng.uniform(0.0, 3.0, grid.ncells)
    red = np.exp(-np.outer(G.sigma_per_H / G.sigma_per_H.max(), tau))
    A = 4 * math.pi * W.isrf(G.nu)[:, None] * scale[None, :] * red * (G.sigma_per_H * G.w)[:, None] * (rho * V)[None, :]
    return rho, V, A


@pytest.mark.parametrize("kind", ["regular", "octree"])
def test_shg_matches_oracle(soc, ctx, kind):
    nu, w = W.frequency_grid(32)
    G = W.grain_model(nu, w, n_size=4, n_enthalpy=48)
    rng = np.random.default_rng(5)
    d = rng.uniform(0.5, 2.0, (3, 4, 5)).astype(np.float32)
    d[1, 2, 3] = 0.0
    grid = W.regular_grid(d, 1.0e17) if kind == "regular" else W.refine_all_once(W.regular_grid(d[:2, :2, :3], 2e17))
    rho, V, A = _cells(grid, G, rng)
    E_o, P_o = O.shg_solve(G, rho, V, A)
    g = soc.grid_from_workload(ctx, grid)
    model = soc.ShgModel(ctx, G)
    Ad = torch.from_numpy(A).cuda()
    E = torch.full_like(Ad, -1.0)
    P = torch.full((grid.ncells, 4, 48), -1.0, dtype=torch.float64, device="cuda")
    soc.shg_solve(ctx, g, model, Ad, E, P)
    e, p = E.cpu().numpy(), P.cpu().numpy()
    leaf = rho > 0
    np.testing.assert_allclose(p[leaf], P_o[leaf], rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(e, E_o, rtol=1e-9, atol=1e-12 * np.abs(E_o).max())
    assert not e[:, ~leaf].any() and not p[~leaf].any()
    # weak and strong cells both present
    assert P_o[leaf][:, 0, 0].max() > 0.5 and P_o[leaf][:, 0, 0].min() < 1e-3
    model.close()


def test_shg_production_size_and_energy_balance(soc, ctx):
    """8 sizes, 128 enthalpy bins, 64 frequencies on 16 cells: the oracle's
    emission to 1e-9; and the emitted power sum_k E_k w_k of cells in a
    strong field equals the absorbed power (the grains' lowest bin then
    holds nothing and no target passes the top)."""
    nu, w = W.frequency_grid(64)
    G = W.grain_model(nu, w)
    rng = np.random.default_rng(7)
    grid = W.regular_grid(rng.uniform(0.5, 2.0, (2, 2, 4)).astype(np.float32), 1.0e17)
    rho, V, A = _cells(grid, G, rng, lo=1.0, hi=3.0)
    E_o, P_o = O.shg_solve(G, rho, V, A)
    g = soc.grid_from_workload(ctx, grid)
    model = soc.ShgModel(ctx, G)
    E = torch.zeros(A.shape, dtype=torch.float64, device="cuda")
    soc.shg_solve(ctx, g, model, torch.from_numpy(A).cuda(), E)
    e = E.cpu().numpy()
    np.testing.assert_allclose(e, E_o, rtol=1e-9, atol=1e-12 * np.abs(E_o).max())
    emitted = (e * G.w[:, None]).sum(axis=0)
    absorbed = A.sum(axis=0)
    assert P_o[:, :, 0].max() < 1e-4
    np.testing.assert_allclose(emitted, absorbed, rtol=1e-6)
    model.close()


def test_shg_error_paths(soc, ctx):
    nu, w = W.frequency_grid(16)
    G = W.grain_model(nu, w, n_size=2, n_enthalpy=8)
    G.U[1, 3] = G.U[1, 2]
    with pytest.raises(soc.SocError, match="increase"):
        soc.ShgModel(ctx, G)
    G2 = W.grain_model(nu, w, n_size=2, n_enthalpy=200)
    with pytest.raises(soc.SocError, match="enthalpy grid"):
        soc.ShgModel(ctx, G2)


def test_shg_from_monte_carlo_spectra(soc, ctx):
    """The whole chain on a small cloud: one Monte Carlo pass per frequency
    into its own row (driver.absorbed_spectra, the grain model's cross
    sections), then the grain solve.  The rows sum to the frequency-integrated
    absorption of the same packages, and the emission from these Monte Carlo
    spectra (empty cells, reddened and unreddened cells, the point sources'
    neighbourhood) matches the oracle's solve of the same arrays to 1e-9."""
    import dataclasses

    from paper_1812_06632_amd.driver import absorbed_spectra
    P0 = W.lognormal_problem(n=10, K=16, sigma_ln=1.0, tau_v_mean=4.0, seed=4, L_star_lsun=1e3,
                             packages_per_freq=20000)
    G = W.grain_model(P0.nu, P0.w, n_size=4, n_enthalpy=48)
    P = dataclasses.replace(P0, sigma_abs=G.sigma_per_H, emit_sigma_abs=G.sigma_per_H)
    g = soc.grid_from_workload(ctx, P.grid)
    A = absorbed_spectra(ctx, g, P, seed=3)
    integ = torch.zeros(P.grid.ncells, dtype=torch.float64, device="cuda")
    have_ps = len(P.ps_pos) > 0
    for k in range(P.K):
        f = (float(P.nu[k]), float(P.w[k]), float(P.sigma_abs[k]), float(P.sigma_sca[k]), float(P.g[k]))
        soc.simulate_frequency(ctx, g, f, integ, I_bg=float(P.I_bg[k]), ps_pos=P.ps_pos if have_ps else None,
                               ps_Lnu=P.ps_Lnu[:, k] if have_ps else None, n_bg=P.n_bg,
                               n_ps_pk=P.n_ps_pk if have_ps else 0, seed=3, iteration=1, freq_index=k)
    a = A.cpu().numpy()
    np.testing.assert_allclose(a.sum(axis=0), integ.cpu().numpy(), rtol=1e-11, atol=0)
    assert (a > 0).mean() > 0.9
    model = soc.ShgModel(ctx, G)
    E = torch.zeros_like(A)
    soc.shg_solve(ctx, g, model, A, E)
    rho = P.grid.density().astype(np.float64)
    V = np.full(P.grid.ncells, P.grid.root_cell_cm ** 3)
    E_o, _ = O.shg_solve(G, rho, V, a)
    np.testing.assert_allclose(E.cpu().numpy(), E_o, rtol=1e-9, atol=1e-12 * np.abs(E_o).max())
    model.close()
