"""Host-side parts of the learned-start pipeline (no GPU): block averages,
network inputs and targets, the training-cloud family."""
import math

import numpy as np
import pytest

from paper_1812_06632_amd import workloads as W

surrogate = pytest.importorskip("paper_1812_06632_amd.surrogate")


def test_block_mean_is_the_mean_over_blocks():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((8, 8, 8))
    m = surrogate.block_mean(a, 4)
    assert m.shape == (4, 4, 4)
    assert m[1, 2, 3] == pytest.approx(a[2:4, 4:6, 6:8].mean())
    assert m.mean() == pytest.approx(a.mean())
    with pytest.raises(ValueError):
        surrogate.block_mean(a, 3)


def test_features_optical_depth_and_source_flux():
    P = W.lognormal_problem(n=32, K=8, packages_per_freq=1000)
    T1 = np.full(P.grid.ncells, 20.0)
    X = surrogate.features(P, 16, T1)
    assert X.shape == (16, 16, 16, 4) and X.dtype == np.float32
    # channel 0: log10 of the 0.55 um optical depth of a 2^3 block, / 2
    rho = P.grid.density().reshape(32, 32, 32).astype(np.float64)
    tau = W.SIGMA_V * rho[0:2, 2:4, 4:6].mean() * P.grid.root_cell_cm * 2
    assert X[0, 1, 2, 0] == pytest.approx(math.log10(tau + 1e-4) / 2, rel=1e-5)
    # channel 1: log10(1 + source flux / external 4 pi J) / 4, largest at the sources
    for (px, py, pz) in P.ps_pos:
        bx, by, bz = int(px // 2), int(py // 2), int(pz // 2)
        assert X[bz, by, bx, 1] == pytest.approx(X[..., 1].max(), rel=0.3)
    Lbol = (P.ps_Lnu * P.w[None, :]).sum(axis=1)
    cell = P.grid.root_cell_cm * 2
    c = np.array([0.5, 0.5, 0.5])                      # block (0, 0, 0)
    d2 = [((np.asarray(p) / 2 - c) ** 2).sum() + 0.25 for p in P.ps_pos]
    ratio = sum(L / (4 * math.pi * d * cell * cell) for L, d in zip(Lbol, d2)) / (4 * math.pi * W.isrf_integral())
    assert X[0, 0, 0, 1] == pytest.approx(math.log10(1 + ratio) / 4, rel=1e-4)
    assert X[0, 0, 0, 1] > 0.1    # a 10^6 L_sun source still dominates the corner of the box
    # no sources: channel 1 vanishes
    P.ps_pos = np.zeros((0, 3))
    P.ps_Lnu = np.zeros((0, 8))
    assert np.all(surrogate.features(P, 16, T1)[..., 1] == 0)


def test_targets_are_block_log_ratios_with_empty_cells_neutral():
    P = W.lognormal_problem(n=16, K=8, packages_per_freq=1000)
    rng = np.random.default_rng(2)
    T1 = rng.uniform(10.0, 50.0, P.grid.ncells)
    T = T1 * 1.25
    Y = surrogate.targets(P, T, T1, 8)
    assert Y.shape == (8, 8, 8, 1)
    rho = P.grid.density().reshape(16, 16, 16)
    lr = np.where(rho > 0, math.log10(1.25), 0.0)     # empty cells sit at the floor on both sides
    assert np.allclose(Y[..., 0], surrogate.block_mean(lr, 8))
    # the fourth input channel carries the block mean of log10 T1
    X = surrogate.features(P, 8, T1)
    lt1 = np.where(rho > 0, np.log10(T1.reshape(16, 16, 16)), math.log10(P.T_floor))
    assert np.allclose(X[..., 3], (surrogate.block_mean(lt1, 8) - 1.5) / 0.5, atol=1e-6)


def test_training_family_ranges():
    rng = np.random.default_rng(3)
    for _ in range(6):
        P = surrogate.random_problem(rng, n=16, K=8, packages=4000)
        rho = P.grid.density().reshape(16, 16, 16).astype(np.float64)
        # mean face-to-face optical depth within the family's range
        tau = W.SIGMA_V * P.grid.root_cell_cm * np.mean([rho.sum(axis=a).mean() for a in range(3)])
        lo, hi = surrogate.TAU_RANGE
        assert lo * 0.7 <= tau <= hi * 1.3
        assert len(P.ps_pos) <= 2
        if len(P.ps_pos):
            assert P.n_bg + len(P.ps_pos) * P.n_ps_pk <= 4000
            Lbol = (P.ps_Lnu * P.w[None, :]).sum(axis=1) / W.L_SUN
            assert np.all((Lbol > 0.5e5) & (Lbol < 2e7))
        else:
            assert P.n_bg == 4000 and P.n_ps_pk == 0


def test_thin_temperature_balances_absorption_and_emission():
    """The optically thin temperature solves 4 pi sum w sigma (B(T) - J) = 0:
    for the external field alone it is one value everywhere, it rises
    towards a point source, and the balance holds at the returned T."""
    P = W.lognormal_problem(n=16, K=32, packages_per_freq=1000)
    X = surrogate.features(P, 8, np.full(P.grid.ncells, 20.0))
    T = 10 ** (X[..., 2].astype(np.float64) * 0.5 + 1.5)
    J = P.I_bg[None, :]
    ws = P.w * P.sigma_abs
    T1 = surrogate.thin_temperature(P, J @ ws)[0]     # external field alone
    assert 5.0 < T1 < 50.0
    assert T.min() > T1                                # the sources only add heating
    for (px, py, pz) in P.ps_pos:
        assert T[int(pz // 2), int(py // 2), int(px // 2)] > 2 * T.min()
    bal = (surrogate._planck(P.nu, np.array([T1])) @ ws)[0] / (J @ ws)[0]
    assert bal == pytest.approx(1.0, rel=2e-3)
    P.ps_pos = np.zeros((0, 3))
    P.ps_Lnu = np.zeros((0, 32))
    X0 = surrogate.features(P, 8, np.full(P.grid.ncells, 20.0))
    assert np.ptp(X0[..., 2]) < 1e-6
    assert 10 ** (float(X0[0, 0, 0, 2]) * 0.5 + 1.5) == pytest.approx(T1, rel=1e-5)
