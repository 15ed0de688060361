"""Host-side part of the learned-start pipeline (no GPU): the family of
training clouds.  The network's input, target and output maps are library
kernels, checked against the oracle in tests/test_gpu_surrogate.py."""
import numpy as np
import pytest

from paper_1812_06632_amd import workloads as W

surrogate = pytest.importorskip("paper_1812_06632_amd.surrogate")


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
            assert P.ps_Lnu.shape == (0, 8)
