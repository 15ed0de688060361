"""The plain-iteration driver and the statistics of a given temperature
field."""
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


def test_given_field_statistics_equal_solve_statistics(soc):
    """soc_temperature_stats of the field a solve produced returns the
    solve's own mean and hottest-5% mean, bit for bit; zeros in the given
    field are tolerated."""
    P = W.lognormal_problem(n=32, K=16, packages_per_freq=20_000)
    ctx = soc.Context(0)
    g = soc.grid_from_workload(ctx, P.grid)
    table = soc.temp_table_build(ctx, P.emit_nu, P.emit_w, P.emit_sigma_abs, P.T_floor, P.T_max, 1024)
    rng = np.random.default_rng(1)
    # absorbed energies of temperatures spread over 8-200 K (input generator only)
    Tt = np.exp(rng.uniform(np.log(8.0), np.log(200.0), P.grid.ncells))
    h, k, c = 6.62607015e-27, 1.380649e-16, 2.99792458e10
    nu = P.emit_nu[None, :]
    B = 2 * h * nu ** 3 / c ** 2 / np.expm1(h * nu / (k * Tt[:, None]))
    gam = 4 * np.pi * (B * (P.emit_w * P.emit_sigma_abs)[None, :]).sum(1)
    A = torch.from_numpy(gam * P.grid.density() * P.grid.root_cell_cm ** 3).cuda()
    T = torch.zeros(P.grid.ncells, dtype=torch.float32, device="cuda")
    s1 = soc.update_temperature(ctx, g, table, A, T, None, stats=True)
    s2 = soc.temperature_stats(ctx, g, table, T)
    assert s1["mean_T"] == s2["mean_T"] and s1["hot5_mean_T"] == s2["hot5_mean_T"]
    T2 = T.clone()
    T2[::7] = 0.0
    s3 = soc.temperature_stats(ctx, g, table, T2)
    h = T2.cpu().numpy().astype(np.float64)[P.grid.density() > 0]
    assert s3["mean_T"] == pytest.approx(h.mean(), rel=1e-12, abs=0)
    k = int(np.ceil(0.05 * h.size))
    assert s3["hot5_mean_T"] == pytest.approx(np.sort(h)[-k:].mean(), rel=1e-9, abs=0)
    ctx.close()


def test_plain_solver_converges_and_restarts(soc):
    """The driver converges by the 1% rule on a small cloud; started again
    from its own converged field it stops after one dust iteration."""
    from paper_1812_06632_amd.driver import PlainSolver, converged
    P = W.lognormal_problem(n=32, K=16, packages_per_freq=50_000)
    ctx = soc.Context(0)
    S = PlainSolver(ctx, P)
    hist, at = S.run(max_iter=20)
    assert at is not None and at >= 3
    for (_, _, a), (_, _, b) in zip(hist[:-2], hist[1:-1]):
        assert not converged(a, b)
    T_conv = S.T.clone()
    hist2, at2 = S.run(max_iter=20, T0=T_conv)
    assert at2 == 2
    assert hist2[0][2]["mean_T"] == pytest.approx(hist[-1][2]["mean_T"], rel=1e-12, abs=0)
    ctx.close()
