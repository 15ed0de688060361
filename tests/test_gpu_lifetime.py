"""Object lifetimes across the C ABI: a grid and a temperature table may be
destroyed after the context that created them (the header allows either
order).  Their destroy calls use only the device id recorded at creation;
an earlier version read the destroyed context and crashed at interpreter
exit, when Python happened to collect the context first."""
import numpy as np
import pytest

from paper_1812_06632_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_grid_and_table_destroyed_after_their_context():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1812_06632_amd import soc
    P = W.sphere_problem(n=8, n_packages=2000)
    ctx = soc.Context(0)
    g = soc.grid_from_workload(ctx, P.grid)
    t = soc.temp_table_build(ctx, P.emit_nu, P.emit_w, P.emit_sigma_abs, P.T_floor, P.T_max, 256)
    A = torch.zeros(P.grid.ncells, dtype=torch.float64, device="cuda")
    f = (float(P.nu[0]), float(P.w[0]), float(P.sigma_abs[0]), float(P.sigma_sca[0]), float(P.g[0]))
    soc.simulate_frequency(ctx, g, f, A, I_bg=float(P.I_bg[0]), n_bg=P.n_bg, seed=3)
    T = torch.zeros(P.grid.ncells, dtype=torch.float32, device="cuda")
    soc.update_temperature(ctx, g, t, A, T)
    torch.cuda.synchronize()
    # the context goes first, bypassing the wrapper's children-first order
    ctx._children.discard(g)
    ctx._children.discard(t)
    ctx.close()
    g.close()
    t.close()
    torch.cuda.synchronize()
    assert np.isfinite(T.cpu().numpy()).all() and float(A.sum()) > 0
