"""Point sources on cell faces, edges and octant planes.  A position on a
face belongs to the cell the package's direction points into (the oracle
finds the cell of the position pushed a tiny step along the direction);
without that rule the kernels took a zero-length step for every package
that starts on a face heading backwards, which shows in the step count.
Same seed as the oracle: identical packages, cell steps and scatterings
to near-tie level, FP64 traces segment for segment."""
import numpy as np
import pytest

from oracle import orc
from paper_1812_06632_amd import workloads as W
from tests.parity_util import compare_trace

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


NU, WN = W.frequency_grid(4)
SABS, SSCA, GG = W.dust_model(NU)
FREQ = (float(NU[2]), float(WN[2]), float(SABS[2]), float(SSCA[2]), float(GG[2]))


def _check(soc, ctx, grid, pos):
    g = soc.grid_from_workload(ctx, grid)
    kw = dict(ps_pos=pos, ps_Lnu=[1e22] * len(pos), n_ps_pk=100000, seed=21, iteration=1, freq_index=2)
    A = torch.zeros(grid.ncells, dtype=torch.float64, device="cuda")
    sg = soc.simulate_frequency(ctx, g, FREQ, A, stats=True, **kw)
    Ao, so, _ = orc.simulate_frequency(grid, FREQ, nthreads=16, **kw)
    print(f"\nsteps gpu {sg['cell_steps']} oracle {so['cell_steps']}")
    assert sg["packages"] == so["packages"] == 100000 * len(pos)
    assert abs(sg["cell_steps"] - so["cell_steps"]) <= 1e-4 * so["cell_steps"]
    assert abs(sg["scatterings"] - so["scatterings"]) <= 1e-4 * so["scatterings"] + 2
    ids = np.arange(0, 100000, 500).astype(np.uint32)
    for s in range(len(pos)):
        segs, nseg = soc.trace_packages(ctx, g, FREQ, soc.CLASS_PS0 + s, ids, precision=1, max_seg=4096, **kw)
        for i, pid in enumerate(ids):
            o = orc.trace_package(grid, FREQ, soc.CLASS_PS0 + s, int(pid), max_seg=4096, **kw)
            assert nseg[i] > 0 and segs[i][0]["ds"] > 0.0, (s, int(pid))   # no zero-length first step
            assert compare_trace(segs[i][: nseg[i]], o, rtol=1e-9, atol=1e-12)[0], (s, int(pid))


def test_regular_grid_face_edge_corner(soc, ctx):
    rho = W.grf_lognormal(24, 1.0, 4)
    s_cm = W.PC_CM / 24.0
    rho *= 3.0 / (W.SIGMA_V * s_cm * 24 * rho.mean())
    G = W.regular_grid(rho.astype(np.float32), s_cm)
    _check(soc, ctx, G, [[12.3, 11.0, 7.6], [12.0, 11.0, 7.4], [6.0, 9.0, 15.0]])


def test_octree_root_face_and_octant_planes(soc, ctx):
    G = W.octree_lognormal(n_root=8, nlevels=3, sigma_ln=1.2, seed=5)
    _check(soc, ctx, G, [[4.0, 3.5, 4.25], [4.3, 4.5, 3.75]])
