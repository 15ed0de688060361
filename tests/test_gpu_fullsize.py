"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (the library's default schedule; no launch
option is changed here).

Workloads:
  * the 128^3 lognormal benchmark cloud: 64 frequencies, 10^6 packages per
    frequency, the external field and two 10^4 K point sources;
  * the octree cloud: 64^3 root cells with three refinement levels (4.68 M
    leaves), a central dense core, a 10^4 K source inside the core and the
    external field.

Same-seed comparisons with the oracle.  Both sides draw the same packages,
so they should agree:
  * package counts exactly;
  * cell steps and scatterings to the near-tie level (FP32 positions
    against FP64);
  * emitted energy to 1e-10;
  * energy conserved on both sides;
  * per-cell tallies closely over the well-sampled cells.

Passes compared:
  * the constant sources at optical, mid- and far-infrared frequencies;
  * the luminosity-weighted dust emission at the temperatures the GPU
    solves from the constant sources (the first dust iteration);
  * on the octree, 10^6 packages at 0.55 and 250 um.

Independent seeds, 32 batches per side (per-cell z-scores and relative
bias over the cells with > 10^3 hits):
  * the benchmark cloud's luminosity-weighted dust emission at 10 um,
    10^5 packages per batch;
  * the octree at 0.55 um, external field and the embedded source,
    5 x 10^4 packages each per batch.

Further checks:
  * a GPU pass with the full 10^7 packages per frequency on the octree
    conserves energy and emits the oracle's total;
  * the temperature update on sampled cells, against the oracle's solve of
    the same absorbed energies (strips of the sampled cells with their
    level's cell size).
"""
import numpy as np
import pytest

from oracle import orc
from paper_1812_06632_amd import workloads as W
from tests.parity_util import check_z

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


def _k_at(nu, lam_um):
    lam = 2.99792458e14 / np.asarray(nu)
    return int(np.argmin(np.abs(np.log(lam / lam_um))))


def _same_seed(soc, ctx, g, grid, f, label, **kw):
    """One pass on both sides with the same seed; returns the GPU tally."""
    A = torch.zeros(grid.ncells, dtype=torch.float64, device="cuda")
    kw_gpu = dict(kw)
    if isinstance(kw_gpu.get("T"), np.ndarray):
        kw_gpu["T"] = torch.from_numpy(kw_gpu["T"]).cuda()
    sg = soc.simulate_frequency(ctx, g, f, A, stats=True, **kw_gpu)
    Ag = A.cpu().numpy()
    hits = np.zeros(grid.ncells, np.int64)
    Ao, so, _ = orc.simulate_frequency(grid, f, nthreads=16, hits=hits, **kw)
    assert sg["packages"] == so["packages"]
    assert abs(sg["cell_steps"] - so["cell_steps"]) <= 1e-4 * so["cell_steps"]
    assert abs(sg["scatterings"] - so["scatterings"]) <= 1e-4 * so["scatterings"] + 2
    assert sg["e_emitted"] == pytest.approx(so["e_emitted"], rel=1e-10, abs=0)
    assert abs((Ag.sum() + sg["e_escaped"]) / sg["e_emitted"] - 1.0) < 1e-6
    assert abs((Ao.sum() + so["e_escaped"]) / so["e_emitted"] - 1.0) < 1e-9
    assert sg["e_absorbed"] == pytest.approx(Ag.sum(), rel=1e-9, abs=0)
    # well-sampled cells: > 1000 depositing segments where there are enough
    # of them (emission spread over all cells gives ~60 per cell), and
    # always > 100
    sel100 = hits > 100
    assert sel100.sum() > 1000
    rel100 = np.abs(Ag[sel100] - Ao[sel100]) / Ao[sel100]
    sel = hits > 1000
    msg = f"\n{label}: {so['packages']} packages, {so['cell_steps']:.3e} steps; per-cell rel diff over " \
          f"{sel100.sum()} cells with > 100 hits: median {np.median(rel100):.2e}"
    if sel.sum() >= 100:
        rel = np.abs(Ag[sel] - Ao[sel]) / Ao[sel]
        msg += f"; over {sel.sum()} cells with > 1000 hits: median {np.median(rel):.2e} p99 {np.quantile(rel, 0.99):.2e}"
        assert np.median(rel) < 1e-4 and np.quantile(rel, 0.99) < 1e-2
    print(msg)
    assert np.median(rel100) < 1e-3
    return Ag


def _temperature_sample(grid, cells, level_of, emit, A, T_gpu, rng_seed, n=5000):
    """Oracle temperatures of sampled cells (strips of cells of one level
    with that level's cell size) against the GPU's; max |dT|."""
    emit_nu, emit_w, emit_sabs, T_floor, T_max = emit
    rng = np.random.default_rng(rng_seed)
    rho = grid.density()
    worst = 0.0
    for L in np.unique(level_of[cells]):
        pool = cells[level_of[cells] == L]
        pick = rng.choice(pool, size=min(n, pool.size), replace=False)
        strip = W.regular_grid(rho[pick].astype(np.float32).reshape(1, 1, -1), grid.root_cell_cm * 0.5 ** int(L))
        To, _ = orc.update_temperature(strip, emit_nu, emit_w, emit_sabs, A[pick], T_floor=T_floor, T_max=T_max)
        worst = max(worst, float(np.abs(To - T_gpu[pick]).max()))
    return worst


# ------------------------------------------------------------------ 128^3 benchmark cloud
@pytest.fixture(scope="module")
def bench_cloud(soc, ctx):
    """The benchmark workload and the GPU's constant-source solution (the
    state a first dust iteration starts from)."""
    from paper_1812_06632_amd.driver import PlainSolver
    P = W.lognormal_problem()
    S = PlainSolver(ctx, P, seed=1)
    S.constant_pass()
    torch.cuda.synchronize()
    return P, S


@pytest.mark.parametrize("lam_um", [0.55, 10.0, 250.0])
def test_benchmark_cloud_constant_sources_same_seed(soc, ctx, bench_cloud, lam_um):
    P, S = bench_cloud
    k = _k_at(P.nu, lam_um)
    _same_seed(soc, ctx, S.grid, P.grid, S.freqs[k], f"128^3 constant sources, {lam_um} um", I_bg=float(P.I_bg[k]),
               ps_pos=P.ps_pos, ps_Lnu=P.ps_Lnu[:, k], n_bg=P.n_bg, n_ps_pk=P.n_ps_pk, seed=5, iteration=1,
               freq_index=k)


@pytest.mark.parametrize("lam_um", [10.0, 250.0])
def test_benchmark_cloud_dust_emission_same_seed(soc, ctx, bench_cloud, lam_um):
    P, S = bench_cloud
    k = _k_at(P.nu, lam_um)
    T = S.T.cpu().numpy()
    assert (T[P.grid.density() > 0] > 2.0).mean() > 0.99
    _same_seed(soc, ctx, S.grid, P.grid, S.freqs[k], f"128^3 dust emission, {lam_um} um", T=T, n_dust=P.n_dust,
               dust_mode=1, seed=9, iteration=2, freq_index=k)


def test_benchmark_cloud_dust_emission_independent_seeds(soc, ctx, bench_cloud):
    """32 independent batches per side of the weighted dust emission at
    10 um (10^5 packages each) at the constant-source temperatures: per-cell
    z-scores and relative bias over the well-sampled cells."""
    P, S = bench_cloud
    k = _k_at(P.nu, 10.0)
    T = S.T.cpu().numpy()
    kw = dict(n_dust=100_000, dust_mode=1, iteration=2, freq_index=k)
    B = 32
    gb, ob = [], []
    hits = np.zeros(P.grid.ncells, np.int64)
    for b in range(B):
        A = torch.zeros(P.grid.ncells, dtype=torch.float64, device="cuda")
        soc.simulate_frequency(ctx, S.grid, S.freqs[k], A, T=S.T, seed=2000 + b, **kw)
        gb.append(A.cpu().numpy())
    for b in range(B):
        Ao, _, _ = orc.simulate_frequency(P.grid, S.freqs[k], T=T, seed=7000 + b, nthreads=16,
                                          hits=hits if b == 0 else None, **kw)
        ob.append(Ao)
    check_z(gb, ob, hits, "128^3 dust emission at 10 um, independent seeds")


def test_benchmark_cloud_temperature_sample(soc, ctx, bench_cloud):
    P, S = bench_cloud
    A = S.A_const.cpu().numpy()
    T = S.T.cpu().numpy()
    cells = np.flatnonzero(P.grid.density() > 0)
    worst = _temperature_sample(P.grid, cells, np.zeros(P.grid.ncells, np.int64),
                                (P.emit_nu, P.emit_w, P.emit_sigma_abs, P.T_floor, P.T_max), A, T, 3, n=20000)
    print(f"\n128^3 temperatures, 20000 sampled cells: max |dT| {worst:.3e} K")
    assert worst <= 0.05


# ------------------------------------------------------------------ octree cloud
@pytest.fixture(scope="module")
def octree_cloud(soc, ctx):
    G = W.octree_lognormal(n_root=64, nlevels=4)
    nu, w = W.frequency_grid(128)
    sabs, ssca, gg = W.dust_model(nu)
    g = soc.grid_from_workload(ctx, G)
    level = np.zeros(G.ncells, np.int64)
    for L in range(G.nlevels):
        level[G.level_offset[L]:G.level_offset[L + 1]] = L
    return G, g, nu, w, sabs, ssca, gg, level


def _octree_sources(nu, k):
    return dict(I_bg=float(W.isrf(nu[k:k + 1])[0]), ps_pos=[[32.1, 31.9, 32.05]],
                ps_Lnu=[float(W.blackbody_Lnu(nu[k:k + 1], 1e6 * W.L_SUN, 1e4)[0])])


def test_octree_structure_at_full_size(soc, ctx, octree_cloud):
    G, g, *_ = octree_cloud
    leaves = int((G.words.view(np.int32) >= 0).sum())
    assert G.nlevels == 4 and (G.level_offset[1] == 64 ** 3)
    assert g.n_leaves == leaves and 4.0e6 < leaves < 6.0e6


@pytest.mark.parametrize("lam_um", [0.55, 250.0])
def test_octree_same_seed(soc, ctx, octree_cloud, lam_um):
    G, g, nu, w, sabs, ssca, gg, _ = octree_cloud
    k = _k_at(nu, lam_um)
    f = (float(nu[k]), float(w[k]), float(sabs[k]), float(ssca[k]), float(gg[k]))
    _same_seed(soc, ctx, g, G, f, f"octree, {lam_um} um", n_bg=500_000, n_ps_pk=500_000, seed=5, iteration=1,
               freq_index=k, **_octree_sources(nu, k))


def test_octree_independent_seeds(soc, ctx, octree_cloud):
    """32 independent batches per side at 0.55 um (external field and the
    embedded source, 5 x 10^4 packages each per batch): per-cell z-scores
    and relative bias over the well-sampled leaves."""
    G, g, nu, w, sabs, ssca, gg, _ = octree_cloud
    k = _k_at(nu, 0.55)
    f = (float(nu[k]), float(w[k]), float(sabs[k]), float(ssca[k]), float(gg[k]))
    kw = dict(n_bg=50_000, n_ps_pk=50_000, iteration=1, freq_index=k, **_octree_sources(nu, k))
    B = 32
    gb, ob = [], []
    hits = np.zeros(G.ncells, np.int64)
    for b in range(B):
        A = torch.zeros(G.ncells, dtype=torch.float64, device="cuda")
        soc.simulate_frequency(ctx, g, f, A, seed=2000 + b, **kw)
        gb.append(A.cpu().numpy())
    for b in range(B):
        Ao, _, _ = orc.simulate_frequency(G, f, seed=7000 + b, nthreads=16, hits=hits if b == 0 else None, **kw)
        ob.append(Ao)
    check_z(gb, ob, hits, "octree at 0.55 um, independent seeds")


def test_octree_full_package_count_and_temperatures(soc, ctx, octree_cloud):
    """10^7 packages at 0.55 um (the configuration's count): every package
    accounted for, energy conserved, the oracle's emitted total; then the
    temperature update of the result on sampled leaves of every level."""
    G, g, nu, w, sabs, ssca, gg, level = octree_cloud
    k = _k_at(nu, 0.55)
    f = (float(nu[k]), float(w[k]), float(sabs[k]), float(ssca[k]), float(gg[k]))
    src = _octree_sources(nu, k)
    A = torch.zeros(G.ncells, dtype=torch.float64, device="cuda")
    st = soc.simulate_frequency(ctx, g, f, A, n_bg=5_000_000, n_ps_pk=5_000_000, seed=8, iteration=1, freq_index=k,
                                stats=True, **src)
    Ag = A.cpu().numpy()
    assert st["packages"] == 10_000_000 and st["runaways"] == 0
    assert abs((Ag.sum() + st["e_escaped"]) / st["e_emitted"] - 1.0) < 1e-6
    _, so, _ = orc.simulate_frequency(G, f, n_bg=1000, n_ps_pk=1000, seed=8, iteration=1, freq_index=k, nthreads=4,
                                      **src)
    assert st["e_emitted"] == pytest.approx(so["e_emitted"], rel=1e-9, abs=0)
    refined = G.words.view(np.int32) < 0
    assert not Ag[refined].any()
    table = soc.temp_table_build(ctx, nu, w, sabs, 2.0, 3000.0, 4096)
    T = torch.zeros(G.ncells, dtype=torch.float32, device="cuda")
    soc.update_temperature(ctx, g, table, A, T, None)
    leaves = np.flatnonzero((~refined) & (G.density() > 0))
    worst = _temperature_sample(G, leaves, level, (nu, w, sabs, 2.0, 3000.0), Ag, T.cpu().numpy(), 4, n=5000)
    print(f"\noctree, 10^7 packages: {st['cell_steps']:.3e} steps, {st['scatterings']:.3e} scatterings; "
          f"temperatures of 5000 sampled leaves per level: max |dT| {worst:.3e} K")
    assert worst <= 0.05


# ------------------------------------------------------------------ batch of 256 clouds
def test_batch_of_256_clouds_at_full_size(soc, ctx):
    """The batched workload as the benchmark runs it: 256 lognormal clouds of
    16^3-96^3 cells, 32 frequencies, 10^5-10^6 packages per (cloud,
    frequency) pair, tiles of 16384 packages.  Sampled clouds equal the
    sum of their 32 single soc_simulate_frequency calls with the batch's
    seeds, up to FP64 summation order.  The pair with the most packages per
    cell against the oracle, same seed.  Energy is conserved over the whole
    batch."""
    grids, (nu, w, sabs, ssca, gg, I), pk = W.batch_clouds(256, 32)
    G = [soc.grid_from_workload(ctx, gr) for gr in grids]
    A = [torch.zeros(gr.ncells, dtype=torch.float64, device="cuda") for gr in grids]
    freqs = [(float(nu[k]), float(w[k]), float(sabs[k]), float(ssca[k]), float(gg[k])) for k in range(len(nu))]
    pairs = [dict(grid=m, freq=freqs[k], freq_index=k, I_bg=float(I[k]), n_bg=int(pk[m, k]), absorbed=A[m])
             for m in range(len(grids)) for k in range(len(nu))]
    seed = 0x5eed_0000_0001
    b = soc.Batch(ctx, G, pairs, seed=seed, tile_packages=16384)
    st = b.run(iteration=4, stats=True)
    b.close()
    assert st["packages"] == int(pk.sum()) and st["runaways"] == 0
    assert abs((st["e_absorbed"] + st["e_escaped"]) / st["e_emitted"] - 1.0) < 1e-6
    rng = np.random.default_rng(11)
    sample = sorted(rng.choice(len(grids), size=6, replace=False).tolist() + [int(np.argmax([g.ncells for g in grids]))])
    for m in sample:
        ref = torch.zeros(grids[m].ncells, dtype=torch.float64, device="cuda")
        for k in range(len(nu)):
            soc.simulate_frequency(ctx, G[m], freqs[k], ref, I_bg=float(I[k]), n_bg=int(pk[m, k]),
                                   seed=seed ^ (m << 32), iteration=4, freq_index=k)
        a, r = A[m].cpu().numpy(), ref.cpu().numpy()
        np.testing.assert_allclose(a, r, rtol=1e-11, atol=1e-12 * r.max())
    # the oracle on the pair with the most packages per cell (well-sampled cells)
    dens = pk / np.array([gr.ncells for gr in grids], dtype=np.float64)[:, None]
    m, k = (int(v) for v in np.unravel_index(int(np.argmax(dens)), dens.shape))
    print(f"\nbatch: {st['packages']} packages, {st['cell_steps']:.3e} steps; clouds {sample} equal their single calls")
    _same_seed(soc, ctx, G[m], grids[m], freqs[k], f"batch cloud {m} ({grids[m].nx}^3), frequency {k}", I_bg=float(I[k]),
               n_bg=int(pk[m, k]), seed=seed ^ (m << 32), iteration=4, freq_index=k)
