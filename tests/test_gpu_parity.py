"""GPU parity tests: the HIP library (through its C ABI) against the FP64
CPU oracle on the same seeded inputs.

  * deterministic traces: same Philox numbers on both sides, so every
    package follows the same cells; FP64 mode to 1e-9, FP32 production
    arithmetic to the tolerances derived in the design notes;
  * per-cell absorbed energy: same-seed agreement and, with independent
    seeds, z-scores against the combined Monte Carlo error (32 batches
    per side, cells with > 10^3 oracle hits);
  * energy conservation, temperatures (0.05 K), maps (1e-5 relative);
  * edge cases and error paths of the ABI.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import orc
from paper_1812_06632_amd import workloads as W
from tests.parity_util import check_z, compare_structure, compare_trace

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


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def _freq_of(P, k):
    return (float(P.nu[k]), float(P.w[k]), float(P.sigma_abs[k]), float(P.sigma_sca[k]), float(P.g[k]))


def _k_at(P, lam_um):
    """Index of the frequency closest to wavelength lam_um (frequencies
    are stored in increasing order, i.e. decreasing wavelength)."""
    lam = 2.99792458e14 / P.nu
    return int(np.argmin(np.abs(np.log(lam / lam_um))))


@pytest.fixture(scope="module")
def sphere():
    return W.sphere_problem(n=32, n_packages=100_000)


@pytest.fixture(scope="module")
def cloud():
    """Small lognormal cloud with two point sources and dust emission."""
    P = W.lognormal_problem(n=24, K=16, sigma_ln=1.0, tau_v_mean=5.0, seed=7, L_star_lsun=1e5,
                            packages_per_freq=40000)
    rng = np.random.default_rng(3)
    T = rng.uniform(10.0, 60.0, P.grid.ncells).astype(np.float32)
    T[P.grid.density() == 0] = 0.0
    return P, T


# ------------------------------------------------------------------ traces
def _trace_both(soc, ctx, grid_h, grid, freq, cls, ids, precision, **kw):
    segs, nseg = soc.trace_packages(ctx, grid_h, freq, cls, ids, precision=precision, max_seg=4096, **kw)
    out = []
    for i, pid in enumerate(ids):
        o = orc.trace_package(grid, freq, cls, int(pid), max_seg=4096, **kw)
        assert nseg[i] <= 4096 and len(o) <= 4096
        out.append(compare_trace(segs[i][: nseg[i]], o, rtol=1e-9 if precision == 1 else 2e-5,
                                 atol=1e-12 if precision == 1 else 2e-5))
    return out


def test_traces_fp64_mode_match_oracle_exactly(soc, ctx, sphere):
    """FP64 instantiation of the production step code follows the oracle
    segment for segment (cells, events, lengths to 1e-9)."""
    P = sphere
    g = soc.grid_from_workload(ctx, P.grid)
    f = _freq_of(P, 0)
    ids = np.arange(0, 100_000, 100)
    res = _trace_both(soc, ctx, g, P.grid, f, soc.CLASS_BG, ids, 1, I_bg=P.I_bg[0], n_bg=P.n_bg)
    ok = [r[0] for r in res]
    assert all(ok), f"{len(ok) - sum(ok)} of {len(ok)} FP64 traces differ"
    assert max(r[3] for r in res) < 1e-12


def test_traces_fp32_production_match_oracle(soc, ctx, sphere):
    """FP32 production arithmetic: packages follow the oracle's cells and
    events; path lengths agree to 1e-6 relative; segment lengths drift by
    at most 1e-3 cell (FP32 rounding of positions and directions
    accumulated over the walk).  A package may leave the oracle's cell
    sequence only at a near-tie of two events."""
    P = sphere
    g = soc.grid_from_workload(ctx, P.grid)
    f = _freq_of(P, 0)
    ids = np.arange(0, 100_000, 50).astype(np.uint32)
    kw = dict(I_bg=P.I_bg[0], n_bg=P.n_bg)
    segs, nseg = soc.trace_packages(ctx, g, f, soc.CLASS_BG, ids, precision=0, max_seg=4096, **kw)
    res = [compare_structure(segs[i][: nseg[i]], orc.trace_package(P.grid, f, soc.CLASS_BG, int(pid), max_seg=4096,
                                                                    **kw)) for i, pid in enumerate(ids)]
    same = np.array([r[0] for r in res])
    path = np.array([r[3] for r in res if r[0]])
    drift = np.array([r[2] for r in res if r[0]])
    print(f"\nFP32 traces: {same.mean():.4f} same cells/events, path rel err median {np.median(path):.2e} "
          f"p99 {np.quantile(path, 0.99):.2e} max {path.max():.2e}; max segment drift {drift.max():.2e}")
    assert same.mean() >= 0.99
    assert np.quantile(path, 0.99) < 1e-6
    assert drift.max() < 1e-3


@pytest.mark.parametrize("cls_name", ["bg", "ps0", "ps1", "dust_weighted", "dust_uniform"])
def test_traces_all_source_classes(soc, ctx, cloud, cls_name):
    P, T = cloud
    g = soc.grid_from_workload(ctx, P.grid)
    k = _k_at(P, 0.55)   # optical: albedo and g ~ 0.4
    f = _freq_of(P, k)
    assert f[3] > 0 and f[4] > 0.1
    Td = _dev(T, torch.float32)
    n = {"bg": 2000, "ps0": 1000, "ps1": 1000, "dust_weighted": 3000, "dust_uniform": P.grid.ncells * 2}
    cls = {"bg": soc.CLASS_BG, "ps0": soc.CLASS_PS0, "ps1": soc.CLASS_PS0 + 1, "dust_weighted": soc.CLASS_DUST,
           "dust_uniform": soc.CLASS_DUST}[cls_name]
    mode = 0 if cls_name == "dust_uniform" else 1
    kw = dict(I_bg=P.I_bg[k], ps_pos=P.ps_pos, ps_Lnu=P.ps_Lnu[:, k], n_bg=2000, n_ps_pk=1000,
              n_dust=n["dust_weighted"] if mode else n["dust_uniform"], dust_mode=mode, seed=11, iteration=2,
              freq_index=k)
    ids = np.arange(0, n[cls_name], max(1, n[cls_name] // 300)).astype(np.uint32)
    segs, nseg = soc.trace_packages(ctx, g, f, cls, ids, precision=1, max_seg=4096, T=Td, **kw)
    bad = 0
    for i, pid in enumerate(ids):
        o = orc.trace_package(P.grid, f, cls, int(pid), max_seg=4096, T=T, **kw)
        r = compare_trace(segs[i][: nseg[i]], o, rtol=1e-9, atol=1e-12)
        bad += not r[0]
    assert bad == 0, f"{bad} of {len(ids)} traces differ ({cls_name})"


# ------------------------------------------------------------------ tallies
def _gpu_run(soc, ctx, g, ncells, f, seed, **kw):
    A = torch.zeros(ncells, dtype=torch.float64, device="cuda")
    st = soc.simulate_frequency(ctx, g, f, A, seed=seed, stats=True, **kw)
    return A.cpu().numpy(), st


def test_same_seed_tallies_and_conservation(soc, ctx, sphere):
    """Same seed: identical package set; totals agree (packages exactly,
    cell steps and scatterings to near-tie level), per-cell absorbed energy
    agrees closely, and both sides conserve energy."""
    P = sphere
    g = soc.grid_from_workload(ctx, P.grid)
    f = _freq_of(P, 0)
    n = 1_000_000
    Ag, sg = _gpu_run(soc, ctx, g, P.grid.ncells, f, 5, I_bg=P.I_bg[0], n_bg=n)
    hits = np.zeros(P.grid.ncells, np.int64)
    Ao, so, _ = orc.simulate_frequency(P.grid, f, I_bg=P.I_bg[0], n_bg=n, seed=5, nthreads=16, hits=hits)
    assert sg["packages"] == so["packages"] == n
    assert abs(sg["cell_steps"] - so["cell_steps"]) <= 1e-4 * so["cell_steps"]
    assert abs(sg["scatterings"] - so["scatterings"]) <= 1e-4 * so["scatterings"]
    assert sg["e_emitted"] == pytest.approx(so["e_emitted"], rel=1e-10, abs=0)   # FP64 atomic summation order
    cons = (Ag.sum() + sg["e_escaped"]) / sg["e_emitted"] - 1.0
    assert abs(cons) < 1e-6
    assert sg["e_absorbed"] == pytest.approx(Ag.sum(), rel=1e-9, abs=0)
    sel = hits > 1000
    assert sel.sum() > 1000
    rel = np.abs(Ag[sel] - Ao[sel]) / Ao[sel]
    print(f"\nsame-seed per-cell rel diff: median {np.median(rel):.2e} max {rel.max():.2e} over {sel.sum()} cells")
    assert np.median(rel) < 1e-4 and rel.max() < 1e-2


def test_statistical_parity_independent_seeds(soc, ctx, sphere):
    """32 independent batches per side: per-cell z-scores of the GPU mean
    against the oracle mean are N(0,1) and the mean relative bias is below
    0.3% over cells with > 10^3 hits."""
    P = sphere
    g = soc.grid_from_workload(ctx, P.grid)
    f = _freq_of(P, 0)
    B = 32
    n = 50_000
    gb = [_gpu_run(soc, ctx, g, P.grid.ncells, f, 1000 + b, I_bg=P.I_bg[0], n_bg=n)[0] for b in range(B)]
    hits = np.zeros(P.grid.ncells, np.int64)
    ob = []
    for b in range(B):
        A, _, _ = orc.simulate_frequency(P.grid, f, I_bg=P.I_bg[0], n_bg=n, seed=5000 + b, nthreads=8,
                                         hits=hits if b == 0 else None)
        ob.append(A)
    check_z(gb, ob, hits, "sphere")


def test_cloud_all_sources_statistical_and_conservation(soc, ctx, cloud):
    """Background + two point sources + weighted dust emission on a
    lognormal cloud: energy conserved on the GPU, per-cell z-scores against
    the oracle with independent seeds."""
    P, T = cloud
    g = soc.grid_from_workload(ctx, P.grid)
    k = _k_at(P, 0.55)
    f = _freq_of(P, k)
    Td = _dev(T, torch.float32)
    kw = dict(I_bg=P.I_bg[k], ps_pos=P.ps_pos, ps_Lnu=P.ps_Lnu[:, k], n_bg=32000, n_ps_pk=16000, n_dust=32000,
              dust_mode=1, iteration=2, freq_index=k)
    B = 32
    gb, ob = [], []
    hits = np.zeros(P.grid.ncells, np.int64)
    for b in range(B):
        A, st = _gpu_run(soc, ctx, g, P.grid.ncells, f, 100 + b, T=Td, **kw)
        assert abs((A.sum() + st["e_escaped"]) / st["e_emitted"] - 1) < 1e-6
        gb.append(A)
        Ao, so, _ = orc.simulate_frequency(P.grid, f, T=T, seed=900 + b, nthreads=8,
                                           hits=hits if b == 0 else None, **kw)
        ob.append(Ao)
        assert st["e_emitted"] == pytest.approx(so["e_emitted"], rel=1e-9, abs=0)
    check_z(gb, ob, hits, "cloud, all sources")


def test_launch_configuration_independence(soc, ctx, cloud):
    """A package's random numbers depend only on its identity: any block
    size, occupancy, refill threshold, inner-step count, or shared versus
    per-XCD accumulation gives the same tallies up to FP64 summation order,
    and identical counters (repeated per-XCD runs also check that every
    fold left the private copies zero)."""
    P, T = cloud
    g = soc.grid_from_workload(ctx, P.grid)
    k = _k_at(P, 2.0)
    f = _freq_of(P, k)
    Td = _dev(T, torch.float32)
    kw = dict(I_bg=P.I_bg[k], ps_pos=P.ps_pos, ps_Lnu=P.ps_Lnu[:, k], n_bg=5000, n_ps_pk=3000, n_dust=7001,
              dust_mode=1, T=Td, iteration=1, freq_index=k)
    ref, sref = _gpu_run(soc, ctx, g, P.grid.ncells, f, 77, **kw)
    saved = {n: ctx.get_option(n) for n in ("block", "blocks_per_cu", "refill_min", "inner_steps", "scatter_min",
                                            "xcd_copies", "chunk")}
    try:
        for cfg in ({"block": 64, "blocks_per_cu": 1}, {"block": 512, "blocks_per_cu": 2},
                    {"refill_min": 32, "inner_steps": 7}, {"refill_min": 64, "inner_steps": 8},
                    {"scatter_min": 24}, {"scatter_min": 64, "inner_steps": 3},
                    {"xcd_copies": 0}, {"xcd_copies": 0, "block": 128}, {"xcd_copies": 1, "block": 192},
                    {"chunk": 64}, {"chunk": 64, "refill_min": 16}, {"chunk": 4096}):
            for n_, v in cfg.items():
                ctx.set_option(n_, v)
            A, st = _gpu_run(soc, ctx, g, P.grid.ncells, f, 77, **kw)
            for key in ("packages", "cell_steps", "scatterings", "runaways"):
                assert st[key] == sref[key], (cfg, key)
            np.testing.assert_allclose(A, ref, rtol=1e-11, atol=1e-30 + 1e-12 * ref.max())
            for n_, v in saved.items():
                ctx.set_option(n_, v)
    finally:
        for n_, v in saved.items():
            ctx.set_option(n_, v)


# ------------------------------------------------------------------ temperature
def test_temperature_parity(soc, ctx, cloud):
    """Same absorbed energies on both sides: temperatures within 0.05 K
    (typically 1e-3 K); statistics agree."""
    P, T = cloud
    g = soc.grid_from_workload(ctx, P.grid)
    rng = np.random.default_rng(5)
    dens = P.grid.density().astype(np.float64)
    V = P.grid.root_cell_cm ** 3
    Ttrue = rng.uniform(3.0, 400.0, P.grid.ncells)
    A = np.array([orc.gamma(P.emit_nu, P.emit_w, P.emit_sigma_abs, t) for t in Ttrue]) * dens * V
    A[::97] = 0.0          # unhit cells
    A[5] = A[5] * 1e12     # beyond T_max
    table = soc.temp_table_build(ctx, P.emit_nu, P.emit_w, P.emit_sigma_abs, 2.0, 3000.0, 4096)
    Told = np.full(P.grid.ncells, 20.0, np.float32)
    Tg = torch.empty(P.grid.ncells, dtype=torch.float32, device="cuda")
    sg = soc.update_temperature(ctx, g, table, _dev(A, torch.float64), Tg, _dev(Told, torch.float32), stats=True)
    To, so = orc.update_temperature(P.grid, P.emit_nu, P.emit_w, P.emit_sigma_abs, A, T_old=Told)
    Tg = Tg.cpu().numpy()
    err = np.abs(Tg.astype(np.float64) - To)
    print(f"\nT max abs err {err.max():.3e} K")
    assert err.max() <= 0.05
    assert sg["clamped"] == so["clamped"]
    assert sg["mean_T"] == pytest.approx(so["mean_T"], rel=1e-6, abs=0)
    assert sg["hot5_mean_T"] == pytest.approx(so["hot5_mean_T"], rel=1e-3, abs=0)
    assert sg["mean_rel_change"] == pytest.approx(so["mean_rel_change"], rel=1e-5, abs=0)


# ------------------------------------------------------------------ map
@pytest.mark.parametrize("axis", [0, 1, 2, 2 | 4])
def test_map_parity(soc, ctx, cloud, axis):
    P, T = cloud
    g = soc.grid_from_workload(ctx, P.grid)
    f = _freq_of(P, _k_at(P, 250.0))   # far infrared, where 10-60 K dust emits
    img = soc.map_image(ctx, g, f, _dev(T, torch.float32), axis).cpu().numpy()
    ref = orc.map_image(P.grid, f, T, axis)
    assert img.shape == ref.shape
    np.testing.assert_allclose(img, ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max())


# ------------------------------------------------------------------ edges
def test_edge_cases(soc, ctx):
    """Empty grid (everything escapes), one package, one cell, a non-cubic
    box, zero packages, a ragged package count, step cap 1."""
    f = (1e13, 1.0, 0.3, 0.4, 0.2)
    for dens in (np.zeros((3, 5, 7), np.float32), np.full((1, 1, 1), 2.0, np.float32),
                 np.random.default_rng(1).uniform(0, 2, (3, 5, 7)).astype(np.float32)):
        G = W.regular_grid(dens, 1.0)
        g = soc.grid_from_workload(ctx, G)
        for n in (0, 1, 257, 12345):
            A, st = _gpu_run(soc, ctx, g, G.ncells, f, 3, I_bg=1.0, n_bg=n)
            Ao, so, _ = orc.simulate_frequency(G, f, I_bg=1.0, n_bg=n, seed=3)
            assert st["packages"] == n and so["packages"] == n
            assert abs(st["cell_steps"] - so["cell_steps"]) <= 1e-4 * max(so["cell_steps"], 1)
            if n:
                assert abs((A.sum() + st["e_escaped"]) / st["e_emitted"] - 1) < 1e-6
                np.testing.assert_allclose(A, Ao, rtol=1e-3, atol=1e-6 * max(Ao.max(), 1e-300))
    G = W.regular_grid(np.full((4, 4, 4), 1.0, np.float32), 1.0)
    g = soc.grid_from_workload(ctx, G)
    ctx.set_option("step_cap", 1)
    try:
        A, st = _gpu_run(soc, ctx, g, G.ncells, (1e12, 1.0, 0.2, 0.5, 0.0), 4, I_bg=1.0, n_bg=2000)
        Ao, so, _ = orc.simulate_frequency(G, (1e12, 1.0, 0.2, 0.5, 0.0), I_bg=1.0, n_bg=2000, seed=4, step_cap=1)
    finally:
        ctx.set_option("step_cap", 10_000_000)
    assert st["cell_steps"] == 2000 and st["runaways"] == so["runaways"] > 0
    assert abs((A.sum() + st["e_escaped"]) / st["e_emitted"] - 1) < 1e-6


def test_error_paths(soc, ctx):
    G = W.refine_all_once(W.regular_grid(np.ones((2, 2, 2), np.float32), 1.0))
    bad = G.words.copy()
    bad.view(np.int32)[0] = -(G.nroot + 3)
    with pytest.raises(soc.SocError) as e:
        soc.build_grid(ctx, G.nx, G.ny, G.nz, G.nlevels, G.level_offset, 1.0,
                       torch.from_numpy(bad.view(np.int32).copy()).cuda())
    assert e.value.status == soc.EGRID
    dens = np.ones((2, 2, 2), np.float32)
    dens[0, 0, 0] = np.nan
    with pytest.raises(soc.SocError) as e:
        soc.grid_from_workload(ctx, W.Grid(2, 2, 2, 1, np.array([0, 8]), 1.0, dens.view(np.uint32).ravel()))
    assert e.value.status == soc.EGRID
    g = soc.grid_from_workload(ctx, W.regular_grid(np.ones((2, 2, 2), np.float32), 1.0))
    A = torch.zeros(8, dtype=torch.float64, device="cuda")
    for f in ((1e12, 1.0, 0.1, 0.1, 1.0), (1e12, 1.0, -0.1, 0.1, 0.0), (1e12, 1.0, float("nan"), 0.1, 0.0)):
        with pytest.raises(soc.SocError) as e:
            soc.simulate_frequency(ctx, g, f, A, I_bg=1.0, n_bg=10)
        assert e.value.status == soc.EINVAL
    T = torch.full((8,), 10.0, device="cuda")
    with pytest.raises(soc.SocError) as e:
        soc.simulate_frequency(ctx, g, (1e12, 1.0, 0.1, 0.1, 0.0), A, T=T, n_dust=9, dust_mode=0)
    assert e.value.status == soc.EINVAL
    with pytest.raises(soc.SocError):
        soc.simulate_frequency(ctx, g, (1e12, 1.0, 0.1, 0.1, 0.0), A, ps_pos=[[5.0, 0.5, 0.5]], ps_Lnu=[1.0],
                               n_ps_pk=4)
