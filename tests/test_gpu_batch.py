"""Batched persistent launch over many (cloud, frequency) pairs, and its
capture in a HIP graph."""
import numpy as np
import pytest

from oracle import orc
from paper_1812_06632_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def soc():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1812_06632_amd import soc as m
    return m


def _clouds():
    """Five lognormal clouds of uneven sizes (cubic and not), three
    frequencies each (optical, near-IR, far-IR)."""
    sizes = [(8, 8, 8), (12, 10, 9), (16, 16, 16), (5, 7, 11), (20, 12, 8)]
    grids = []
    for m, (nx, ny, nz) in enumerate(sizes):
        n = max(nx, ny, nz)
        rho = W.grf_lognormal(n, 1.0, 100 + m)[:nz, :ny, :nx]
        rho *= (2.0 + m) / (W.SIGMA_V * (W.PC_CM / n) * n * rho.mean())
        grids.append(W.regular_grid(rho.astype(np.float32), W.PC_CM / n))
    nu, w = W.frequency_grid(32)
    sabs, ssca, g = W.dust_model(nu)
    lam = 2.99792458e14 / nu
    ks = [int(np.argmin(np.abs(np.log(lam / l)))) for l in (0.55, 2.2, 100.0)]
    freqs = [(k, (float(nu[k]), float(w[k]), float(sabs[k]), float(ssca[k]), float(g[k])), float(W.isrf(nu[k:k + 1])[0]))
             for k in ks]
    return grids, freqs


def _pairs(grids, freqs, A, n_bg=3000):
    pairs = []
    for m in range(len(grids)):
        for (k, f, I) in freqs:
            q = dict(grid=m, freq=f, freq_index=k, I_bg=I, n_bg=n_bg + 37 * m, absorbed=A[m])
            if m == 2:
                q.update(ps_pos=[[8.5, 8.5, 8.5]], ps_Lnu=[1e20], n_ps_pk=1500)
            pairs.append(q)
    return pairs


@pytest.mark.parametrize("lds_cells,copies", [(None, 1), (0, 1), (1000, 1), (0, 0)])
def test_batch_equals_single_calls(soc, lds_cells, copies):
    """Pair (m, k) of a batch follows the same random numbers as a single
    soc_simulate_frequency call with seed ^ (m << 32): identical counters,
    identical absorbed energies up to FP64 summation order, for several
    tile sizes; with every grid tallied in LDS by whole-pair workgroups
    (the default: all five grids are small), none, or the grids of at most
    1000 cells (a mix of both phases in one launch).  Tiled grids with even
    dimensions are tallied in a brick-ordered scratch copy that is folded
    into their arrays after the launch (private copies on, copies 1), or
    straight into their arrays (copies 0)."""
    grids, freqs = _clouds()
    ctx = soc.Context(0)
    ctx.set_option("xcd_copies", copies)
    if lds_cells is not None:
        ctx.set_option("batch_lds_cells", lds_cells)
    assert ctx.get_option("batch_lds_cells") >= (lds_cells or 0)
    G = [soc.grid_from_workload(ctx, g) for g in grids]
    seed = 0x1234_0000_0042
    ref = [torch.zeros(g.ncells, dtype=torch.float64, device="cuda") for g in grids]
    ctx.read_stats(reset=True)
    tot = None
    for q in _pairs(grids, freqs, ref):
        st = soc.simulate_frequency(ctx, G[q["grid"]], q["freq"], q["absorbed"], I_bg=q["I_bg"], n_bg=q["n_bg"],
                                    ps_pos=q.get("ps_pos"), ps_Lnu=q.get("ps_Lnu"), n_ps_pk=q.get("n_ps_pk", 0),
                                    seed=seed ^ (q["grid"] << 32), iteration=3, freq_index=q["freq_index"], stats=True)
        tot = st if tot is None else {k: tot[k] + st[k] for k in tot}
    for tile in (64, 1000, 1 << 20):
        A = [torch.zeros(g.ncells, dtype=torch.float64, device="cuda") for g in grids]
        b = soc.Batch(ctx, G, _pairs(grids, freqs, A), seed=seed, tile_packages=tile)
        st = b.run(iteration=3, stats=True)
        for key in ("packages", "cell_steps", "scatterings", "runaways"):
            assert st[key] == tot[key], (tile, key)
        assert st["e_emitted"] == pytest.approx(tot["e_emitted"], rel=1e-12, abs=0)
        for m in range(len(grids)):
            a, r = A[m].cpu().numpy(), ref[m].cpu().numpy()
            np.testing.assert_allclose(a, r, rtol=1e-11, atol=1e-12 * r.max())
        b.close()
    ctx.close()


def test_batch_matches_oracle_counts(soc):
    """Same seed, same package set: the batch's per-model totals agree with
    the oracle (cell steps to near-tie level, energy conserved)."""
    grids, freqs = _clouds()
    ctx = soc.Context(0)
    G = [soc.grid_from_workload(ctx, g) for g in grids]
    A = [torch.zeros(g.ncells, dtype=torch.float64, device="cuda") for g in grids]
    pairs = _pairs(grids, freqs, A)
    b = soc.Batch(ctx, G, pairs, seed=9, tile_packages=512)
    st = b.run(iteration=1, stats=True)
    steps = 0
    absorbed = 0.0
    for q in pairs:
        Ao, so, _ = orc.simulate_frequency(grids[q["grid"]], q["freq"], I_bg=q["I_bg"], n_bg=q["n_bg"],
                                           ps_pos=q.get("ps_pos"), ps_Lnu=q.get("ps_Lnu"), n_ps_pk=q.get("n_ps_pk", 0),
                                           seed=9 ^ (q["grid"] << 32), iteration=1, freq_index=q["freq_index"],
                                           nthreads=8)
        steps += so["cell_steps"]
        absorbed += Ao.sum()
    assert abs(st["cell_steps"] - steps) <= 1e-4 * steps
    assert sum(a.sum().item() for a in A) == pytest.approx(absorbed, rel=1e-4, abs=0)
    assert abs((st["e_absorbed"] + st["e_escaped"]) / st["e_emitted"] - 1) < 1e-6
    ctx.close()


@pytest.mark.parametrize("lds_cells", [None, 0])
def test_batch_graph_replays_match_eager(soc, lds_cells):
    """Capture [zero the absorbed arrays, batch launch with an advancing
    iteration, temperature update of every model] in a HIP graph; every
    replay equals the eager computation of the same iteration (replays
    interleaved with eager work and synchronisations).  With every grid
    tiled (lds_cells 0) the graph also holds the fold of the brick-ordered
    scratch tallies."""
    grids, freqs = _clouds()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = soc.Context(0, stream=s)
        if lds_cells is not None:
            ctx.set_option("batch_lds_cells", lds_cells)
        G = [soc.grid_from_workload(ctx, g) for g in grids]
        nu, w = W.frequency_grid(32)
        sabs, _, _ = W.dust_model(nu)
        table = soc.temp_table_build(ctx, nu, w, sabs, 2.0, 3000.0, 1024)
        A = [torch.zeros(g.ncells, dtype=torch.float64, device="cuda") for g in grids]
        T = [torch.zeros(g.ncells, dtype=torch.float32, device="cuda") for g in grids]
        b = soc.Batch(ctx, G, _pairs(grids, freqs, A), seed=5, tile_packages=2048)
        Ae = [torch.zeros_like(a) for a in A]
        Te = [torch.zeros_like(t) for t in T]
        be = soc.Batch(ctx, G, _pairs(grids, freqs, Ae), seed=5, tile_packages=2048)
        b.run(iteration=0)   # iteration word starts at 0; the graph advances it
        torch.cuda.synchronize()
        soc.graph_begin(ctx)
        for a in A:
            a.zero_()
        b.run(iteration=soc.ITER_ADVANCE)
        for m in range(len(grids)):
            soc.update_temperature(ctx, G[m], table, A[m], T[m])
        graph = soc.graph_end(ctx)
        for it in (1, 2, 3):
            graph.launch()
            torch.cuda.synchronize()
            got_A = [a.cpu().numpy() for a in A]
            got_T = [t.cpu().numpy() for t in T]
            for a in Ae:
                a.zero_()
            be.run(iteration=it)
            for m in range(len(grids)):
                soc.update_temperature(ctx, G[m], table, Ae[m], Te[m])
            torch.cuda.synchronize()
            for m in range(len(grids)):
                r = Ae[m].cpu().numpy()
                np.testing.assert_allclose(got_A[m], r, rtol=1e-11, atol=1e-12 * r.max())
                np.testing.assert_allclose(got_T[m], Te[m].cpu().numpy(), rtol=1e-6)
        soc.graph_begin(ctx)
        with pytest.raises(soc.SocError) as e:
            b.run(iteration=1, stats=True)   # synchronising call refused while capturing
        assert e.value.status == soc.ESTATE
        try:
            soc.graph_end(ctx).close()
        except soc.SocError:
            pass
    ctx.close()


def test_batch_errors(soc):
    grids, freqs = _clouds()
    ctx = soc.Context(0)
    G = [soc.grid_from_workload(ctx, g) for g in grids[:2]]
    A = [torch.zeros(g.ncells, dtype=torch.float64, device="cuda") for g in grids[:2]]
    bad = _pairs(grids[:2], freqs, A)
    bad[0]["grid"] = 7
    with pytest.raises(soc.SocError) as e:
        soc.Batch(ctx, G, bad)
    assert e.value.status == soc.EINVAL
    oc = soc.grid_from_workload(ctx, W.refine_all_once(W.regular_grid(np.ones((2, 2, 2), np.float32), 1.0)))
    with pytest.raises(soc.SocError):
        soc.Batch(ctx, [oc], [dict(grid=0, freq=freqs[0][1], I_bg=1.0, n_bg=10,
                                   absorbed=torch.zeros(oc.ncells, dtype=torch.float64, device="cuda"))])
    with pytest.raises(soc.SocError, match="LDS"):
        ctx.set_option("batch_lds_cells", 1 << 30)   # more than any workgroup's LDS holds
    with pytest.raises(soc.SocError):
        ctx.set_option("batch_lds_cells", -1)
    ctx.close()


def test_autotuner_on_batch(soc, tmp_path):
    """The autotuner times candidate schedules of a batch on the device and
    returns one of them; every candidate gives the same counters."""
    from paper_1812_06632_amd import autotune
    grids, freqs = _clouds()
    ctx = soc.Context(0)
    G = [soc.grid_from_workload(ctx, g) for g in grids]
    A = [torch.zeros(g.ncells, dtype=torch.float64, device="cuda") for g in grids]
    b = soc.Batch(ctx, G, _pairs(grids, freqs, A), seed=3, tile_packages=1024)
    counts = []

    def run(cfg):
        st = b.run(iteration=1, stats=True)
        counts.append((st["packages"], st["cell_steps"], st["scatterings"]))

    space = {"block": (128, 256), "blocks_per_cu": (2, 8), "refill_min": (1, 32)}
    tu = autotune.Autotuner(str(tmp_path / "t.json"))
    best = tu.tune("batch:test", autotune.event_timer(ctx, run), space, repeats=1)
    assert best in list(autotune.candidates(space))
    assert len(set(counts)) == 1
    ctx.close()
