"""soc_simulate_frequencies (every frequency of a pass in one persistent
launch) against the same work done by one soc_simulate_frequency call per
frequency: the packages draw the same random numbers, so the counters are
identical and the frequency-integrated absorbed energy equal up to FP64
summation order.  Covered: constant sources (field and point sources),
luminosity-weighted dust emission with and without the per-cell cap,
uniform dust emission, the reference-field correction (mode 2, its
per-frequency reference blended in place), frequencies with different
package counts, a call that mixes these setups, the diagonal-ALI tallies,
an octree, K = 1, and the argument errors.  The
iteration drivers run on top of it (tests/test_gpu_driver.py,
tests/test_gpu_reference.py)."""
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


def _freqs(P):
    return [(float(P.nu[k]), float(P.w[k]), float(P.sigma_abs[k]), float(P.sigma_sca[k]), float(P.g[k]))
            for k in range(P.K)]


def _both(soc, ctx, g, ncells, freqs, sources, ks, seed, iteration, copies=None):
    """(A, stats) of the single calls and of the multi-frequency call."""
    A1 = torch.zeros(ncells, dtype=torch.float64, device="cuda")
    tot = None
    for f, q, k in zip(freqs, sources, ks):
        st = soc.simulate_frequency(ctx, g, f, A1, seed=seed, iteration=iteration, freq_index=k, stats=True, **q)
        tot = st if tot is None else {key: tot[key] + st[key] for key in tot}
    A2 = torch.zeros(ncells, dtype=torch.float64, device="cuda")
    st2 = soc.simulate_frequencies(ctx, g, freqs, A2, sources, ks, seed=seed, iteration=iteration, stats=True)
    return A1.cpu().numpy(), tot, A2.cpu().numpy(), st2


def _check(a1, s1, a2, s2):
    for key in ("packages", "cell_steps", "scatterings", "runaways"):
        assert s2[key] == s1[key], key
    for key in ("e_emitted", "e_absorbed", "e_escaped"):
        assert s2[key] == pytest.approx(s1[key], rel=1e-11, abs=1e-300), key
    assert s1["packages"] > 0
    np.testing.assert_allclose(a2, a1, rtol=1e-11, atol=1e-12 * np.abs(a1).max())


@pytest.fixture(scope="module")
def cloud():
    P = W.lognormal_problem(n=24, K=12, sigma_ln=1.0, tau_v_mean=5.0, seed=7, L_star_lsun=1e5,
                            packages_per_freq=30000)
    rng = np.random.default_rng(3)
    T = rng.uniform(10.0, 60.0, P.grid.ncells).astype(np.float32)
    T[P.grid.density() == 0] = 0.0
    return P, torch.from_numpy(T).cuda()


@pytest.mark.parametrize("copies", [1, 0])
def test_constant_sources(soc, ctx, cloud, copies):
    P, _ = cloud
    saved = ctx.get_option("xcd_copies")
    ctx.set_option("xcd_copies", copies)
    try:
        g = soc.grid_from_workload(ctx, P.grid)
        src = [dict(I_bg=float(P.I_bg[k]), ps_pos=P.ps_pos, ps_Lnu=P.ps_Lnu[:, k], n_bg=6000 + 100 * k,
                    n_ps_pk=2000 + 37 * k) for k in range(P.K)]
        _check(*_both(soc, ctx, g, P.grid.ncells, _freqs(P), src, list(range(P.K)), 11, 1))
    finally:
        ctx.set_option("xcd_copies", saved)


@pytest.mark.parametrize("cap,spread", [(0.0, 1), (8.0, 1), (0.0, 0)])
def test_weighted_dust_emission(soc, ctx, cloud, cap, spread):
    """Both orders in which the waves take the frequencies (option
    multi_spread) give the same counters and tallies."""
    P, T = cloud
    saved = ctx.get_option("multi_spread")
    ctx.set_option("multi_spread", spread)
    try:
        g = soc.grid_from_workload(ctx, P.grid)
        src = [dict(T=T, n_dust=20000 + 1001 * k, dust_mode=1, dust_cap=cap) for k in range(P.K)]
        _check(*_both(soc, ctx, g, P.grid.ncells, _freqs(P), src, list(range(P.K)), 12, 4))
    finally:
        ctx.set_option("multi_spread", saved)


def test_uniform_dust_emission_and_subset_of_frequencies(soc, ctx, cloud):
    """Mode 0 at three frequencies given out of order (their indices)."""
    P, T = cloud
    g = soc.grid_from_workload(ctx, P.grid)
    ks = [9, 2, 5]
    fr = [_freqs(P)[k] for k in ks]
    src = [dict(T=T, n_dust=P.grid.ncells * (2 + i), dust_mode=0) for i in range(3)]
    _check(*_both(soc, ctx, g, P.grid.ncells, fr, src, ks, 13, 2))


def test_reference_field_correction(soc, ctx, cloud):
    """Mode 2: each frequency emits the signed difference to its own
    reference emission, which the call blends in place."""
    P, T = cloud
    g = soc.grid_from_workload(ctx, P.grid)
    gen = torch.Generator(device="cuda").manual_seed(4)
    L0 = torch.rand((P.K, P.grid.ncells), dtype=torch.float64, device="cuda", generator=gen) * 1e30
    outs = []
    for multi in (False, True):
        L = L0.clone()
        src = [dict(T=T, n_dust=15000, dust_mode=2, L_ref=L[k], ref_beta=0.3) for k in range(P.K)]
        A = torch.zeros(P.grid.ncells, dtype=torch.float64, device="cuda")
        if multi:
            st = soc.simulate_frequencies(ctx, g, _freqs(P), A, src, list(range(P.K)), seed=14, iteration=3,
                                          stats=True)
        else:
            st = None
            for k in range(P.K):
                s = soc.simulate_frequency(ctx, g, _freqs(P)[k], A, seed=14, iteration=3, freq_index=k, stats=True,
                                           **src[k])
                st = s if st is None else {key: st[key] + s[key] for key in st}
        outs.append((A.cpu().numpy(), st, L.cpu().numpy()))
    (a1, s1, l1), (a2, s2, l2) = outs
    _check(a1, s1, a2, s2)
    np.testing.assert_array_equal(l2, l1)


def test_octree_and_single_frequency(soc, ctx):
    G = W.octree_lognormal(n_root=8, nlevels=3, sigma_ln=1.2, seed=5)
    nu, w = W.frequency_grid(6)
    sabs, ssca, gg = W.dust_model(nu)
    freqs = [(float(nu[k]), float(w[k]), float(sabs[k]), float(ssca[k]), float(gg[k])) for k in range(6)]
    g = soc.grid_from_workload(ctx, G)
    I = W.isrf(nu)
    src = [dict(I_bg=float(I[k]), ps_pos=[[4.1, 3.9, 4.05]], ps_Lnu=[1e21], n_bg=5000, n_ps_pk=3000) for k in range(6)]
    _check(*_both(soc, ctx, g, G.ncells, freqs, src, list(range(6)), 15, 1))
    _check(*_both(soc, ctx, g, G.ncells, freqs[2:3], src[2:3], [2], 16, 1))


def test_mixed_dust_setups(soc, ctx, cloud):
    """One call whose frequencies mix the weighted mode without a cap
    (their tables are built together for all of them), the capped mode and
    constant sources only (built one frequency at a time), on the regular
    cloud and on an octree (the luminosity of refined levels)."""
    P, T = cloud
    g = soc.grid_from_workload(ctx, P.grid)
    kinds = [dict(T=T, n_dust=18000 + 700 * k, dust_mode=1) if k % 3 == 0 else
             dict(T=T, n_dust=16000, dust_mode=1, dust_cap=6.0) if k % 3 == 1 else
             dict(I_bg=float(P.I_bg[k]), n_bg=5000) for k in range(P.K)]
    _check(*_both(soc, ctx, g, P.grid.ncells, _freqs(P), kinds, list(range(P.K)), 18, 5))
    G = W.octree_lognormal(n_root=8, nlevels=3, sigma_ln=1.2, seed=6)
    go = soc.grid_from_workload(ctx, G)
    rng = np.random.default_rng(8)
    To = rng.uniform(10.0, 60.0, G.ncells).astype(np.float32)
    To[G.density() == 0] = 0.0
    Td = torch.from_numpy(To).cuda()
    src = [dict(T=Td, n_dust=12000 + 300 * k, dust_mode=1) for k in range(P.K)]
    _check(*_both(soc, ctx, go, G.ncells, _freqs(P), src, list(range(P.K)), 19, 5))


@pytest.mark.parametrize("copies", [1, 0])
def test_ali_tallies(soc, ctx, cloud, copies):
    """Diagonal ALI in one launch: the absorbed energy, the self-absorption
    and the emitted-energy tallies equal those of one call per frequency."""
    P, T = cloud
    saved = ctx.get_option("xcd_copies")
    ctx.set_option("xcd_copies", copies)
    try:
        g = soc.grid_from_workload(ctx, P.grid)
        out = []
        for multi in (False, True):
            A = torch.zeros(P.grid.ncells, dtype=torch.float64, device="cuda")
            S = torch.zeros_like(A)
            E = torch.zeros_like(A)
            src = [dict(T=T, n_dust=20000 + 501 * k, dust_mode=1, ali_self=S, ali_emitted=E) for k in range(P.K)]
            if multi:
                st = soc.simulate_frequencies(ctx, g, _freqs(P), A, src, list(range(P.K)), seed=17, iteration=2,
                                              stats=True)
            else:
                st = None
                for k in range(P.K):
                    s = soc.simulate_frequency(ctx, g, _freqs(P)[k], A, seed=17, iteration=2, freq_index=k,
                                               stats=True, **src[k])
                    st = s if st is None else {key: st[key] + s[key] for key in st}
            out.append((A.cpu().numpy(), st, S.cpu().numpy(), E.cpu().numpy()))
        (a1, s1, S1, E1), (a2, s2, S2, E2) = out
        _check(a1, s1, a2, s2)
        assert np.abs(S1).max() > 0 and np.abs(E1).max() > 0
        np.testing.assert_allclose(S2, S1, rtol=1e-11, atol=1e-12 * np.abs(S1).max())
        np.testing.assert_allclose(E2, E1, rtol=1e-11, atol=1e-12 * np.abs(E1).max())
    finally:
        ctx.set_option("xcd_copies", saved)


def test_errors(soc, ctx, cloud):
    P, T = cloud
    g = soc.grid_from_workload(ctx, P.grid)
    A = torch.zeros(P.grid.ncells, dtype=torch.float64, device="cuda")
    S, E = torch.zeros_like(A), torch.zeros_like(A)
    with pytest.raises(soc.SocError, match="same ALI tallies"):
        soc.simulate_frequencies(ctx, g, _freqs(P)[:2], A, [dict(T=T, n_dust=100, dust_mode=1, ali_self=S,
                                                               ali_emitted=E), dict(T=T, n_dust=100, dust_mode=1)],
                                 [0, 1])
    with pytest.raises(soc.SocError, match="frequency 1"):
        soc.simulate_frequencies(ctx, g, _freqs(P)[:2], A, [dict(I_bg=1.0, n_bg=10), dict(I_bg=-1.0, n_bg=10)],
                                 [0, 1])
    with pytest.raises(ValueError):
        soc.simulate_frequencies(ctx, g, _freqs(P)[:2], A, [dict(I_bg=1.0, n_bg=10)], [0, 1])
    assert float(A.abs().sum()) == 0.0
