"""Seeded synthetic inputs for the SOC hot path.

This module only builds input data: density grids in the hierarchical
encoding of Juvela (2019) Sect. 2.1.1 (one 32-bit word per cell, a refined
cell holding the negated index of its first child), frequency grids, dust
opacity tables, external-field and point-source spectra.  It holds none of
the Monte Carlo, temperature or map arithmetic, and both the GPU library
tests and the CPU oracle draw their inputs from here.

Workload shapes follow the paper where the configurations leave them open:
K log-spaced frequencies between 0.1 and 3000 um (Sect. 2.2), blackbody
point sources of 10^4 K placed in empty cells (Sect. 2.2, 3.1), and
lognormal clouds standing in for the MHD snapshot the paper used (Sect. 2.2),
which is not available.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# CODATA 2018 (cgs); used here only to build input spectra.
_H = 6.62607015e-27
_K = 1.380649e-16
_C = 2.99792458e10
_SIGMA_SB = 5.670374419e-5
PC_CM = 3.0856775814913673e18
L_SUN = 3.828e33
SIGMA_V = 5.0e-22          # extinction cross section at 0.55 um, cm^2 per H
LAMBDA_V_UM = 0.55
LAMBDA_BREAK_UM = 20.0     # UV-optical / FIR break of the synthetic dust


@dataclasses.dataclass
class Grid:
    """Cell vector of a regular (nlevels == 1) or octree grid.

    words[c] is the bit pattern of an FP32 density >= 0 (H cm^-3) or, read
    as int32, -(index of the first child of the octet) for a refined cell.
    Root cells come first with x fastest; child octant o = ix + 2 iy + 4 iz.
    """
    nx: int
    ny: int
    nz: int
    nlevels: int
    level_offset: np.ndarray   # int64[nlevels + 1]
    root_cell_cm: float
    words: np.ndarray          # uint32[ncells]

    @property
    def ncells(self) -> int:
        return int(self.words.shape[0])

    @property
    def nroot(self) -> int:
        return self.nx * self.ny * self.nz

    def is_link(self) -> np.ndarray:
        return self.words.view(np.int32) < 0

    def density(self) -> np.ndarray:
        """Densities as float32 (0 for refined cells)."""
        d = self.words.view(np.float32).copy()
        d[self.is_link()] = 0.0
        return d


def regular_grid(density_zyx: np.ndarray, root_cell_cm: float) -> Grid:
    """Regular grid from a (nz, ny, nx) density array."""
    d = np.ascontiguousarray(density_zyx, dtype=np.float32)
    if d.ndim != 3 or np.any(~np.isfinite(d)) or np.any(d < 0):
        raise ValueError("density must be a finite, non-negative 3-D array")
    nz, ny, nx = d.shape
    words = d.reshape(-1).view(np.uint32).copy()
    lo = np.array([0, nx * ny * nz], dtype=np.int64)
    return Grid(nx, ny, nz, 1, lo, float(root_cell_cm), words)


def refine_all_once(g: Grid) -> Grid:
    """Octree with every root cell of a regular grid refined into an octet of
    children with the parent's density (used by the octree equivalence pin:
    it describes the same medium as the regular grid of twice the
    resolution)."""
    if g.nlevels != 1:
        raise ValueError("expects a regular grid")
    n = g.nroot
    dens = g.words.view(np.float32)
    root = (-(n + 8 * np.arange(n, dtype=np.int64))).astype(np.int32).view(np.uint32)
    child = np.repeat(dens, 8).astype(np.float32).view(np.uint32)
    words = np.concatenate([root, child])
    lo = np.array([0, n, n + 8 * n], dtype=np.int64)
    return Grid(g.nx, g.ny, g.nz, 2, lo, g.root_cell_cm, words)


def octree_from_function(nx: int, ny: int, nz: int, nlevels: int, root_cell_cm: float,
                         refine, density) -> Grid:
    """Octree built top-down.  refine(level, lo_xyz[m,3], size) -> bool[m]
    decides which cells split; density(lo_xyz[m,3], size) -> float[m] gives
    leaf densities.  Levels are stored in order, octets consecutive."""
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lo = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    size = 1.0
    levels_words = []
    level_offset = [0]
    base = 0
    for L in range(nlevels):
        m = lo.shape[0]
        split = np.zeros(m, dtype=bool) if L == nlevels - 1 else np.asarray(refine(L, lo, size), dtype=bool)
        words = np.asarray(density(lo, size), dtype=np.float32).view(np.uint32).copy()
        nsplit = int(split.sum())
        next_base = base + m
        first = next_base + 8 * np.arange(nsplit, dtype=np.int64)
        words[split] = (-first).astype(np.int32).view(np.uint32)
        levels_words.append(words)
        level_offset.append(next_base)
        if nsplit == 0:
            break
        half = size / 2
        plo = lo[split]
        o = np.arange(8)
        offs = np.stack([(o & 1), (o >> 1) & 1, (o >> 2) & 1], axis=1).astype(np.float64) * half
        lo = (plo[:, None, :] + offs[None, :, :]).reshape(-1, 3)
        size = half
        base = next_base
    words = np.concatenate(levels_words)
    nl = len(levels_words)
    return Grid(nx, ny, nz, nl, np.array(level_offset[: nl + 1], dtype=np.int64), root_cell_cm, words)


def parent_links(g: Grid) -> np.ndarray:
    """Reverse links of Sect. 2.1.1: for every non-root octet, the index of
    its parent cell (int32[(ncells - nroot) / 8])."""
    n_oct = (g.ncells - g.nroot) // 8
    par = np.full(n_oct, -1, dtype=np.int32)
    w = g.words.view(np.int32)
    links = np.nonzero(w < 0)[0]
    par[(-w[links].astype(np.int64) - g.nroot) // 8] = links.astype(np.int32)
    return par


# ---------------------------------------------------------------- clouds
def grf_lognormal(n: int, sigma_ln: float, seed: int, slope: float = -3.0) -> np.ndarray:
    """Lognormal density exp(sigma_ln * delta - sigma_ln^2 / 2) of a periodic
    Gaussian random field delta with power spectrum P(k) ~ k^slope (P(0) = 0),
    normalised to unit variance.  Returns float64 (n, n, n), mean ~ 1."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    k = np.fft.fftfreq(n) * n
    kz, ky, kx = np.meshgrid(k, k, np.fft.rfftfreq(n) * n, indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = kk[nz] ** (slope / 2.0)
    field = np.fft.irfftn(np.fft.rfftn(white) * amp, s=(n, n, n), axes=(0, 1, 2))
    field -= field.mean()
    field /= field.std()
    return np.exp(sigma_ln * field - 0.5 * sigma_ln * sigma_ln)


def sphere_density(n: int, radius_cells: float, n0: float) -> np.ndarray:
    """Uniform sphere: cells whose centre lies within radius_cells of the box
    centre get density n0, the others 0.  Returns float32 (n, n, n)."""
    c = (np.arange(n) + 0.5) - n / 2.0
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    inside = x * x + y * y + z * z <= radius_cells * radius_cells
    return np.where(inside, n0, 0.0).astype(np.float32)


# ---------------------------------------------------------------- spectra
def frequency_grid(K: int, lam_min_um: float = 0.1, lam_max_um: float = 3000.0):
    """K frequencies log-spaced between lam_max and lam_min (Sect. 2.2) and
    trapezoid quadrature weights in ln(nu): w_k = nu_k dln(nu), halved at
    the two ends, so that sum_k w_k f(nu_k) approximates the integral of f
    over nu.  Returns (nu [Hz], w [Hz]) in increasing frequency."""
    nu_lo = _C / (lam_max_um * 1e-4)
    nu_hi = _C / (lam_min_um * 1e-4)
    if K == 1:
        return np.array([math.sqrt(nu_lo * nu_hi)]), np.array([nu_hi - nu_lo])
    lnu = np.linspace(math.log(nu_lo), math.log(nu_hi), K)
    nu = np.exp(lnu)
    d = lnu[1] - lnu[0]
    w = nu * d
    w[0] *= 0.5
    w[-1] *= 0.5
    return nu, w


def dust_model(nu: np.ndarray):
    """Synthetic dust: sigma_ext ~ nu^1 shortward of 20 um (normalised to
    SIGMA_V at 0.55 um); albedo and g fall from 0.6 at 0.1 um linearly in
    ln(lambda) to 0 at 20 um; longward of 20 um pure absorption with
    sigma_abs ~ nu^1.8, continuous at the break.  Returns float64
    (sigma_abs, sigma_sca, g) per frequency."""
    lam_um = _C / nu * 1e4
    nu_v = _C / (LAMBDA_V_UM * 1e-4)
    nu_b = _C / (LAMBDA_BREAK_UM * 1e-4)
    sext = SIGMA_V * (nu / nu_v)
    frac = np.clip(1.0 - np.log(lam_um / 0.1) / math.log(LAMBDA_BREAK_UM / 0.1), 0.0, 1.0)
    alb = 0.6 * frac
    g = 0.6 * frac
    sabs = (1.0 - alb) * sext
    ssca = alb * sext
    fir = lam_um > LAMBDA_BREAK_UM
    sabs_b = SIGMA_V * (nu_b / nu_v)
    sabs = np.where(fir, sabs_b * (nu / nu_b) ** 1.8, sabs)
    ssca = np.where(fir, 0.0, ssca)
    g = np.where(fir, 0.0, g)
    return sabs, ssca, g


def _bb(nu, T):
    x = _H * np.asarray(nu, dtype=np.float64) / (_K * T)
    return 2.0 * _H * nu ** 3 / _C ** 2 / np.expm1(np.minimum(x, 700.0))


# Diluted blackbodies (T [K], dilution) of the synthetic interstellar field
# standing in for the Mathis et al. (1983) field of Sect. 2.2, plus the CMB.
ISRF_COMPONENTS = ((7500.0, 1.0e-14), (4000.0, 1.65e-13), (3000.0, 4.0e-13), (2.728, 1.0))


def isrf(nu: np.ndarray) -> np.ndarray:
    """Synthetic isotropic external intensity I_nu (erg s-1 cm-2 Hz-1 sr-1)."""
    out = np.zeros_like(np.asarray(nu, dtype=np.float64))
    for T, Wd in ISRF_COMPONENTS:
        out += Wd * _bb(nu, T)
    return out


def isrf_integral(n_quad: int = 20000) -> float:
    """Frequency integral of the synthetic field over 0.1-3000 um (dense
    log-trapezoid), erg s-1 cm-2 sr-1."""
    nu, w = frequency_grid(n_quad)
    return float(np.sum(w * isrf(nu)))


def blackbody_Lnu(nu: np.ndarray, L_total: float, T_star: float) -> np.ndarray:
    """Luminosity density of a blackbody source of total luminosity L_total
    (erg/s): L_nu = L_total * pi B_nu(T) / (sigma_SB T^4)."""
    return L_total * math.pi * _bb(nu, T_star) / (_SIGMA_SB * T_star ** 4)


# ---------------------------------------------------------------- grains
@dataclasses.dataclass
class GrainModel:
    """A synthetic size distribution of stochastically heated grains (the
    DustEM silicates of the paper's Appendix A are not available): per size
    bin s the grains per H, the absorption cross section per grain at the K
    frequencies, and an enthalpy grid of nE bins (enthalpy U and
    temperature T of each bin)."""
    nu: np.ndarray            # [K] Hz
    w: np.ndarray             # [K] quadrature weights, Hz
    a_cm: np.ndarray          # [S] grain radius
    abundance: np.ndarray     # [S] grains per H
    sigma: np.ndarray         # [S, K] cm^2 per grain
    U: np.ndarray             # [S, nE] erg per grain
    T: np.ndarray             # [S, nE] K

    @property
    def sigma_per_H(self) -> np.ndarray:
        """[K] absorption cross section per H of the whole distribution."""
        return (self.abundance[:, None] * self.sigma).sum(axis=0)


def grain_model(nu: np.ndarray, w: np.ndarray, n_size: int = 8, n_enthalpy: int = 128,
                a_min_um: float = 0.001, a_max_um: float = 0.3, T_min: float = 4.0) -> GrainModel:
    """Grains of radii log-spaced in [a_min, a_max] with an a^-3.5 size
    distribution scaled so that the whole distribution absorbs
    sigma_abs(0.55 um) of `dust_model` per H; Q_abs = x/(1+x) with x = 2 pi a
    q(lambda)/lambda, q = (lambda/1 um)^-1 (Q ~ a lambda^-2 for small grains,
    ~1 for large); density 3 g cm^-3, 20 amu per atom, heat capacity
    3 N k f(T/500 K) with f(y) = c y^3/(1 + c y^3), c = 4 pi^4/5 (the Debye
    T^3 law at low temperature, 3 N k at high); enthalpy bins at
    temperatures log-spaced from T_min to T_max(a), which falls from
    2500 K for the smallest to 150 K for the largest grains (log-linear in
    a), as in the paper's tests."""
    nu = np.asarray(nu, dtype=np.float64)
    lam_cm = _C / nu
    a = np.exp(np.linspace(math.log(a_min_um), math.log(a_max_um), n_size)) * 1e-4
    dlna = (math.log(a_max_um) - math.log(a_min_um)) / max(n_size - 1, 1)
    x = 2.0 * math.pi * a[:, None] * (lam_cm[None, :] / 1e-4) ** -1.0 / lam_cm[None, :]
    sigma = math.pi * a[:, None] ** 2 * x / (1.0 + x)
    ab = a ** -3.5 * a * dlna        # dn ~ a^-3.5 da
    nu_v = _C / (LAMBDA_V_UM * 1e-4)
    sv = np.array([math.pi * aa ** 2 * (lambda xx: xx / (1 + xx))(2 * math.pi * aa * (LAMBDA_V_UM) ** -1.0 /
                                                                      (LAMBDA_V_UM * 1e-4)) for aa in a])
    sabs_v = dust_model(np.array([nu_v]))[0][0]
    ab *= sabs_v / float((ab * sv).sum())
    rho, m_atom, theta = 3.0, 20.0 * 1.66053906660e-24, 500.0
    c = 4.0 * math.pi ** 4 / 5.0
    frac = (np.log(a) - math.log(a[0])) / max(math.log(a[-1]) - math.log(a[0]), 1e-30)
    T_top = np.exp(math.log(2500.0) + frac * (math.log(150.0) - math.log(2500.0)))
    U = np.empty((n_size, n_enthalpy))
    T = np.empty((n_size, n_enthalpy))
    for s in range(n_size):
        n_atoms = 4.0 / 3.0 * math.pi * a[s] ** 3 * rho / m_atom
        Tf = np.exp(np.linspace(math.log(1e-3), math.log(T_top[s] * 1.01), 40000))
        y = Tf / theta
        C = 3.0 * n_atoms * _K * c * y ** 3 / (1.0 + c * y ** 3)
        Uf = np.concatenate([[0.0], np.cumsum(0.5 * (C[1:] + C[:-1]) * np.diff(Tf))])
        T[s] = np.exp(np.linspace(math.log(T_min), math.log(T_top[s]), n_enthalpy))
        U[s] = np.interp(np.log(T[s]), np.log(Tf), Uf)
    return GrainModel(nu=nu, w=np.asarray(w, dtype=np.float64), a_cm=a, abundance=ab, sigma=sigma, U=U, T=T)


# ---------------------------------------------------------------- problems
@dataclasses.dataclass
class Problem:
    """One synthetic workload: grid, frequencies, dust and sources."""
    name: str
    grid: Grid
    nu: np.ndarray
    w: np.ndarray
    sigma_abs: np.ndarray
    sigma_sca: np.ndarray
    g: np.ndarray
    I_bg: np.ndarray             # per frequency
    ps_pos: np.ndarray           # (n_ps, 3) root units
    ps_Lnu: np.ndarray           # (n_ps, K)
    emit_nu: np.ndarray          # frequency grid of the temperature solve
    emit_w: np.ndarray
    emit_sigma_abs: np.ndarray
    n_bg: int = 0
    n_ps_pk: int = 0
    n_dust: int = 0
    T_floor: float = 2.0
    T_max: float = 3000.0

    @property
    def K(self) -> int:
        return int(self.nu.shape[0])


def sphere_problem(n: int = 32, n_packages: int = 100_000, tau_centre_edge: float = 1.0,
                   albedo: float = 0.5, g: float = 0.5, box_pc: float = 1.0,
                   K_emit: int = 64) -> Problem:
    """Uniform sphere of radius n/2 cells on an n^3 grid, centre-to-edge
    optical depth tau at one frequency (0.55 um) with the given albedo and
    HG asymmetry, heated by the isotropic external field whose frequency
    integral is carried by that single frequency; temperatures from the
    K_emit-frequency synthetic dust."""
    s_cm = box_pc * PC_CM / n
    R = n / 2.0
    n0 = tau_centre_edge / (SIGMA_V * R * s_cm)
    grid = regular_grid(sphere_density(n, R, n0), s_cm)
    nu0 = _C / (LAMBDA_V_UM * 1e-4)
    I0 = float(isrf(np.array([nu0]))[0])
    w0 = isrf_integral() / I0
    enu, ew = frequency_grid(K_emit)
    esabs, _, _ = dust_model(enu)
    return Problem("sphere", grid, np.array([nu0]), np.array([w0]),
                   np.array([(1 - albedo) * SIGMA_V]), np.array([albedo * SIGMA_V]), np.array([g]),
                   np.array([I0]), np.zeros((0, 3)), np.zeros((0, 1)), enu, ew, esabs,
                   n_bg=n_packages)


def lognormal_problem(n: int = 128, K: int = 64, sigma_ln: float = 1.0, tau_v_mean: float = 5.0,
                      seed: int = 2, box_pc: float = 1.0, L_star_lsun: float = 1.0e6,
                      T_star: float = 1.0e4, packages_per_freq: int = 1_000_000,
                      ps_frac=((0.3, 0.5, 0.5), (0.7, 0.5, 0.5))) -> Problem:
    """Lognormal cloud on an n^3 regular grid (GRF with P(k) ~ k^-3),
    scaled so that the mean face-to-face optical depth at 0.55 um over the
    axis-aligned sightlines is tau_v_mean, K frequencies with the synthetic
    dust, isotropic synthetic field and blackbody point sources placed at
    the centres of the cells containing ps_frac * n, those cells emptied."""
    s_cm = box_pc * PC_CM / n
    rho = grf_lognormal(n, sigma_ln, seed)
    rho *= tau_v_mean / (SIGMA_V * s_cm * n * rho.mean())
    ps = np.array([[math.floor(f * n) + 0.5 for f in fr] for fr in ps_frac], dtype=np.float64)
    for p in ps:
        ix, iy, iz = (int(v) for v in p)
        rho[iz, iy, ix] = 0.0
    grid = regular_grid(rho.astype(np.float32), s_cm)
    nu, w = frequency_grid(K)
    sabs, ssca, g = dust_model(nu)
    Lnu = np.stack([blackbody_Lnu(nu, L_star_lsun * L_SUN, T_star) for _ in ps]) if len(ps) else np.zeros((0, K))
    n_ps = len(ps)
    return Problem("lognormal", grid, nu, w, sabs, ssca, g, isrf(nu), ps, Lnu, nu, w, sabs,
                   n_bg=packages_per_freq // 2,
                   n_ps_pk=(packages_per_freq // 2) // max(n_ps, 1) if n_ps else 0,
                   n_dust=packages_per_freq)


def octree_from_field(field: np.ndarray, n_root: int, nlevels: int, root_cell_cm: float,
                      threshold: float = 4.0) -> Grid:
    """Octree over a cubic field sampled at the finest resolution
    n_root * 2^(nlevels-1): a cell is refined when the mean of the field
    over its volume exceeds `threshold` times the global mean; leaves hold
    the mean over their volume (block averages, so mass is conserved)."""
    M = n_root << (nlevels - 1)
    f = np.asarray(field, dtype=np.float64)
    if f.shape != (M, M, M):
        raise ValueError(f"field must be {M}^3")
    means = []
    for L in range(nlevels):
        b = 1 << (nlevels - 1 - L)
        n = n_root << L
        means.append(f.reshape(n, b, n, b, n, b).mean(axis=(1, 3, 5)))   # [z, y, x]
    gmean = f.mean()

    def _lookup(L, lo):
        idx = np.rint(lo * (1 << L)).astype(np.int64)
        return means[L][idx[:, 2], idx[:, 1], idx[:, 0]]

    def refine(L, lo, size):
        return _lookup(L, lo) > threshold * gmean

    def density(lo, size):
        L = int(round(-math.log2(size)))
        return _lookup(L, lo)

    return octree_from_function(n_root, n_root, n_root, nlevels, root_cell_cm, refine, density)


def octree_lognormal(n_root: int = 64, nlevels: int = 4, sigma_ln: float = 1.5, seed: int = 3,
                     tau_v_core: float = 100.0, core_contrast: float = 200.0, box_pc: float = 1.0,
                     threshold: float = 4.0) -> Grid:
    """Lognormal cloud (GRF, P(k) ~ k^-3) times a central Gaussian core of
    the given contrast, refined top-down where the cell mean exceeds
    `threshold` times the mean, scaled so that the optical depth at 0.55 um
    from the centre to the edge along +x is tau_v_core."""
    M = n_root << (nlevels - 1)
    rho = grf_lognormal(M, sigma_ln, seed)
    c = (np.arange(M) + 0.5) / M - 0.5
    z, y, x = np.meshgrid(c, c, c, indexing="ij", sparse=True)
    r2 = x * x + y * y + z * z
    sig = 0.1
    rho = rho * (1.0 + (core_contrast - 1.0) * np.exp(-0.5 * r2 / (sig * sig)))
    s_fine = box_pc * PC_CM / M
    col = rho[M // 2, M // 2, M // 2:].sum() * s_fine
    rho *= tau_v_core / (SIGMA_V * col)
    return octree_from_field(rho, n_root, nlevels, box_pc * PC_CM / n_root, threshold)


def batch_clouds(n_models: int = 256, K: int = 32, n_min: int = 16, n_max: int = 96, seed: int = 4000,
                 pk_min: float = 1e5, pk_max: float = 1e6, box_pc: float = 1.0):
    """Independent lognormal clouds of uneven size for the batched launch:
    model m has an N_m^3 grid with N_m log-uniform in [n_min, n_max] (a
    multiple of 8), sigma_ln ~ U(0.5, 1.5), mean face-to-face tau_V
    log-uniform in [1, 50], GRF seed seed + m; K frequencies; the package
    count of every (model, frequency) pair log-uniform in [pk_min, pk_max].
    Returns (grids, frequency table (nu, w, sigma_abs, sigma_sca, g, I_bg),
    packages[m, k])."""
    rng = np.random.default_rng(seed)
    grids = []
    for m in range(n_models):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max))) / 8.0)) * 8
        n = max(n_min, min(n_max, n))
        sig = rng.uniform(0.5, 1.5)
        tau = math.exp(rng.uniform(math.log(1.0), math.log(50.0)))
        rho = grf_lognormal(n, sig, seed + m)
        s_cm = box_pc * PC_CM / n
        rho *= tau / (SIGMA_V * s_cm * n * rho.mean())
        grids.append(regular_grid(rho.astype(np.float32), s_cm))
    nu, w = frequency_grid(K)
    sabs, ssca, g = dust_model(nu)
    pk = np.exp(rng.uniform(math.log(pk_min), math.log(pk_max), size=(n_models, K))).astype(np.int64)
    return grids, (nu, w, sabs, ssca, g, isrf(nu)), pk
