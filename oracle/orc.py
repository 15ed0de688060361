"""ctypes wrapper of the FP64 CPU oracle (liborc.so).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the GPU library or its binding.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")

CROSS, SCATTER, ESCAPE, FLOOR, RUNAWAY = 0, 1, 2, 3, 4
CLASS_BG, CLASS_DUST, CLASS_PS0 = 0, 1, 2


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nlevels", C.c_int32),
                ("ncells", C.c_int64), ("level_offset", C.POINTER(C.c_int64)),
                ("root_cell_cm", C.c_double), ("words", C.POINTER(C.c_uint32))]


class _Freq(C.Structure):
    _fields_ = [("nu", C.c_double), ("w_nu", C.c_double), ("sigma_abs", C.c_double),
                ("sigma_sca", C.c_double), ("g", C.c_double)]


class _Sources(C.Structure):
    _fields_ = [("I_bg_nu", C.c_double), ("n_ps", C.c_int32), ("ps_pos", C.POINTER(C.c_double)),
                ("ps_L_nu", C.POINTER(C.c_double)), ("T", C.POINTER(C.c_float)),
                ("n_bg", C.c_uint64), ("n_ps_pk", C.c_uint64), ("n_dust", C.c_uint64),
                ("dust_mode", C.c_int32), ("L_ref", C.POINTER(C.c_double)), ("dust_cap", C.c_double),
                ("ali_self", C.POINTER(C.c_double)), ("ali_emitted", C.POINTER(C.c_double))]


class _ScatterParams(C.Structure):
    _fields_ = [("axis", C.c_int32), ("forced", C.c_int32), ("max_scatter", C.c_int32), ("direct", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("packages", C.c_uint64), ("cell_steps", C.c_uint64), ("scatterings", C.c_uint64),
                ("runaways", C.c_uint64), ("e_emitted", C.c_double), ("e_absorbed", C.c_double),
                ("e_escaped", C.c_double)]


class _Segment(C.Structure):
    _fields_ = [("cell", C.c_int64), ("ds", C.c_double), ("event", C.c_int32)]


class _TStats(C.Structure):
    _fields_ = [("mean_T", C.c_double), ("hot5_mean_T", C.c_double),
                ("mean_rel_change", C.c_double), ("clamped", C.c_uint64)]


SEGMENT_DTYPE = np.dtype([("cell", np.int64), ("ds", np.float64), ("event", np.int32)], align=True)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"oracle library not built: {_LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(_LIB_PATH)
        L.orc_u01.restype = C.c_double
        L.orc_planck.restype = C.c_double
        L.orc_planck.argtypes = [C.c_double, C.c_double]
        L.orc_gamma.restype = C.c_double
        L.orc_gamma.argtypes = [C.POINTER(_Freq), C.c_int32, C.c_double]
        L.orc_leaf.restype = C.c_int64
        L.orc_validate_grid.restype = C.c_int32
        for name in ("orc_simulate_frequency", "orc_trace_package", "orc_trace_from",
                     "orc_update_temperature", "orc_map", "orc_dust_luminosity",
                     "orc_update_temperature_ali", "orc_scatter_map"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


class GridView:
    """Keeps the numpy arrays of a workloads.Grid alive for a call."""

    def __init__(self, g):
        self.lo = np.ascontiguousarray(g.level_offset, dtype=np.int64)
        self.words = np.ascontiguousarray(g.words, dtype=np.uint32)
        self.s = _Grid(g.nx, g.ny, g.nz, g.nlevels, self.words.shape[0], _p(self.lo, C.c_int64),
                       float(g.root_cell_cm), _p(self.words, C.c_uint32))


def _freq(f):
    nu, w, sabs, ssca, g = f
    return _Freq(float(nu), float(w), float(sabs), float(ssca), float(g))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def u01(x):
    return lib().orc_u01(C.c_uint32(x))


def uniforms(seed, iteration, cls, freq_index, package_id, n):
    out = np.zeros(n, dtype=np.float64)
    lib().orc_uniforms(C.c_uint64(seed), C.c_uint32(iteration), C.c_uint32(cls), C.c_uint32(freq_index),
                       C.c_uint32(package_id), C.c_int32(n), _p(out, C.c_double))
    return out


def planck(nu, T):
    return lib().orc_planck(float(nu), float(T))


def gamma(emit_nu, emit_w, emit_sabs, T):
    arr = (_Freq * len(emit_nu))(*[_Freq(float(a), float(b), float(c), 0.0, 0.0)
                                   for a, b, c in zip(emit_nu, emit_w, emit_sabs)])
    return lib().orc_gamma(arr, len(emit_nu), float(T))


def leaf(grid, p):
    gv = GridView(grid)
    pp = (C.c_double * 3)(*p)
    lo = (C.c_double * 3)()
    sz = C.c_double()
    c = lib().orc_leaf(C.byref(gv.s), pp, lo, C.byref(sz))
    return int(c), (lo[0], lo[1], lo[2]), sz.value


def validate(grid):
    gv = GridView(grid)
    return int(lib().orc_validate_grid(C.byref(gv.s)))


def hg_scatter(g, u0, xi):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    n = xi.shape[0] // 2
    out = np.zeros((n, 3), dtype=np.float64)
    u = (C.c_double * 3)(*u0)
    lib().orc_hg_scatter(C.c_double(g), u, C.c_int32(n), _p(xi, C.c_double), _p(out, C.c_double))
    return out


class _SourcesView:
    def __init__(self, I_bg=0.0, ps_pos=None, ps_Lnu=None, T=None, n_bg=0, n_ps_pk=0, n_dust=0, dust_mode=1,
                 L_ref=None, dust_cap=0.0, ali_self=None, ali_emitted=None):
        self.pos = np.ascontiguousarray(ps_pos if ps_pos is not None else np.zeros((0, 3)), dtype=np.float64)
        self.L = np.ascontiguousarray(ps_Lnu if ps_Lnu is not None else np.zeros(0), dtype=np.float64)
        self.T = None if T is None else np.ascontiguousarray(T, dtype=np.float32)
        self.Lref = None if L_ref is None else np.ascontiguousarray(L_ref, dtype=np.float64)
        n_ps = self.pos.shape[0]
        self.s = _Sources(float(I_bg), n_ps, _p(self.pos, C.c_double) if n_ps else None,
                          _p(self.L, C.c_double) if n_ps else None,
                          _p(self.T, C.c_float) if self.T is not None else None,
                          int(n_bg), int(n_ps_pk), int(n_dust), int(dust_mode),
                          _p(self.Lref, C.c_double) if self.Lref is not None else None, float(dust_cap),
                          _p(ali_self, C.c_double) if ali_self is not None else None,
                          _p(ali_emitted, C.c_double) if ali_emitted is not None else None)
        self.keep = (ali_self, ali_emitted)


def _stats_dict(st):
    return {k: getattr(st, k) for k, _ in _Stats._fields_}


def simulate_frequency(grid, freq, *, I_bg=0.0, ps_pos=None, ps_Lnu=None, T=None, n_bg=0, n_ps_pk=0,
                       n_dust=0, dust_mode=1, L_ref=None, dust_cap=0.0, seed=1, iteration=0, freq_index=0,
                       step_cap=0, nthreads=1, absorbed=None, want_path=False, hits=None, ali_self=None,
                       ali_emitted=None):
    """One Monte Carlo pass at one frequency.  freq = (nu, w, sigma_abs,
    sigma_sca, g).  Returns (absorbed float64[ncells], stats dict,
    path lengths or None).  hits: optional int64[ncells] accumulated with
    the number of depositing segments per cell.  dust_mode 2 emits the
    difference between the dust emission at T and L_ref (per cell, erg/s).
    ali_self / ali_emitted (float64[ncells], +=): diagonal ALI tallies."""
    gv = GridView(grid)
    for a in (ali_self, ali_emitted):
        if a is not None and (a.dtype != np.float64 or not a.flags.c_contiguous or a.size != grid.ncells):
            raise ValueError("ALI tallies must be contiguous float64 arrays of ncells")
    sv = _SourcesView(I_bg, ps_pos, ps_Lnu, T, n_bg, n_ps_pk, n_dust, dust_mode, L_ref, dust_cap, ali_self,
                      ali_emitted)
    f = _freq(freq)
    if absorbed is None:
        absorbed = np.zeros(grid.ncells, dtype=np.float64)
    n_tot = int(n_bg) + sv.pos.shape[0] * int(n_ps_pk) + (int(n_dust) if T is not None else 0)
    path = np.zeros(n_tot, dtype=np.float64) if want_path else None
    st = _Stats()
    rc = lib().orc_simulate_frequency(C.byref(gv.s), C.byref(f), C.byref(sv.s), C.c_uint64(seed),
                                      C.c_uint32(iteration), C.c_uint32(freq_index), C.c_int64(step_cap),
                                      C.c_int32(nthreads), _p(absorbed, C.c_double), C.byref(st),
                                      _p(path, C.c_double) if path is not None else None,
                                      _p(hits, C.c_int64) if hits is not None else None)
    if rc != 0:
        raise ValueError(f"orc_simulate_frequency failed: {rc}")
    return absorbed, _stats_dict(st), path


def trace_package(grid, freq, cls, package_id, *, I_bg=0.0, ps_pos=None, ps_Lnu=None, T=None, n_bg=0,
                  n_ps_pk=0, n_dust=0, dust_mode=1, L_ref=None, dust_cap=0.0, seed=1, iteration=0, freq_index=0,
                  step_cap=0, max_seg=100000):
    gv = GridView(grid)
    sv = _SourcesView(I_bg, ps_pos, ps_Lnu, T, n_bg, n_ps_pk, n_dust, dust_mode, L_ref, dust_cap)
    f = _freq(freq)
    out = np.zeros(max_seg, dtype=SEGMENT_DTYPE)
    ns = C.c_int32()
    rc = lib().orc_trace_package(C.byref(gv.s), C.byref(f), C.byref(sv.s), C.c_uint64(seed),
                                 C.c_uint32(iteration), C.c_uint32(freq_index), C.c_uint32(cls),
                                 C.c_uint32(package_id), C.c_int64(step_cap),
                                 out.ctypes.data_as(C.POINTER(_Segment)), C.c_int32(max_seg), C.byref(ns))
    if rc != 0:
        raise ValueError(f"orc_trace_package failed: {rc}")
    return out[: min(ns.value, max_seg)].copy()


def scatter_map(grid, freq, *, axis=2, forced=True, max_scatter=0, direct=False, I_bg=0.0, ps_pos=None,
                ps_Lnu=None, n_bg=0, n_ps_pk=0, seed=1, iteration=0, freq_index=0, step_cap=0, nthreads=8):
    """Peel-off image of scattered light (erg s^-1 cm^-2 Hz^-1 sr^-1),
    npy x npx as map_image, and the run's statistics."""
    gv = GridView(grid)
    sv = _SourcesView(I_bg, ps_pos, ps_Lnu, None, n_bg, n_ps_pk, 0, 1)
    f = _freq(freq)
    a = axis & 3
    N = [grid.nx, grid.ny, grid.nz]
    b, c = (1 if a == 0 else 0), (1 if a == 2 else 2)
    fine = 1 << (grid.nlevels - 1)
    npx, npy = N[b] * fine, N[c] * fine
    img = np.zeros(npx * npy, dtype=np.float64)
    sp = _ScatterParams(int(axis), int(bool(forced)), int(max_scatter), int(bool(direct)))
    st = _Stats()
    rc = lib().orc_scatter_map(C.byref(gv.s), C.byref(f), C.byref(sv.s), C.c_uint64(seed), C.c_uint32(iteration),
                               C.c_uint32(freq_index), C.byref(sp), C.c_int64(step_cap), C.c_int32(nthreads),
                               _p(img, C.c_double), C.byref(st))
    if rc != 0:
        raise ValueError(f"orc_scatter_map failed: {rc}")
    return img.reshape(npy, npx), _stats_dict(st)


def dust_luminosity(grid, freq, T):
    """Dust emission of every cell at one frequency (erg/s, times w)."""
    gv = GridView(grid)
    f = _freq(freq)
    Tc = np.ascontiguousarray(T, dtype=np.float32)
    L = np.zeros(grid.ncells, dtype=np.float64)
    rc = lib().orc_dust_luminosity(C.byref(gv.s), C.byref(f), _p(Tc, C.c_float), _p(L, C.c_double))
    if rc != 0:
        raise ValueError(f"orc_dust_luminosity failed: {rc}")
    return L


def trace_from(grid, freq, p0, u0, W0, tau0, *, seed=1, package_id=0, step_cap=0, absorbed=None,
               max_seg=100000):
    gv = GridView(grid)
    f = _freq(freq)
    out = np.zeros(max_seg, dtype=SEGMENT_DTYPE)
    ns = C.c_int32()
    wesc = C.c_double()
    rc = lib().orc_trace_from(C.byref(gv.s), C.byref(f), (C.c_double * 3)(*p0), (C.c_double * 3)(*u0),
                              C.c_double(W0), C.c_double(tau0), C.c_uint64(seed), C.c_uint32(package_id),
                              C.c_int64(step_cap), _p(absorbed, C.c_double),
                              out.ctypes.data_as(C.POINTER(_Segment)), C.c_int32(max_seg), C.byref(ns),
                              C.byref(wesc))
    if rc != 0:
        raise ValueError(f"orc_trace_from failed: {rc}")
    return out[: min(ns.value, max_seg)].copy(), wesc.value


def update_temperature(grid, emit_nu, emit_w, emit_sabs, absorbed, T_old=None, T_floor=2.0, T_max=3000.0,
                       ali_self=None, ali_emitted=None):
    """Equilibrium temperatures; with the ALI tallies, the diagonal-ALI solve."""
    gv = GridView(grid)
    K = len(emit_nu)
    arr = (_Freq * K)(*[_Freq(float(a), float(b), float(c), 0.0, 0.0)
                        for a, b, c in zip(emit_nu, emit_w, emit_sabs)])
    A = np.ascontiguousarray(absorbed, dtype=np.float64)
    To = None if T_old is None else np.ascontiguousarray(T_old, dtype=np.float32)
    Tn = np.zeros(grid.ncells, dtype=np.float32)
    st = _TStats()
    if ali_self is not None:
        Sa = np.ascontiguousarray(ali_self, dtype=np.float64)
        Ea = np.ascontiguousarray(ali_emitted, dtype=np.float64)
        rc = lib().orc_update_temperature_ali(C.byref(gv.s), arr, C.c_int32(K), C.c_double(T_floor),
                                              C.c_double(T_max), _p(A, C.c_double), _p(Sa, C.c_double),
                                              _p(Ea, C.c_double), _p(To, C.c_float) if To is not None else None,
                                              _p(Tn, C.c_float), C.byref(st))
    else:
        rc = lib().orc_update_temperature(C.byref(gv.s), arr, C.c_int32(K), C.c_double(T_floor),
                                          C.c_double(T_max), _p(A, C.c_double),
                                          _p(To, C.c_float) if To is not None else None, _p(Tn, C.c_float),
                                          C.byref(st))
    if rc != 0:
        raise ValueError(f"orc_update_temperature failed: {rc}")
    return Tn, {k: getattr(st, k) for k, _ in _TStats._fields_}


def map_image(grid, freq, T, axis):
    gv = GridView(grid)
    f = _freq(freq)
    Tc = np.ascontiguousarray(T, dtype=np.float32)
    npx, npy = C.c_int32(), C.c_int32()
    lib().orc_map(C.byref(gv.s), C.byref(f), _p(Tc, C.c_float), C.c_int32(axis), None,
                  C.byref(npx), C.byref(npy))
    img = np.zeros(npx.value * npy.value, dtype=np.float64)
    rc = lib().orc_map(C.byref(gv.s), C.byref(f), _p(Tc, C.c_float), C.c_int32(axis), _p(img, C.c_double),
                       C.byref(npx), C.byref(npy))
    if rc != 0:
        raise ValueError(f"orc_map failed: {rc}")
    return img.reshape(npy.value, npx.value)


def iterate(P, *, seed, iterations, packages=None, reference=False, cap=0.0, nthreads=8, dust_seed=None,
            ali=False):
    """The iteration of Sect. 2.1.2 on a problem P (attributes of a
    workloads.Problem: grid, nu, w, sigma_abs, sigma_sca, g, I_bg, ps_pos,
    ps_Lnu, n_bg, n_ps_pk, n_dust, emit_nu, emit_w, emit_sigma_abs,
    T_floor, T_max).

    Iteration 1 simulates the constant sources (external field, point
    sources) at every frequency and keeps their absorption A_const; its
    temperatures come from A_const alone.  Iteration i >= 2 uses
    packages(i) dust packages per frequency (default P.n_dust):
      * plain: A_i = A_const + the dust emission at T_{i-1};
      * reference field, reference=True or "correction": the packages
        carry the difference between the emission at T_{i-1} and the
        reference emission L_ref, A_i = A_ref + their absorption, and both
        references then move to the package-weighted running mean,
        X_ref += n_i / (n_2 + ... + n_i) (X_i - X_ref) -- so the constant
        sources, part of A_ref from the start, are never simulated again;
      * reference field, reference="average": the packages carry the whole
        emission at T_{i-1} as in the plain method, A_i = A_const + their
        absorption, the reference absorption moves to the package-weighted
        running mean of the A_i in the same way, and the temperatures come
        from the reference absorption (one stored number per cell).
    With ali (plain iteration only), every dust iteration also counts what
    each cell's packages deposit in that cell and the energy it emitted,
    and the temperatures come from the diagonal-ALI solve (Sect. 2.1.2).
    The dust packages draw from dust_seed (default: seed).  Returns
    [(T_i, stats_i)] for i = 1..iterations."""
    dseed = seed if dust_seed is None else dust_seed
    g = P.grid
    K = len(P.nu)
    emit = (P.emit_nu, P.emit_w, P.emit_sigma_abs)
    fr = [(P.nu[k], P.w[k], P.sigma_abs[k], P.sigma_sca[k], P.g[k]) for k in range(K)]
    have_ps = len(P.ps_pos) > 0
    A_const = np.zeros(g.ncells)
    for k in range(K):
        simulate_frequency(g, fr[k], I_bg=P.I_bg[k], ps_pos=P.ps_pos if have_ps else None,
                           ps_Lnu=P.ps_Lnu[:, k] if have_ps else None, n_bg=P.n_bg,
                           n_ps_pk=P.n_ps_pk if have_ps else 0, seed=seed, iteration=1, freq_index=k,
                           nthreads=nthreads, absorbed=A_const)
    T, st = update_temperature(g, *emit, A_const, T_floor=P.T_floor, T_max=P.T_max)
    out = [(T, st)]
    A_ref = A_const.copy()
    L_ref = np.zeros((K, g.ncells))
    n_sum = 0
    mode = "correction" if reference is True else (reference or None)
    if mode not in (None, "correction", "average"):
        raise ValueError("reference must be False, True, 'correction' or 'average'")
    if ali and mode:
        raise ValueError("ALI is combined here with the plain iteration only")
    for it in range(2, iterations + 1):
        n = int(packages(it)) if packages is not None else int(P.n_dust)
        if mode:
            n_sum += n
            beta = n / n_sum
        if mode == "correction":
            A = A_ref.copy()
            for k in range(K):
                simulate_frequency(g, fr[k], T=T, n_dust=n, dust_mode=2, L_ref=L_ref[k], dust_cap=cap, seed=dseed,
                                   iteration=it, freq_index=k, nthreads=nthreads, absorbed=A)
                L_ref[k] += beta * (dust_luminosity(g, fr[k], T) - L_ref[k])
        else:
            A = A_const.copy()
            S_ali = np.zeros(g.ncells) if ali else None
            E_ali = np.zeros(g.ncells) if ali else None
            for k in range(K):
                simulate_frequency(g, fr[k], T=T, n_dust=n, dust_mode=1, dust_cap=cap, seed=dseed, iteration=it,
                                   freq_index=k, nthreads=nthreads, absorbed=A, ali_self=S_ali, ali_emitted=E_ali)
        if mode == "average":
            A_ref += beta * (A - A_ref)
            A = A_ref
        if ali:
            T_new, st = update_temperature(g, *emit, A, T_old=T, T_floor=P.T_floor, T_max=P.T_max, ali_self=S_ali,
                                           ali_emitted=E_ali)
        else:
            T_new, st = update_temperature(g, *emit, A, T_old=T, T_floor=P.T_floor, T_max=P.T_max)
        if mode == "correction":
            A_ref += beta * (A - A_ref)
        T = T_new
        out.append((T, st))
    return out
