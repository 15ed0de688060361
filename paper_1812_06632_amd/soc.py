"""Python binding of the SOC C-ABI library (libsoc.so, gfx950).

Argument marshalling only: every step of the Monte Carlo path, the
temperature solve and the map runs in the HIP kernels behind include/soc.h.
Device arrays are torch CUDA tensors (passed by data_ptr()); the library
enqueues its work on the torch stream given to the Context.  There is no
CPU fallback: importing this module fails if the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsoc.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first (python __graft_entry__.py)")
_lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EHIP, EGRID, ESTATE = 0, -1, -2, -3, -4, -5
CROSS, SCATTER, ESCAPE, FLOOR, RUNAWAY = 0, 1, 2, 3, 4
CLASS_BG, CLASS_DUST, CLASS_PS0 = 0, 1, 2
OPTIONS = {"step_cap": 0, "block": 1, "blocks_per_cu": 2, "refill_min": 3, "inner_steps": 4, "timing": 5,
           "scatter_min": 6, "xcd_copies": 7, "chunk": 8, "batch_lds_cells": 9, "multi_spread": 10}


class SocError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"soc status {status}: {msg}")
        self.status = status


class _GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nlevels", C.c_int32),
                ("ncells", C.c_int64), ("level_offset", C.POINTER(C.c_int64)),
                ("root_cell_cm", C.c_double), ("d_words", C.c_void_p)]


class _Freq(C.Structure):
    _fields_ = [("nu", C.c_double), ("w_nu", C.c_double), ("sigma_abs", C.c_double),
                ("sigma_sca", C.c_double), ("g", C.c_double)]


class _PointSource(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("z", C.c_double), ("L_nu", C.c_double)]


class _Sources(C.Structure):
    _fields_ = [("I_bg_nu", C.c_double), ("n_ps", C.c_int32), ("ps", C.POINTER(_PointSource)),
                ("d_T", C.c_void_p), ("n_bg", C.c_uint64), ("n_ps_pk", C.c_uint64), ("n_dust", C.c_uint64),
                ("dust_mode", C.c_int32), ("d_L_ref", C.c_void_p), ("ref_beta", C.c_double),
                ("dust_cap", C.c_double), ("d_ali_self", C.c_void_p), ("d_ali_emitted", C.c_void_p)]


class _SimStats(C.Structure):
    _fields_ = [("packages", C.c_uint64), ("cell_steps", C.c_uint64), ("scatterings", C.c_uint64),
                ("runaways", C.c_uint64), ("e_emitted", C.c_double), ("e_absorbed", C.c_double),
                ("e_escaped", C.c_double)]


class _ScatterParams(C.Structure):
    _fields_ = [("axis", C.c_int32), ("forced", C.c_int32), ("max_scatter", C.c_int32), ("direct", C.c_int32)]


class _ScatterStats(C.Structure):
    _fields_ = [("packages", C.c_uint64), ("cell_steps", C.c_uint64), ("scatterings", C.c_uint64),
                ("ray_steps", C.c_uint64), ("e_emitted", C.c_double), ("e_escaped", C.c_double)]


class _TempStats(C.Structure):
    _fields_ = [("mean_T", C.c_double), ("hot5_mean_T", C.c_double), ("mean_rel_change", C.c_double),
                ("clamped", C.c_uint64)]


SEGMENT_DTYPE = np.dtype([("cell", np.int64), ("ds", np.float64), ("event", np.int32), ("pad", np.int32)])

_lib.soc_last_error.restype = C.c_char_p
_lib.soc_last_error.argtypes = [C.c_void_p]
_lib.soc_ctx_create.argtypes = [C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
_lib.soc_ctx_destroy.argtypes = [C.c_void_p]
_lib.soc_ctx_set_stream.argtypes = [C.c_void_p, C.c_void_p]
_lib.soc_ctx_set_option.argtypes = [C.c_void_p, C.c_int, C.c_int64]
_lib.soc_ctx_get_option.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int64)]
_lib.soc_ctx_mc_timing.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
_lib.soc_build_grid.argtypes = [C.c_void_p, C.POINTER(_GridDesc), C.POINTER(C.c_void_p)]
_lib.soc_grid_destroy.argtypes = [C.c_void_p]
_lib.soc_grid_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_void_p)]
_lib.soc_simulate_frequency.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(_Freq), C.POINTER(_Sources), C.c_uint64,
                                        C.c_uint32, C.c_uint32, C.c_void_p, C.POINTER(_SimStats)]
_lib.soc_simulate_frequency_noalloc.argtypes = _lib.soc_simulate_frequency.argtypes
_lib.soc_simulate_frequencies.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(_Freq), C.POINTER(_Sources),
                                          C.POINTER(C.c_uint32), C.c_uint64, C.c_uint32, C.c_void_p,
                                          C.POINTER(_SimStats)]
_lib.soc_update_temperature_ali.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(_TempStats)]
_lib.soc_scatter_map.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(_Freq), C.POINTER(_Sources), C.c_uint64,
                                 C.c_uint32, C.c_uint32, C.POINTER(_ScatterParams), C.c_void_p, C.c_int32, C.c_int32,
                                 C.POINTER(_ScatterStats)]
_lib.soc_shg_model_create.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32,
                                      C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_void_p)]
_lib.soc_shg_model_destroy.argtypes = [C.c_void_p]
_lib.soc_shg_model_destroy.restype = None
_lib.soc_shg_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.soc_reference_blend.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p]
_lib.soc_read_stats.argtypes = [C.c_void_p, C.POINTER(_SimStats), C.c_int32]
_lib.soc_trace_packages.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(_Freq), C.POINTER(_Sources), C.c_uint64,
                                    C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32), C.c_int32, C.c_int32,
                                    C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
_lib.soc_temp_table_build.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.c_double, C.c_double, C.c_int32,
                                      C.POINTER(C.c_void_p)]
_lib.soc_temp_table_destroy.argtypes = [C.c_void_p]
_lib.soc_update_temperature.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.POINTER(_TempStats)]
_lib.soc_map.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(_Freq), C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                         C.c_int32]


def exported_symbols():
    """Names of the C-ABI entry points this binding uses."""
    return [n for n in dir(_lib) if n.startswith("soc_")]


def _dev_ptr(t, dtype, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return C.c_void_p(t.data_ptr())


class Context:
    """A library context bound to one device and one torch stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        rc = _lib.soc_ctx_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != OK:
            raise SocError(rc, "soc_ctx_create failed")
        self.h = h
        self._children = weakref.WeakSet()

    def check(self, rc):
        if rc != OK:
            raise SocError(rc, _lib.soc_last_error(self.h).decode())

    def set_option(self, name: str, value: int):
        self.check(_lib.soc_ctx_set_option(self.h, OPTIONS[name], int(value)))

    def get_option(self, name: str) -> int:
        v = C.c_int64()
        self.check(_lib.soc_ctx_get_option(self.h, OPTIONS[name], C.byref(v)))
        return v.value

    def mc_timing(self, reset: bool = False):
        ms, n = C.c_double(), C.c_int64()
        self.check(_lib.soc_ctx_mc_timing(self.h, C.byref(ms), C.byref(n), int(reset)))
        return ms.value, n.value

    def read_stats(self, reset: bool = False) -> dict:
        st = _SimStats()
        self.check(_lib.soc_read_stats(self.h, C.byref(st), int(reset)))
        return {k: getattr(st, k) for k, _ in _SimStats._fields_}

    def close(self):
        """Destroy the context after the grids and tables created on it."""
        if getattr(self, "h", None):
            for ch in list(getattr(self, "_children", ())):
                ch.close()
            _lib.soc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Grid:
    """A validated grid; keeps the caller's device word array alive."""

    def __init__(self, ctx: Context, h, words: torch.Tensor, desc):
        self.ctx, self.h, self.words, self.desc = ctx, h, words, desc
        ctx._children.add(self)
        self.nx, self.ny, self.nz, self.nlevels = desc.nx, desc.ny, desc.nz, desc.nlevels
        self.ncells = desc.ncells

    @property
    def n_leaves(self) -> int:
        n = C.c_int64()
        self.ctx.check(_lib.soc_grid_info(self.h, C.byref(n), None))
        return n.value

    def close(self):
        if getattr(self, "h", None):
            _lib.soc_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_grid(ctx: Context, nx, ny, nz, nlevels, level_offset, root_cell_cm, words: torch.Tensor) -> Grid:
    """soc_build_grid: words is a device int32/uint32-bit tensor of ncells words."""
    if words.dtype not in (torch.int32,):
        raise TypeError("words must be an int32 tensor holding the raw 32-bit cell words")
    lo = np.ascontiguousarray(level_offset, dtype=np.int64)
    desc = _GridDesc(int(nx), int(ny), int(nz), int(nlevels), int(words.numel()),
                     lo.ctypes.data_as(C.POINTER(C.c_int64)), float(root_cell_cm), _dev_ptr(words, torch.int32, "words"))
    desc._lo = lo
    h = C.c_void_p()
    ctx.check(_lib.soc_build_grid(ctx.h, C.byref(desc), C.byref(h)))
    return Grid(ctx, h, words, desc)


def grid_from_workload(ctx: Context, g, device="cuda") -> Grid:
    """Upload a workloads.Grid and build it."""
    words = torch.from_numpy(g.words.view(np.int32).copy()).to(device)
    return build_grid(ctx, g.nx, g.ny, g.nz, g.nlevels, g.level_offset, g.root_cell_cm, words)


def _freq(f):
    nu, w, sabs, ssca, g = (float(x) for x in f)
    return _Freq(nu, w, sabs, ssca, g)


class _SourceView:
    def __init__(self, I_bg=0.0, ps_pos=None, ps_Lnu=None, T=None, n_bg=0, n_ps_pk=0, n_dust=0, dust_mode=1,
                 L_ref=None, ref_beta=0.0, dust_cap=0.0, ali_self=None, ali_emitted=None):
        pos = np.zeros((0, 3)) if ps_pos is None else np.asarray(ps_pos, dtype=np.float64).reshape(-1, 3)
        L = np.zeros(0) if ps_Lnu is None else np.asarray(ps_Lnu, dtype=np.float64).reshape(-1)
        n_ps = pos.shape[0]
        self.arr = (_PointSource * max(n_ps, 1))(*[_PointSource(*pos[i], L[i]) for i in range(n_ps)])
        self.T = T
        self.L_ref = L_ref
        self.s = _Sources(float(I_bg), n_ps, C.cast(self.arr, C.POINTER(_PointSource)) if n_ps else None,
                          _dev_ptr(T, torch.float32, "T") if T is not None else None,
                          int(n_bg), int(n_ps_pk), int(n_dust), int(dust_mode),
                          _dev_ptr(L_ref, torch.float64, "L_ref") if L_ref is not None else None,
                          float(ref_beta), float(dust_cap),
                          _dev_ptr(ali_self, torch.float64, "ali_self") if ali_self is not None else None,
                          _dev_ptr(ali_emitted, torch.float64, "ali_emitted") if ali_emitted is not None else None)
        self.ali = (ali_self, ali_emitted)


def simulate_frequency(ctx: Context, grid: Grid, freq, absorbed: torch.Tensor, *, I_bg=0.0, ps_pos=None,
                       ps_Lnu=None, T=None, n_bg=0, n_ps_pk=0, n_dust=0, dust_mode=1, L_ref=None, ref_beta=0.0,
                       dust_cap=0.0, ali_self=None, ali_emitted=None, seed=1, iteration=0, freq_index=0,
                       stats=False, noalloc=False):
    """soc_simulate_frequency (soc_simulate_frequency_noalloc if noalloc).
    freq = (nu, w_nu, sigma_abs, sigma_sca, g); absorbed: float64 CUDA
    tensor of ncells (accumulated).  dust_mode 2 emits the difference to
    L_ref (float64 CUDA tensor of ncells, blended in place with weight
    ref_beta).  ali_self / ali_emitted: float64 CUDA tensors of ncells, the
    diagonal-ALI tallies (+=).  Returns the call's statistics dict if
    stats, else None (asynchronous)."""
    sv = _SourceView(I_bg, ps_pos, ps_Lnu, T, n_bg, n_ps_pk, n_dust, dust_mode, L_ref, ref_beta, dust_cap,
                     ali_self, ali_emitted)
    f = _freq(freq)
    st = _SimStats() if stats else None
    fn = _lib.soc_simulate_frequency_noalloc if noalloc else _lib.soc_simulate_frequency
    ctx.check(fn(ctx.h, grid.h, C.byref(f), C.byref(sv.s), C.c_uint64(seed), C.c_uint32(iteration),
                 C.c_uint32(freq_index), _dev_ptr(absorbed, torch.float64, "absorbed"),
                 C.byref(st) if st is not None else None))
    if st is None:
        return None
    return {k: getattr(st, k) for k, _ in _SimStats._fields_}


def simulate_frequencies(ctx: Context, grid: Grid, freqs, absorbed: torch.Tensor, sources, freq_indices, *,
                         seed=1, iteration=0, stats=False):
    """soc_simulate_frequencies: freqs a list of K (nu, w_nu, sigma_abs,
    sigma_sca, g); sources a list of K dicts with the keyword arguments of
    simulate_frequency's sources (I_bg, ps_pos, ps_Lnu, T, n_bg, n_ps_pk,
    n_dust, dust_mode, L_ref, ref_beta, dust_cap); freq_indices K ints.
    All deposits are added to absorbed.  Returns the statistics dict if
    stats."""
    K = len(freqs)
    if len(sources) != K or len(freq_indices) != K:
        raise ValueError("one source set and one frequency index per frequency")
    # a source set given for several frequencies (the same dict object) is
    # marshalled once
    built = {}
    views = []
    for q in sources:
        v = built.get(id(q))
        if v is None:
            v = built[id(q)] = _SourceView(**q)
        views.append(v)
    farr = (_Freq * K)(*[_freq(f) for f in freqs])
    sarr = (_Sources * K)(*[v.s for v in views])
    karr = (C.c_uint32 * K)(*[int(k) for k in freq_indices])
    st = _SimStats() if stats else None
    ctx.check(_lib.soc_simulate_frequencies(ctx.h, grid.h, K, farr, sarr, karr, C.c_uint64(seed), C.c_uint32(iteration),
                                            _dev_ptr(absorbed, torch.float64, "absorbed"),
                                            C.byref(st) if st is not None else None))
    if st is None:
        return None
    return {k: getattr(st, k) for k, _ in _SimStats._fields_}


def trace_packages(ctx: Context, grid: Grid, freq, cls, ids, *, precision=0, max_seg=4096, I_bg=0.0, ps_pos=None,
                   ps_Lnu=None, T=None, n_bg=0, n_ps_pk=0, n_dust=0, dust_mode=1, L_ref=None, dust_cap=0.0, seed=1,
                   iteration=0, freq_index=0):
    """soc_trace_packages: returns (segments[n, max_seg], n_seg[n])."""
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    n = ids.shape[0]
    out = np.zeros((n, max_seg), dtype=SEGMENT_DTYPE)
    nseg = np.zeros(n, dtype=np.int32)
    sv = _SourceView(I_bg, ps_pos, ps_Lnu, T, n_bg, n_ps_pk, n_dust, dust_mode, L_ref, 0.0, dust_cap)
    f = _freq(freq)
    ctx.check(_lib.soc_trace_packages(ctx.h, grid.h, C.byref(f), C.byref(sv.s), C.c_uint64(seed),
                                      C.c_uint32(iteration), C.c_uint32(freq_index), C.c_uint32(cls),
                                      ids.ctypes.data_as(C.POINTER(C.c_uint32)), n, int(precision),
                                      C.c_void_p(out.ctypes.data), int(max_seg),
                                      nseg.ctypes.data_as(C.POINTER(C.c_int32))))
    return out, nseg


def scatter_image_shape(grid: Grid, axis: int):
    """(npy, npx) of a map or scattered-light image along axis."""
    a = axis & 3
    N = [grid.nx, grid.ny, grid.nz]
    fine = 1 << (grid.nlevels - 1)
    b, c = (1 if a == 0 else 0), (1 if a == 2 else 2)
    return N[c] * fine, N[b] * fine


def scatter_map(ctx: Context, grid: Grid, freq, image: torch.Tensor, *, axis=2, forced=True, max_scatter=0,
                direct=False, I_bg=0.0, ps_pos=None, ps_Lnu=None, n_bg=0, n_ps_pk=0, seed=1, iteration=0,
                freq_index=0, stats=False):
    """soc_scatter_map: image is a float64 CUDA tensor (npy, npx),
    accumulated.  Returns the statistics dict if stats."""
    sv = _SourceView(I_bg, ps_pos, ps_Lnu, None, n_bg, n_ps_pk, 0, 1)
    f = _freq(freq)
    npy, npx = image.shape
    sp = _ScatterParams(int(axis), int(bool(forced)), int(max_scatter), int(bool(direct)))
    st = _ScatterStats() if stats else None
    ctx.check(_lib.soc_scatter_map(ctx.h, grid.h, C.byref(f), C.byref(sv.s), C.c_uint64(seed), C.c_uint32(iteration),
                                   C.c_uint32(freq_index), C.byref(sp), _dev_ptr(image, torch.float64, "image"),
                                   int(npx), int(npy), C.byref(st) if st is not None else None))
    if st is None:
        return None
    return {k: getattr(st, k) for k, _ in _ScatterStats._fields_}


class ShgModel:
    """soc_shg_model: a grain model (workloads.GrainModel) on the device."""

    def __init__(self, ctx: Context, G):
        self.ctx = ctx
        self.S, self.K, self.N = len(G.a_cm), len(G.nu), G.U.shape[1]
        arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (G.nu, G.w, G.abundance, G.sigma, G.U, G.T)]
        P = C.POINTER(C.c_double)
        h = C.c_void_p()
        ctx.check(_lib.soc_shg_model_create(ctx.h, self.K, arrs[0].ctypes.data_as(P), arrs[1].ctypes.data_as(P),
                                            self.S, arrs[2].ctypes.data_as(P), arrs[3].ctypes.data_as(P), self.N,
                                            arrs[4].ctypes.data_as(P), arrs[5].ctypes.data_as(P), C.byref(h)))
        self.h = h
        ctx._children.add(self)

    def close(self):
        if getattr(self, "h", None):
            _lib.soc_shg_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shg_solve(ctx: Context, grid: Grid, model: ShgModel, absorbed: torch.Tensor, emission: torch.Tensor,
              P: torch.Tensor | None = None):
    """soc_shg_solve: absorbed and emission float64 CUDA tensors [K, ncells];
    P optional float64 [ncells, S, N]."""
    ctx.check(_lib.soc_shg_solve(ctx.h, grid.h, model.h, _dev_ptr(absorbed, torch.float64, "absorbed"),
                                 _dev_ptr(emission, torch.float64, "emission"),
                                 _dev_ptr(P, torch.float64, "P") if P is not None else None))


def reference_blend(ctx: Context, x: torch.Tensor, ref: torch.Tensor, beta: float):
    """soc_reference_blend: ref += beta (x - ref), float64 CUDA tensors."""
    if x.numel() != ref.numel():
        raise ValueError("x and ref differ in size")
    ctx.check(_lib.soc_reference_blend(ctx.h, C.c_int64(ref.numel()), C.c_double(beta),
                                       _dev_ptr(x, torch.float64, "x"), _dev_ptr(ref, torch.float64, "ref")))


class TempTable:
    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h
        ctx._children.add(self)

    def close(self):
        if getattr(self, "h", None):
            _lib.soc_temp_table_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def temp_table_build(ctx: Context, nu, w_nu, sigma_abs, T_floor=2.0, T_max=3000.0, nT=4096) -> TempTable:
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    w = np.ascontiguousarray(w_nu, dtype=np.float64)
    s = np.ascontiguousarray(sigma_abs, dtype=np.float64)
    h = C.c_void_p()
    P = C.POINTER(C.c_double)
    ctx.check(_lib.soc_temp_table_build(ctx.h, nu.shape[0], nu.ctypes.data_as(P), w.ctypes.data_as(P),
                                        s.ctypes.data_as(P), float(T_floor), float(T_max), int(nT), C.byref(h)))
    return TempTable(ctx, h)


def update_temperature(ctx: Context, grid: Grid, table: TempTable, absorbed: torch.Tensor, T_new: torch.Tensor,
                       T_old: torch.Tensor | None = None, stats=False, ali_self=None, ali_emitted=None):
    """soc_update_temperature, or soc_update_temperature_ali with the ALI
    tallies."""
    st = _TempStats() if stats else None
    T_old_p = _dev_ptr(T_old, torch.float32, "T_old") if T_old is not None else None
    if ali_self is not None or ali_emitted is not None:
        ctx.check(_lib.soc_update_temperature_ali(ctx.h, grid.h, table.h,
                                                  _dev_ptr(absorbed, torch.float64, "absorbed"),
                                                  _dev_ptr(ali_self, torch.float64, "ali_self"),
                                                  _dev_ptr(ali_emitted, torch.float64, "ali_emitted"), T_old_p,
                                                  _dev_ptr(T_new, torch.float32, "T_new"),
                                                  C.byref(st) if st is not None else None))
    else:
        ctx.check(_lib.soc_update_temperature(ctx.h, grid.h, table.h, _dev_ptr(absorbed, torch.float64, "absorbed"),
                                              T_old_p, _dev_ptr(T_new, torch.float32, "T_new"),
                                              C.byref(st) if st is not None else None))
    if st is None:
        return None
    return {k: getattr(st, k) for k, _ in _TempStats._fields_}


_lib.soc_temperature_stats.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(_TempStats)]


def temperature_stats(ctx: Context, grid: Grid, table: TempTable, T: torch.Tensor) -> dict:
    """soc_temperature_stats: <T> and the hottest-5% mean of a given field."""
    if T.numel() != grid.ncells:
        raise ValueError("T must hold one value per cell")
    st = _TempStats()
    ctx.check(_lib.soc_temperature_stats(ctx.h, grid.h, table.h, _dev_ptr(T, torch.float32, "T"), C.byref(st)))
    return {k: getattr(st, k) for k, _ in _TempStats._fields_}


def map_shape(grid: Grid, axis: int):
    a = axis & 3
    N = [grid.nx, grid.ny, grid.nz]
    b, c = (1, 2) if a == 0 else ((0, 2) if a == 1 else (0, 1))
    scale = 1 << (grid.nlevels - 1)
    return N[c] * scale, N[b] * scale


def map_image(ctx: Context, grid: Grid, freq, T: torch.Tensor, axis: int, image: torch.Tensor | None = None):
    npy, npx = map_shape(grid, axis)
    if image is None:
        image = torch.empty((npy, npx), dtype=torch.float32, device=T.device)
    f = _freq(freq)
    ctx.check(_lib.soc_map(ctx.h, grid.h, C.byref(f), _dev_ptr(T, torch.float32, "T"), int(axis),
                           _dev_ptr(image, torch.float32, "image"), npx, npy))
    return image


# ---------------------------------------------------------------- batches
class _BatchPair(C.Structure):
    _fields_ = [("grid", C.c_int32), ("freq_index", C.c_uint32), ("freq", _Freq), ("I_bg_nu", C.c_double),
                ("n_bg", C.c_uint64), ("n_ps", C.c_int32), ("ps", C.POINTER(_PointSource)), ("n_ps_pk", C.c_uint64),
                ("d_absorbed", C.c_void_p)]


ITER_ADVANCE = 0xFFFFFFFF

_lib.soc_batch_create.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_int32, C.POINTER(_BatchPair),
                                  C.c_uint64, C.c_uint64, C.POINTER(C.c_void_p)]
_lib.soc_batch_destroy.argtypes = [C.c_void_p]
_lib.soc_batch_info.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_uint64)]
_lib.soc_batch_run.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(_SimStats)]
_lib.soc_graph_begin.argtypes = [C.c_void_p]
_lib.soc_graph_end.argtypes = [C.c_void_p, C.POINTER(C.c_void_p)]
_lib.soc_graph_launch.argtypes = [C.c_void_p]
_lib.soc_graph_destroy.argtypes = [C.c_void_p]


class Batch:
    """soc_batch: (grid, frequency) pairs simulated by one persistent launch."""

    def __init__(self, ctx: Context, grids, pairs, seed=1, tile_packages=16384):
        """pairs: list of dicts with keys grid (index), freq (5-tuple),
        freq_index, absorbed (float64 CUDA tensor of that grid's ncells),
        I_bg, n_bg, and optionally ps_pos, ps_Lnu, n_ps_pk."""
        self.ctx, self.grids = ctx, list(grids)
        self._keep = []
        arr = (_BatchPair * len(pairs))()
        for i, q in enumerate(pairs):
            pos = np.asarray(q.get("ps_pos", np.zeros((0, 3))), dtype=np.float64).reshape(-1, 3)
            L = np.asarray(q.get("ps_Lnu", np.zeros(0)), dtype=np.float64).reshape(-1)
            ps = (_PointSource * max(len(pos), 1))(*[_PointSource(*pos[k], L[k]) for k in range(len(pos))])
            self._keep.append((ps, q["absorbed"]))
            arr[i] = _BatchPair(int(q["grid"]), int(q.get("freq_index", 0)), _freq(q["freq"]), float(q.get("I_bg", 0.0)),
                                int(q.get("n_bg", 0)), len(pos), C.cast(ps, C.POINTER(_PointSource)) if len(pos) else None,
                                int(q.get("n_ps_pk", 0)), _dev_ptr(q["absorbed"], torch.float64, "absorbed"))
        gh = (C.c_void_p * len(self.grids))(*[g.h.value if isinstance(g.h, C.c_void_p) else g.h for g in self.grids])
        h = C.c_void_p()
        ctx.check(_lib.soc_batch_create(ctx.h, len(self.grids), gh, len(pairs), arr, C.c_uint64(seed),
                                        C.c_uint64(tile_packages), C.byref(h)))
        self.h = h
        ctx._children.add(self)

    def info(self):
        nt, npk = C.c_int32(), C.c_uint64()
        self.ctx.check(_lib.soc_batch_info(self.h, C.byref(nt), C.byref(npk)))
        return nt.value, npk.value

    def run(self, iteration=0, stats=False):
        st = _SimStats() if stats else None
        self.ctx.check(_lib.soc_batch_run(self.h, C.c_uint32(iteration), C.byref(st) if st is not None else None))
        return None if st is None else {k: getattr(st, k) for k, _ in _SimStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            _lib.soc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured sequence of library calls (soc_graph_begin/end)."""

    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h
        ctx._children.add(self)

    def launch(self):
        rc = _lib.soc_graph_launch(self.h)
        if rc != OK:
            raise SocError(rc, "soc_graph_launch failed")

    def close(self):
        if getattr(self, "h", None):
            _lib.soc_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def graph_begin(ctx: Context):
    ctx.check(_lib.soc_graph_begin(ctx.h))


def graph_end(ctx: Context) -> Graph:
    h = C.c_void_p()
    ctx.check(_lib.soc_graph_end(ctx.h, C.byref(h)))
    return Graph(ctx, h)


_lib.soc_ubench.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_uint64, C.c_int32, C.c_int32,
                            C.c_int32, C.c_int32, C.POINTER(C.c_double)]


def ubench(ctx: Context, which: int, buf: torch.Tensor, buf2: torch.Tensor | None, n: int, per_thread: int,
           mode: int = 0, blocks: int = 4096, threads: int = 256) -> float:
    """soc_ubench: milliseconds of one micro-benchmark launch."""
    ms = C.c_double()
    ctx.check(_lib.soc_ubench(ctx.h, int(which), C.c_void_p(buf.data_ptr()),
                              C.c_void_p(buf2.data_ptr()) if buf2 is not None else None, C.c_uint64(n),
                              int(per_thread), int(mode), int(blocks), int(threads), C.byref(ms)))
    return ms.value


# ---------------------------------------------------------------- surrogate
class _UnetDesc(C.Structure):
    _fields_ = [("cin", C.c_int32), ("cout", C.c_int32), ("base", C.c_int32), ("levels", C.c_int32),
                ("nmax", C.c_int32), ("nz", C.c_int32), ("ny", C.c_int32), ("nx", C.c_int32)]


_lib.soc_unet_create.argtypes = [C.c_void_p, C.POINTER(_UnetDesc), C.c_uint64, C.POINTER(C.c_void_p)]
_lib.soc_unet_destroy.argtypes = [C.c_void_p]
_lib.soc_unet_param_count.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
_lib.soc_unet_flops.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]
for _n in ("soc_unet_set_params", "soc_unet_get_params", "soc_unet_get_grads"):
    getattr(_lib, _n).argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
_lib.soc_unet_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
_lib.soc_unet_backward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
_lib.soc_unet_mse.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.POINTER(C.c_double)]
_lib.soc_unet_backward_to.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]
_lib.soc_unet_read.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int64]
_lib.soc_unet_adam.argtypes = [C.c_void_p, C.c_void_p, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32]


_lib.soc_surrogate_features.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.c_double, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.c_void_p, C.c_void_p]
_lib.soc_surrogate_target.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                      C.c_double, C.c_void_p, C.c_int32, C.c_int32]
_lib.soc_surrogate_target_absorbed.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                                               C.c_void_p, C.c_int32, C.c_int32]
_lib.soc_surrogate_apply.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32,
                                     C.c_double, C.c_double, C.c_void_p, C.c_void_p]
_lib.soc_surrogate_apply_absorbed.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32,
                                              C.c_double, C.c_void_p, C.c_void_p]


def surrogate_features(ctx: Context, grid: Grid, table: TempTable, S: int, w_nu, sigma_abs, I_bg, sigma_v: float,
                       ps_pos, ps_Lnu, T1: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """soc_surrogate_features: float32 CUDA tensor [S, S, S, 4]."""
    P = C.POINTER(C.c_double)
    w = np.ascontiguousarray(w_nu, dtype=np.float64)
    sa = np.ascontiguousarray(sigma_abs, dtype=np.float64)
    I = np.ascontiguousarray(I_bg, dtype=np.float64)
    K = w.shape[0]
    if sa.shape != (K,) or I.shape != (K,):
        raise ValueError("w_nu, sigma_abs and I_bg need one value per frequency")
    pos = np.ascontiguousarray(ps_pos if ps_pos is not None else np.zeros((0, 3)), dtype=np.float64).reshape(-1, 3)
    L = np.ascontiguousarray(ps_Lnu if ps_Lnu is not None else np.zeros((0, K)), dtype=np.float64).reshape(-1, K)
    if L.shape[0] != pos.shape[0]:
        raise ValueError("one luminosity row per point source")
    if T1.numel() != grid.ncells:
        raise ValueError("T1 must hold one value per cell")
    if out is None:
        out = torch.empty((S, S, S, 4), dtype=torch.float32, device="cuda")
    if out.numel() != 4 * S ** 3:
        raise ValueError("out must hold [S, S, S, 4] values")
    ctx.check(_lib.soc_surrogate_features(ctx.h, grid.h, table.h, int(S), int(K), w.ctypes.data_as(P),
                                          sa.ctypes.data_as(P), I.ctypes.data_as(P), float(sigma_v), pos.shape[0],
                                          pos.ctypes.data_as(P), L.ctypes.data_as(P),
                                          _dev_ptr(T1, torch.float32, "T1"), _dev_ptr(out, torch.float32, "out")))
    return out


def _coarse(out, S, channels, name):
    if out is None:
        out = torch.empty((S, S, S, channels), dtype=torch.float32, device="cuda")
    if out.numel() % (S ** 3) != 0 or out.numel() // (S ** 3) != channels:
        raise ValueError(f"{name} must hold S^3 x {channels} values")
    return out


def surrogate_target(ctx: Context, grid: Grid, table: TempTable, S: int, T: torch.Tensor, T1: torch.Tensor,
                     scale: float, out: torch.Tensor | None = None, channels: int = 1,
                     channel: int = 0) -> torch.Tensor:
    """soc_surrogate_target into channel `channel` of a float32 CUDA
    tensor [S, S, S, channels]."""
    if T.numel() != grid.ncells or T1.numel() != grid.ncells:
        raise ValueError("T and T1 must hold one value per cell")
    out = _coarse(out, S, channels, "out")
    ctx.check(_lib.soc_surrogate_target(ctx.h, grid.h, table.h, int(S), _dev_ptr(T, torch.float32, "T"),
                                        _dev_ptr(T1, torch.float32, "T1"), float(scale),
                                        _dev_ptr(out, torch.float32, "out"), int(channels), int(channel)))
    return out


def surrogate_target_absorbed(ctx: Context, grid: Grid, S: int, A: torch.Tensor, A1: torch.Tensor, scale: float,
                              out: torch.Tensor | None = None, channels: int = 1, channel: int = 0) -> torch.Tensor:
    """soc_surrogate_target_absorbed into channel `channel` of a float32
    CUDA tensor [S, S, S, channels]."""
    if A.numel() != grid.ncells or A1.numel() != grid.ncells:
        raise ValueError("A and A1 must hold one value per cell")
    out = _coarse(out, S, channels, "out")
    ctx.check(_lib.soc_surrogate_target_absorbed(ctx.h, grid.h, int(S), _dev_ptr(A, torch.float64, "A"),
                                                 _dev_ptr(A1, torch.float64, "A1"), float(scale),
                                                 _dev_ptr(out, torch.float32, "out"), int(channels), int(channel)))
    return out


def surrogate_apply(ctx: Context, grid: Grid, table: TempTable, S: int, pred: torch.Tensor, scale: float,
                    offset: float, T1: torch.Tensor, out: torch.Tensor | None = None, channels: int = 1,
                    channel: int = 0) -> torch.Tensor:
    """soc_surrogate_apply: float32 CUDA tensor of ncells start
    temperatures from channel `channel` of pred [S, S, S, channels]."""
    _coarse(pred, S, channels, "pred")
    if T1.numel() != grid.ncells:
        raise ValueError("T1 must hold one value per cell")
    if out is None:
        out = torch.empty(grid.ncells, dtype=torch.float32, device="cuda")
    if out.numel() != grid.ncells:
        raise ValueError("out must hold one value per cell")
    ctx.check(_lib.soc_surrogate_apply(ctx.h, grid.h, table.h, int(S), _dev_ptr(pred, torch.float32, "pred"),
                                       int(channels), int(channel), float(scale), float(offset),
                                       _dev_ptr(T1, torch.float32, "T1"), _dev_ptr(out, torch.float32, "out")))
    return out


def surrogate_apply_absorbed(ctx: Context, grid: Grid, S: int, pred: torch.Tensor, scale: float, A1: torch.Tensor,
                             out: torch.Tensor | None = None, channels: int = 1, channel: int = 0) -> torch.Tensor:
    """soc_surrogate_apply_absorbed: float64 CUDA tensor of ncells absorbed
    energies from channel `channel` of pred [S, S, S, channels]."""
    _coarse(pred, S, channels, "pred")
    if A1.numel() != grid.ncells:
        raise ValueError("A1 must hold one value per cell")
    if out is None:
        out = torch.empty(grid.ncells, dtype=torch.float64, device="cuda")
    if out.numel() != grid.ncells:
        raise ValueError("out must hold one value per cell")
    ctx.check(_lib.soc_surrogate_apply_absorbed(ctx.h, grid.h, int(S), _dev_ptr(pred, torch.float32, "pred"),
                                                int(channels), int(channel), float(scale),
                                                _dev_ptr(A1, torch.float64, "A1"), _dev_ptr(out, torch.float64, "out")))
    return out


class UNet:
    """The 3-D U-Net surrogate (soc_unet_*): FP32 channels-last device
    tensors in and out, BF16 matrix-core convolutions inside."""

    def __init__(self, ctx: Context, cin: int, cout: int, base: int, levels: int, nmax: int, shape, seed: int = 0):
        nz, ny, nx = (int(v) for v in shape)
        self.ctx, self.cin, self.cout, self.nmax, self.shape = ctx, cin, cout, nmax, (nz, ny, nx)
        self.base, self.levels = base, levels
        d = _UnetDesc(cin, cout, base, levels, nmax, nz, ny, nx)
        h = C.c_void_p()
        ctx.check(_lib.soc_unet_create(ctx.h, C.byref(d), C.c_uint64(seed & (2**64 - 1)), C.byref(h)))
        self.h = h
        ctx._children.add(self)
        n = C.c_int64()
        ctx.check(_lib.soc_unet_param_count(h, C.byref(n)))
        self.param_count = n.value
        self.step = 0

    def flops(self, n: int) -> int:
        f = C.c_int64()
        self.ctx.check(_lib.soc_unet_flops(self.h, int(n), C.byref(f)))
        return f.value

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32).ravel()
        if a.size != self.param_count:
            raise ValueError(f"expected {self.param_count} parameters, got {a.size}")
        self.ctx.check(_lib.soc_unet_set_params(self.ctx.h, self.h, a.ctypes.data_as(C.c_void_p)))

    def _get(self, fn):
        a = np.empty(self.param_count, np.float32)
        self.ctx.check(fn(self.ctx.h, self.h, a.ctypes.data_as(C.c_void_p)))
        return a

    def get_params(self) -> np.ndarray:
        return self._get(_lib.soc_unet_get_params)

    def get_grads(self) -> np.ndarray:
        return self._get(_lib.soc_unet_get_grads)

    def _check_x(self, x, c, name):
        if x.dim() != 5 or tuple(x.shape[1:4]) != self.shape or x.shape[4] != c:
            raise ValueError(f"{name} must be [n, {self.shape[0]}, {self.shape[1]}, {self.shape[2]}, {c}]")
        return _dev_ptr(x, torch.float32, name)

    def forward(self, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        n = x.shape[0]
        px = self._check_x(x, self.cin, "x")
        if y is None:
            y = torch.empty((n,) + self.shape + (self.cout,), dtype=torch.float32, device=x.device)
        py = self._check_x(y, self.cout, "y")
        self.ctx.check(_lib.soc_unet_forward(self.ctx.h, self.h, int(n), px, py))
        return y

    def backward(self, dy: torch.Tensor):
        self.ctx.check(_lib.soc_unet_backward(self.ctx.h, self.h, self._check_x(dy, self.cout, "dy")))

    def backward_to(self, dy: torch.Tensor, layer: int):
        """Backward pass up to and including one layer (parameter order)."""
        self.ctx.check(_lib.soc_unet_backward_to(self.ctx.h, self.h, self._check_x(dy, self.cout, "dy"), int(layer)))

    def read(self, layer: int, which: int, n: int, positions: int, channels: int) -> np.ndarray:
        """A stored tensor of one layer as FP32 [n * positions, channels]
        (which: 0 forward input, 1 forward output, 2 output-side gradient,
        3 backward-data result)."""
        a = np.empty((n * positions, channels), np.float32)
        self.ctx.check(_lib.soc_unet_read(self.ctx.h, self.h, int(layer), int(which), a.ctypes.data_as(C.c_void_p),
                                          C.c_int64(a.size)))
        return a

    def mse(self, y: torch.Tensor, t: torch.Tensor, grad: bool = True, loss: bool = True):
        """(loss or None, dy or None)."""
        n = y.shape[0]
        dy = torch.empty_like(y) if grad else None
        out = C.c_double()
        self.ctx.check(_lib.soc_unet_mse(self.ctx.h, self.h, int(n), self._check_x(y, self.cout, "y"),
                                         self._check_x(t, self.cout, "t"),
                                         _dev_ptr(dy, torch.float32, "dy") if grad else None,
                                         C.byref(out) if loss else None))
        return (out.value if loss else None), dy

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, step: int | None = None):
        self.step = self.step + 1 if step is None else int(step)
        self.ctx.check(_lib.soc_unet_adam(self.ctx.h, self.h, lr, beta1, beta2, eps, self.step))

    def close(self):
        if getattr(self, "h", None):
            _lib.soc_unet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
