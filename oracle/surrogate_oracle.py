"""Oracle of the learned start's input, target and output maps (test
infrastructure: only tests, the smoke check and the benchmark's CPU
baseline may import it).

The paper starts the dust iterations from a reference field to need fewer
of them (Sect. 2.1.2) and judges convergence by the change of the
temperatures (Sect. 3.3).  The library's learned start predicts, on S^3
blocks of b^3 cells of a regular n^3 grid, how much the dust re-emission
raises the temperatures T1 that the constant sources alone give.  This
module writes out, plainly and in FP64, what the library's three maps
compute:

  features(...)          -> [S, S, S, 4]   network input
  target(...)            -> [S, S, S]      block mean of log10(T / T1) / scale
  target_absorbed(...)   -> [S, S, S]      block mean of log10(A / A1) / scale
  apply(...)             -> [n^3]          T1 10^(interpolated output), clamped
  apply_absorbed(...)    -> [n^3]          A1 10^(interpolated output)

Definitions (block centre r = (x + 1/2, y + 1/2, z + 1/2) in block units,
block edge s cm, sources p at r_p = (root position) / b):
  d_p^2 = (|r - r_p|^2 + 1/4) s^2
  0: log10(sigma_V <n> s + 1e-4) / 2
  1: log10(1 + sum_p L_p / (4 pi d_p^2) / F_ext) / 4,
     L_p = sum_k w_k L_p,k,  F_ext = 4 pi sum_k w_k I_k
  2: (log10 T_thin - 1.5) / 0.5 with T_thin the root of
     sum_k w_k sigma_k B(nu_k, T) = sum_k w_k sigma_k I_k
                                    + sum_p sum_k w_k sigma_k L_p,k / (16 pi^2 d_p^2)
     (found by bisection in log T on [T_floor, T_max], clamped there)
  3: (mean over the block of log10 T1' - 1.5) / 0.5
where T' is T_floor in cells of density 0 and max(T, T_floor) elsewhere.
For the absorbed energies (A the field's, A1 the constant sources') a
cell counts log10(A / A1) where it has dust and A1, A > 0, else 0.
The interpolation of apply maps fine cell j to coarse coordinate
(j + 1/2) / b - 1/2, clamped below at 0, and interpolates linearly
between the two nearest coarse cells along each axis (the upper one
clamped at S - 1).

Pins (tests/test_surrogate_oracle.py): brute-force block means, the grey
dust closed form T_thin^4 = L / (16 pi d^2 sigma_SB) of a point source,
the external-field-only temperature against a direct root of the Planck
sum, and the interpolation against torch's trilinear upsampling.
"""
from __future__ import annotations

import math

import numpy as np

H = 6.62607015e-27
K_B = 1.380649e-16
C_LIGHT = 2.99792458e10


def planck(nu: np.ndarray, T: float) -> np.ndarray:
    """B_nu(T), erg s-1 cm-2 Hz-1 sr-1."""
    x = H * nu / (K_B * T)
    return 2.0 * H * nu ** 3 / C_LIGHT ** 2 / np.expm1(np.minimum(x, 700.0))


def thin_temperature(emit_nu, emit_w, emit_sigma, Jw: float, T_floor: float, T_max: float) -> float:
    """Root T of sum_k w_k sigma_k B(nu_k, T) = Jw (bisection in log T),
    clamped to [T_floor, T_max]."""
    ws = np.asarray(emit_w) * np.asarray(emit_sigma)
    nu = np.asarray(emit_nu)

    def f(lt):
        return float(ws @ planck(nu, math.exp(lt))) - Jw

    lo, hi = math.log(T_floor), math.log(T_max)
    if f(lo) >= 0.0:
        return T_floor
    if f(hi) <= 0.0:
        return T_max
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        if f(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    return math.exp(0.5 * (lo + hi))


def _floored(density: np.ndarray, T: np.ndarray, T_floor: float) -> np.ndarray:
    return np.where(density > 0, np.maximum(T.astype(np.float64), T_floor), T_floor)


def _block_mean(a: np.ndarray, S: int) -> np.ndarray:
    """Mean of every b^3 block of a cubic (z, y, x) array (plain loops over
    the blocks)."""
    n = a.shape[0]
    b = n // S
    out = np.empty((S, S, S))
    for z in range(S):
        for y in range(S):
            for x in range(S):
                out[z, y, x] = a[z * b:(z + 1) * b, y * b:(y + 1) * b, x * b:(x + 1) * b].mean()
    return out


def features(density: np.ndarray, root_cell_cm: float, S: int, T1: np.ndarray, w, sigma_abs, I_bg,
             sigma_v: float, ps_pos, ps_Lnu, emit_nu, emit_w, emit_sigma, T_floor: float,
             T_max: float, blocks=None) -> np.ndarray:
    """[S, S, S, 4] float64 network input (module docstring), or, given a
    list of blocks (z, y, x), their [len(blocks), 4] rows only."""
    n = round(len(density) ** (1.0 / 3.0))
    rho = density.reshape(n, n, n).astype(np.float64)
    b = n // S
    s = root_cell_cm * b
    w = np.asarray(w, np.float64)
    sig = np.asarray(sigma_abs, np.float64)
    I = np.asarray(I_bg, np.float64)
    F_ext = 4.0 * math.pi * float(w @ I)
    J_bg = float((w * sig) @ I)
    pos = np.asarray(ps_pos, np.float64).reshape(-1, 3) / b
    Lnu = np.asarray(ps_Lnu, np.float64).reshape(pos.shape[0], w.shape[0])
    L = Lnu @ w
    Lw = Lnu @ (w * sig)
    logT1 = np.log10(_floored(rho, T1.reshape(n, n, n), T_floor))
    want = blocks if blocks is not None else [(z, y, x) for z in range(S) for y in range(S) for x in range(S)]
    rows = np.empty((len(want), 4))
    for i, (z, y, x) in enumerate(want):
        blk = (slice(z * b, (z + 1) * b), slice(y * b, (y + 1) * b), slice(x * b, (x + 1) * b))
        r = np.array([x + 0.5, y + 0.5, z + 0.5])
        ratio, Jw = 0.0, J_bg
        for p in range(pos.shape[0]):
            d2 = (float(((r - pos[p]) ** 2).sum()) + 0.25) * s * s
            ratio += L[p] / (4.0 * math.pi * d2)
            Jw += Lw[p] / (16.0 * math.pi ** 2 * d2)
        Tt = thin_temperature(emit_nu, emit_w, emit_sigma, Jw, T_floor, T_max)
        rows[i, 0] = math.log10(sigma_v * rho[blk].mean() * s + 1e-4) / 2.0
        rows[i, 1] = math.log10(1.0 + ratio / F_ext) / 4.0
        rows[i, 2] = (math.log10(Tt) - 1.5) / 0.5
        rows[i, 3] = (logT1[blk].mean() - 1.5) / 0.5
    return rows if blocks is not None else rows.reshape(S, S, S, 4)


def target(density: np.ndarray, S: int, T: np.ndarray, T1: np.ndarray, T_floor: float, scale: float) -> np.ndarray:
    """[S, S, S]: block mean of log10(T' / T1') divided by scale."""
    n = round(len(density) ** (1.0 / 3.0))
    rho = density.reshape(n, n, n)
    lr = np.log10(_floored(rho, T.reshape(n, n, n), T_floor)) - np.log10(_floored(rho, T1.reshape(n, n, n), T_floor))
    return _block_mean(lr, S) / scale


def _axis_weights(n: int, S: int):
    """For every fine index j: (i0, i1, t) of the interpolation along one
    axis."""
    out = []
    for j in range(n):
        u = max((j + 0.5) * S / n - 0.5, 0.0)
        i0 = min(int(math.floor(u)), S - 1)
        out.append((i0, min(i0 + 1, S - 1), u - i0))
    return out


def upsample(pred: np.ndarray, n: int) -> np.ndarray:
    """[n, n, n] trilinear interpolation of an [S, S, S] field."""
    S = pred.shape[0]
    wts = _axis_weights(n, S)
    out = np.empty((n, n, n))
    for z in range(n):
        z0, z1, tz = wts[z]
        for y in range(n):
            y0, y1, ty = wts[y]
            for x in range(n):
                x0, x1, tx = wts[x]
                v = 0.0
                for zi, wz in ((z0, 1 - tz), (z1, tz)):
                    for yi, wy in ((y0, 1 - ty), (y1, ty)):
                        for xi, wx in ((x0, 1 - tx), (x1, tx)):
                            v += wz * wy * wx * pred[zi, yi, xi]
                out[z, y, x] = v
    return out


def apply(density: np.ndarray, pred: np.ndarray, scale: float, offset: float, T1: np.ndarray, T_floor: float,
          T_max: float) -> np.ndarray:
    """[n^3] start temperatures: T1' 10^(upsampled pred * scale + offset)
    clamped to [T_floor, T_max], 0 where the density is 0."""
    n = round(len(density) ** (1.0 / 3.0))
    r = upsample(np.asarray(pred, np.float64).reshape(pred.shape[0], pred.shape[0], pred.shape[0]), n)
    r = r.reshape(-1) * scale + offset
    T1f = np.maximum(T1.astype(np.float64), T_floor)
    T = np.clip(T1f * 10.0 ** r, T_floor, T_max)
    return np.where(density.reshape(-1) > 0, T, 0.0)


def target_absorbed(density: np.ndarray, S: int, A: np.ndarray, A1: np.ndarray, scale: float) -> np.ndarray:
    """[S, S, S]: block mean of log10(A / A1) (0 where a cell is empty or
    either value is not > 0) divided by scale."""
    n = round(len(density) ** (1.0 / 3.0))
    A = np.asarray(A, np.float64)
    A1 = np.asarray(A1, np.float64)
    ok = (density > 0) & (A1 > 0) & (A > 0)
    lr = np.zeros(n ** 3)
    lr[ok] = np.log10(A[ok] / A1[ok])
    return _block_mean(lr.reshape(n, n, n), S) / scale


def apply_absorbed(density: np.ndarray, pred: np.ndarray, scale: float, A1: np.ndarray) -> np.ndarray:
    """[n^3] absorbed energies A1 10^(upsampled pred * scale), 0 where the
    density is 0."""
    n = round(len(density) ** (1.0 / 3.0))
    S = pred.shape[0]
    r = upsample(np.asarray(pred, np.float64).reshape(S, S, S), n).reshape(-1) * scale
    A = np.asarray(A1, np.float64) * 10.0 ** r
    return np.where(density.reshape(-1) > 0, A, 0.0)
