"""Learned starting temperatures for the plain iteration.

The paper shortens the iteration by starting it from a reference field
(Sect. 2.1.2).  Here the starting field comes from the 3-D U-Net of the
library (soc_unet_*): trained on clouds the plain method solved, it maps
a density field and its point sources to the temperature field, and the
plain iterations that follow the prediction keep the result unbiased (the
stopping rule then acts as a judge of the prediction: a poor start simply
takes more iterations).

Inputs of the network (channels-last, S^3 cells, block averages of the
cloud): the log10 of the optical depth of one cell at 0.55 um; the log10
of 1 + the ratio of the unattenuated bolometric flux of the point
sources, sum L / (4 pi d^2), to the bolometric 4 pi J of the external
field; the optically thin temperature of the cell -- the solution of
4 pi sum_k w_k sigma_k B(nu_k, T) = 4 pi sum_k w_k sigma_k J_k with J the
external field plus the unattenuated sources, L_nu / (16 pi^2 d^2); and
the temperature T1 the constant sources alone give (the plain method's
first iteration, which is run in any case).  Output: log10(T / T1), the
part the dust re-emission adds and the iteration has to build up,
normalised by the training-set mean and standard deviation.  The start
field is T1 times the predicted ratio; on a finer grid the ratio is
trilinearly interpolated and applied to T1 at full resolution, so the
structure that T1 resolves is kept.

Everything runs on the device through the library; torch supplies the
device arrays and the elementwise glue (normalisation, flips, the
interpolation of the prediction).
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import soc
from . import workloads as W
from .driver import PlainSolver


def block_mean(a: np.ndarray, S: int) -> np.ndarray:
    n = a.shape[0]
    if a.shape != (n, n, n) or n % S:
        raise ValueError("cubic field with a size divisible by S expected")
    b = n // S
    return a.reshape(S, b, S, b, S, b).mean(axis=(1, 3, 5))


_ISRF_BOL = None


def _isrf_bolometric() -> float:
    """Frequency integral of the external field's intensity (cached)."""
    global _ISRF_BOL
    if _ISRF_BOL is None:
        _ISRF_BOL = W.isrf_integral()
    return _ISRF_BOL


N_FEATURES = 4


def _planck(nu: np.ndarray, T: np.ndarray) -> np.ndarray:
    """B_nu(T) in erg s-1 cm-2 Hz-1 sr-1 (outer product of T and nu)."""
    x = W._H * nu[None, :] / (W._K * T[:, None])
    return 2.0 * W._H * nu[None, :] ** 3 / W._C ** 2 / np.expm1(np.minimum(x, 700.0))


def thin_temperature(P: W.Problem, Jw: np.ndarray) -> np.ndarray:
    """Equilibrium temperature of dust whose absorption is
    Jw = sum_k w_k sigma_k J_k (per cell, J the mean intensity on the
    problem's frequency grid), without attenuation: the root of
    sum_k w_k sigma_k B(nu_k, T) = Jw, from a log-log table of the emission
    on [T_floor, T_max]."""
    ws = P.w * P.sigma_abs
    Tg = np.exp(np.linspace(math.log(P.T_floor), math.log(P.T_max), 1024))
    lg_emit = np.log(_planck(P.nu, Tg) @ ws)
    lg_in = np.log(np.maximum(np.asarray(Jw, dtype=np.float64), 1e-300))
    return np.exp(np.interp(lg_in, lg_emit, np.log(Tg)))


def _log_T(P: W.Problem, T: np.ndarray) -> np.ndarray:
    """log10 of a temperature field with empty and unset cells at the floor."""
    rho = P.grid.density()
    return np.log10(np.where(rho > 0, np.maximum(T, P.T_floor), P.T_floor))


def features(P: W.Problem, S: int, T1: np.ndarray) -> np.ndarray:
    """[S, S, S, 4] float32 network input of a regular cubic problem whose
    constant-source temperatures are T1 (one per cell)."""
    g = P.grid
    if g.nlevels != 1 or not (g.nx == g.ny == g.nz):
        raise ValueError("the surrogate takes regular cubic grids")
    n = g.nx
    rho = block_mean(g.density().reshape(n, n, n).astype(np.float64), S)
    cell = g.root_cell_cm * n / S
    f0 = np.log10(W.SIGMA_V * rho * cell + 1e-4) / 2.0
    c = (np.arange(S) + 0.5)
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    ratio = np.zeros((S, S, S))
    ws = P.w * P.sigma_abs
    Jw = np.full((S, S, S), float(P.I_bg @ ws))   # external field, isotropic: J = I
    if len(P.ps_pos):
        Lbol = (P.ps_Lnu * P.w[None, :]).sum(axis=1)
        f_ext = 4.0 * math.pi * _isrf_bolometric()
        for (px, py, pz), L, Lnu in zip(np.asarray(P.ps_pos) * S / n, Lbol, P.ps_Lnu):
            d2 = ((xx - px) ** 2 + (yy - py) ** 2 + (zz - pz) ** 2 + 0.25) * cell * cell   # cm^2, softened
            ratio += L / (4.0 * math.pi * d2) / f_ext
            Jw += float(Lnu @ ws) / (16.0 * math.pi ** 2 * d2)
    f1 = np.log10(1.0 + ratio) / 4.0
    f2 = (np.log10(thin_temperature(P, Jw.reshape(-1))).reshape(S, S, S) - 1.5) / 0.5
    f3 = (block_mean(_log_T(P, T1).reshape(n, n, n), S) - 1.5) / 0.5
    return np.stack([f0, f1, f2, f3], axis=-1).astype(np.float32)


def targets(P: W.Problem, T: np.ndarray, T1: np.ndarray, S: int) -> np.ndarray:
    """[S, S, S, 1] float64: block means of log10(T / T1) (empty cells at
    the floor temperature on both sides, so they contribute zero)."""
    n = P.grid.nx
    return block_mean((_log_T(P, T) - _log_T(P, T1)).reshape(n, n, n), S)[..., None]


TAU_RANGE = (2.0, 100.0)


def random_problem(rng: np.random.Generator, n: int = 64, K: int = 32, packages: int = 200_000) -> W.Problem:
    """A lognormal cloud of the training family: sigma_ln ~ U(0.5, 1.5),
    mean tau_V ~ log-U(2, 100), 0-2 blackbody sources at random cells with
    luminosities ~ log-U(1e5, 1e7) L_sun."""
    sigma = float(rng.uniform(0.5, 1.5))
    tau = float(math.exp(rng.uniform(math.log(TAU_RANGE[0]), math.log(TAU_RANGE[1]))))
    nsrc = int(rng.integers(0, 3))
    pos = tuple(tuple(float(v) for v in rng.uniform(0.15, 0.85, 3)) for _ in range(nsrc))
    L = np.exp(rng.uniform(math.log(1e5), math.log(1e7), nsrc))
    P = W.lognormal_problem(n=n, K=K, sigma_ln=sigma, tau_v_mean=tau, seed=int(rng.integers(1 << 30)),
                            L_star_lsun=1.0, ps_frac=pos, packages_per_freq=packages)
    if nsrc:
        P.ps_Lnu = P.ps_Lnu * L[:, None]
    else:
        P.ps_pos = np.zeros((0, 3))
        P.ps_Lnu = np.zeros((0, K))
        P.n_bg = packages
        P.n_ps_pk = 0
    return P


def make_dataset(ctx: soc.Context, count: int, seed: int, n: int = 64, S: int = 64, K: int = 32,
                 packages: int = 200_000, max_iter: int = 10, log=None):
    """(X [count, S, S, S, N_FEATURES] float32, Y [count, S, S, S, 1]
    float64): random clouds solved by the plain method to the 1% rule."""
    rng = np.random.default_rng(seed)
    X = np.empty((count, S, S, S, N_FEATURES), np.float32)
    Y = np.empty((count, S, S, S, 1), np.float64)
    t0 = time.time()
    for m in range(count):
        P = random_problem(rng, n, K, packages)
        solver = PlainSolver(ctx, P, seed=seed * 100003 + m)
        _, at = solver.run(max_iter=max_iter)
        T1 = solver.T1.cpu().numpy().astype(np.float64)
        X[m] = features(P, S, T1)
        Y[m] = targets(P, solver.T.cpu().numpy().astype(np.float64), T1, S)
        if log and (m + 1) % 16 == 0:
            log(f"training cloud {m + 1}/{count} solved ({time.time() - t0:.1f}s, last stopped at iteration {at})")
    return X, Y


def _augment(x: torch.Tensor, y: torch.Tensor, g: torch.Generator):
    """The same random axis flips and axis permutation for input and target
    (the transport is symmetric under both)."""
    flips = [d + 1 for d in range(3) if torch.rand((), generator=g).item() < 0.5]
    if flips:
        x, y = x.flip(flips), y.flip(flips)
    perm = torch.randperm(3, generator=g).tolist()
    order = [0] + [p + 1 for p in perm] + [4]
    return x.permute(order).contiguous(), y.permute(order).contiguous()


class Surrogate:
    """The U-Net with its target normalisation."""

    def __init__(self, ctx: soc.Context, S: int = 64, base: int = 32, levels: int = 4, batch: int = 4,
                 seed: int = 0):
        self.ctx, self.S, self.batch = ctx, S, batch
        self.net = soc.UNet(ctx, N_FEATURES, 1, base, levels, batch, (S, S, S), seed=seed)
        self.ymean = 0.0
        self.ystd = 1.0

    def fit(self, X: np.ndarray, Y: np.ndarray, steps: int, lr: float = 3e-4, warmup: int = 200, seed: int = 0,
            log=None):
        """Adam on the MSE of the normalised log ratio; the step size rises
        linearly over `warmup` steps, then decays on a cosine to zero."""
        self.ymean = float(Y.mean())
        self.ystd = float(Y.std()) + 1e-6
        Xd = torch.from_numpy(X).cuda()
        Yd = torch.from_numpy(((Y - self.ymean) / self.ystd).astype(np.float32)).cuda()
        g = torch.Generator().manual_seed(seed)
        losses = []
        t0 = time.time()
        for step in range(1, steps + 1):
            idx = torch.randint(0, X.shape[0], (self.batch,), generator=g)
            xb, yb = _augment(Xd[idx.cuda()], Yd[idx.cuda()], g)
            y = self.net.forward(xb)
            want = step % 100 == 0 or step == steps
            loss, dy = self.net.mse(y, yb, grad=True, loss=want)
            self.net.backward(dy)
            if step <= warmup:
                lr_t = lr * step / warmup
            else:
                lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * (step - warmup) / max(steps - warmup, 1)))
            self.net.adam(lr=lr_t)
            if want:
                losses.append((step, loss))
                if log:
                    log(f"training step {step}/{steps}: loss {loss:.4f} ({time.time() - t0:.1f}s)")
        return losses

    def predict_T(self, P: W.Problem, T1: torch.Tensor) -> torch.Tensor:
        """Start temperatures (device FP32, one per cell; 0 in empty cells)
        of a regular cubic problem whose size is a multiple of S, from its
        constant-source temperatures T1 (device, one per cell)."""
        n = P.grid.nx
        x = torch.from_numpy(features(P, self.S, T1.cpu().numpy().astype(np.float64))[None]).cuda()
        y = self.net.forward(x)
        lr = y[..., 0] * self.ystd + self.ymean            # log10(T / T1) at S^3
        if n != self.S:
            lr = torch.nn.functional.interpolate(lr[:, None], size=(n, n, n), mode="trilinear",
                                                 align_corners=False)[:, 0]
        rho = torch.from_numpy(P.grid.density()).cuda()
        T1c = torch.clamp(T1.reshape(-1).float(), min=P.T_floor)
        T = (T1c * torch.pow(10.0, lr.reshape(-1).float())).clamp(P.T_floor, P.T_max)
        return torch.where(rho > 0, T, torch.zeros_like(T))

    def close(self):
        self.net.close()
