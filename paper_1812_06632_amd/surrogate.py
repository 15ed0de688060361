"""Learned starting temperatures for the plain iteration.

The paper shortens the iteration by starting it from a reference field
(Sect. 2.1.2) and measures convergence by the change of the temperatures
(Sect. 3.3).  Here the starting field comes from the 3-D U-Net of the
library (soc_unet_*): trained on clouds the plain method solved, it maps
a cloud and its point sources to how much the dust re-emission raises the
temperatures T1 of the constant sources (the plain method's first
iteration, which is run in any case).  The plain iterations that follow
the prediction keep the result unbiased; the stopping rule then acts as a
judge of the prediction (a poor start takes more iterations).

The network has two outputs per block: log10(T / T1) / Y_SCALE and
log10(A / A1) / A_SCALE, A the absorbed energy of the converged solution
and A1 the constant sources' part of it.  The first gives the start
temperatures (mode A: plain iterations from there); the second gives the
absorption that seeds a reference field (mode B, Sect. 2.1.2: the
reference-field iteration then averages Monte Carlo estimates into it, so
the prediction's weight falls as the packages accumulate).

Every step is a library call on the device: the network input
(soc_surrogate_features: optical depth of each block, flux of the
unattenuated point sources against the external field, the optically thin
temperature, and T1), the training targets (soc_surrogate_target and
soc_surrogate_target_absorbed), the network, and the start fields
(soc_surrogate_apply and soc_surrogate_apply_absorbed: the prediction
interpolated to the cells and applied to T1 and A1).  torch holds the
device arrays and the batches (random axis flips and permutations of the
training samples).
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import soc
from . import workloads as W
from .driver import PlainSolver

N_FEATURES = 4
N_OUT = 2
Y_SCALE = 0.1   # the network's output unit in log10(T / T1)
A_SCALE = 0.5   # and in log10(A / A1)
TAU_RANGE = (2.0, 100.0)


def random_problem(rng: np.random.Generator, n: int = 64, K: int = 32, packages: int = 200_000,
                   tau_range=TAU_RANGE) -> W.Problem:
    """A lognormal cloud of the training family: sigma_ln ~ U(0.5, 1.5),
    mean tau_V ~ log-U(tau_range), 0-2 blackbody sources at random cells
    with luminosities ~ log-U(1e5, 1e7) L_sun."""
    sigma = float(rng.uniform(0.5, 1.5))
    tau = float(math.exp(rng.uniform(math.log(tau_range[0]), math.log(tau_range[1]))))
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


def features(solver: PlainSolver, S: int, T1: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """[S, S, S, 4] device network input of the solver's problem given its
    constant-source temperatures T1 (soc_surrogate_features)."""
    P = solver.P
    return soc.surrogate_features(solver.ctx, solver.grid, solver.table, S, P.w, P.sigma_abs, P.I_bg, W.SIGMA_V,
                                  P.ps_pos if len(P.ps_pos) else None, P.ps_Lnu if len(P.ps_pos) else None,
                                  T1.reshape(-1), out=out)


def make_dataset(ctx: soc.Context, count: int, seed: int, n: int = 64, S: int = 64, K: int = 32,
                 packages: int = 200_000, max_iter: int = 10, tau_range=TAU_RANGE, log=None):
    """Device tensors (X [count, S, S, S, N_FEATURES], Y [count, S, S, S,
    N_OUT]): random clouds solved by the plain method to the 1% rule; X
    from their constant-source temperatures, Y the targets of their
    solution (temperatures, absorbed energies)."""
    rng = np.random.default_rng(seed)
    X = torch.empty((count, S, S, S, N_FEATURES), dtype=torch.float32, device="cuda")
    Y = torch.empty((count, S, S, S, N_OUT), dtype=torch.float32, device="cuda")
    t0 = time.time()
    for m in range(count):
        P = random_problem(rng, n, K, packages, tau_range)
        solver = PlainSolver(ctx, P, seed=seed * 100003 + m)
        _, at = solver.run(max_iter=max_iter)
        features(solver, S, solver.T1, out=X[m])
        soc.surrogate_target(ctx, solver.grid, solver.table, S, solver.T, solver.T1, Y_SCALE, out=Y[m],
                             channels=N_OUT, channel=0)
        soc.surrogate_target_absorbed(ctx, solver.grid, S, solver.A, solver.A_const, A_SCALE, out=Y[m],
                                      channels=N_OUT, channel=1)
        if log and (m + 1) % 32 == 0:
            torch.cuda.synchronize()
            log(f"training cloud {m + 1}/{count} solved ({time.time() - t0:.1f}s, last stopped at iteration {at})")
    torch.cuda.synchronize()
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
    """The U-Net on S^3 blocks."""

    def __init__(self, ctx: soc.Context, S: int = 64, base: int = 32, levels: int = 4, batch: int = 4,
                 seed: int = 0):
        self.ctx, self.S, self.batch = ctx, S, batch
        self.net = soc.UNet(ctx, N_FEATURES, N_OUT, base, levels, batch, (S, S, S), seed=seed)

    def fit(self, X: torch.Tensor, Y: torch.Tensor, steps: int, lr: float = 3e-4, warmup: int = 200, seed: int = 0,
            log=None):
        """Adam on the MSE of the target (device tensors from make_dataset);
        the step size rises linearly over `warmup` steps, then decays on a
        cosine to zero."""
        g = torch.Generator().manual_seed(seed)
        losses = []
        t0 = time.time()
        for step in range(1, steps + 1):
            idx = torch.randint(0, X.shape[0], (self.batch,), generator=g).cuda()
            xb, yb = _augment(X[idx], Y[idx], g)
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

    def predict(self, solver: PlainSolver, T1: torch.Tensor) -> torch.Tensor:
        """Network output [1, S, S, S, N_OUT] for the solver's problem from
        its constant-source temperatures T1."""
        return self.net.forward(features(solver, self.S, T1)[None])

    def predict_T(self, solver: PlainSolver, T1: torch.Tensor, out: torch.Tensor | None = None,
                  y: torch.Tensor | None = None) -> torch.Tensor:
        """Start temperatures (device FP32, one per cell; 0 in empty cells)
        of the solver's regular cubic problem, whose size is a multiple of
        S, from its constant-source temperatures T1: library calls only,
        no host round trip.  y: a network output already computed."""
        y = self.predict(solver, T1) if y is None else y
        return soc.surrogate_apply(self.ctx, solver.grid, solver.table, self.S, y, Y_SCALE, 0.0, T1.reshape(-1),
                                   out=out, channels=N_OUT, channel=0)

    def predict_A(self, solver: PlainSolver, A1: torch.Tensor, y: torch.Tensor,
                  out: torch.Tensor | None = None) -> torch.Tensor:
        """Absorbed energies (device FP64 per cell) of the predicted
        solution, from the constant sources' absorption A1 and a network
        output y."""
        return soc.surrogate_apply_absorbed(self.ctx, solver.grid, self.S, y, A_SCALE, A1.reshape(-1), out=out,
                                            channels=N_OUT, channel=1)

    def close(self):
        self.net.close()
