"""Iteration drivers (Sect. 2.1.2, 3.3, 3.6 of the paper).

Plain method: the constant sources (external field, point sources) are
simulated once at every frequency and their absorbed energies kept; each
later iteration re-simulates the dust emission at the current temperatures
on top of the kept absorption and solves new temperatures.  The run stops
when the relative change of the mean temperature, over all cells and over
the hottest 5% of cells, falls below the tolerance between two consecutive
iterations (the paper's two convergence statistics).

Reference-field method, two readings of Sect. 2.1.2: "correction" -- each
dust iteration simulates only the difference between the current emission
and a reference emission (packages of either sign), adds their absorption
to the reference absorption, and moves both references to the
package-weighted running mean; "average" -- each dust iteration simulates
the whole emission and the temperatures come from the package-weighted
running mean of the absorption estimates (one stored number per cell).
The number of packages may grow over the iterations (a geometric
schedule).

Diagonal ALI (Sect. 2.1.2, 4.1, plain iteration): the dust packages count
what they deposit in their own emitting cell apart, and the temperature
solve takes each cell's own absorption-emission cycle exactly.

Control flow only: every step is a call through the C-ABI library; the
stopping rule compares two scalars the temperature kernel returns.
"""
from __future__ import annotations

import time

import torch

from . import soc


def converged(prev: dict, cur: dict, tol: float = 0.01) -> bool:
    """Relative change of <T> and of the hottest-5% mean both below tol."""
    return (abs(cur["mean_T"] - prev["mean_T"]) < tol * prev["mean_T"]
            and abs(cur["hot5_mean_T"] - prev["hot5_mean_T"]) < tol * prev["hot5_mean_T"])


class PlainSolver:
    """One problem (workloads.Problem) resident on the device."""

    def __init__(self, ctx: soc.Context, P, seed: int = 1, nT: int = 4096, packages=None, cap: float = 0.0,
                 ali: bool = False, multi: bool = True):
        """packages(it): dust packages per frequency of iteration it
        (default P.n_dust); cap: expected packages per cell at most (0 =
        none); ali: diagonal ALI (Sect. 2.1.2) in the dust iterations;
        multi: every frequency of a pass in one launch
        (soc_simulate_frequencies) rather than one launch per frequency --
        the same packages and results up to FP64 summation order."""
        self.ctx, self.P, self.seed = ctx, P, seed
        self.packages = packages
        self.cap = float(cap)
        self.ali = bool(ali)
        self.multi = bool(multi)
        self.grid = soc.grid_from_workload(ctx, P.grid)
        self.table = soc.temp_table_build(ctx, P.emit_nu, P.emit_w, P.emit_sigma_abs, P.T_floor, P.T_max, nT)
        nc = P.grid.ncells
        dev = "cuda"
        self.A_const = torch.zeros(nc, dtype=torch.float64, device=dev)
        self.A = torch.zeros(nc, dtype=torch.float64, device=dev)
        self.T = torch.zeros(nc, dtype=torch.float32, device=dev)
        self.T_new = torch.zeros(nc, dtype=torch.float32, device=dev)
        self.freqs = [(float(P.nu[k]), float(P.w[k]), float(P.sigma_abs[k]), float(P.sigma_sca[k]), float(P.g[k]))
                      for k in range(P.K)]
        self.S_ali = torch.zeros(nc, dtype=torch.float64, device=dev) if self.ali else None
        self.E_ali = torch.zeros(nc, dtype=torch.float64, device=dev) if self.ali else None

    def constant_pass(self) -> dict:
        """Iteration 1: the constant sources at every frequency, then the
        temperatures they alone give (dust emission is zero at T = 0)."""
        P = self.P
        self.A_const.zero_()
        have_ps = len(P.ps_pos) > 0
        src = [dict(I_bg=float(P.I_bg[k]), ps_pos=P.ps_pos if have_ps else None,
                    ps_Lnu=P.ps_Lnu[:, k] if have_ps else None, n_bg=P.n_bg, n_ps_pk=P.n_ps_pk if have_ps else 0)
               for k in range(P.K)]
        self._simulate(self.A_const, src, iteration=1)
        return soc.update_temperature(self.ctx, self.grid, self.table, self.A_const, self.T, None, stats=True)

    def _simulate(self, A: torch.Tensor, sources, iteration: int):
        """One pass over every frequency (source keyword sets per
        frequency) into A: one launch, or one per frequency."""
        if self.multi:
            soc.simulate_frequencies(self.ctx, self.grid, self.freqs, A, sources, range(self.P.K), seed=self.seed,
                                     iteration=iteration)
            return
        for k, q in enumerate(sources):
            soc.simulate_frequency(self.ctx, self.grid, self.freqs[k], A, seed=self.seed, iteration=iteration,
                                   freq_index=k, **q)

    def set_temperature(self, T0: torch.Tensor) -> dict:
        """Start the dust iterations from T0 instead of the constant-source
        temperatures; returns its statistics (absorption unchanged)."""
        self.T.copy_(T0.to(self.T.dtype).reshape(-1))
        return self.temperature_stats(self.T)

    def temperature_stats(self, T: torch.Tensor) -> dict:
        """<T> and hottest-5% mean of a given field (library kernels)."""
        return soc.temperature_stats(self.ctx, self.grid, self.table, T.reshape(-1))

    def dust_iteration(self, it: int) -> dict:
        """Dust emission at the current temperatures on top of the kept
        constant-source absorption, then the temperature solve."""
        P = self.P
        n = self.n_packages(it)
        self.A.copy_(self.A_const)
        if self.ali:
            self.S_ali.zero_()
            self.E_ali.zero_()
            self._simulate(self.A, [dict(T=self.T, n_dust=n, dust_mode=1, dust_cap=self.cap, ali_self=self.S_ali,
                                         ali_emitted=self.E_ali)] * P.K, iteration=it)
        else:
            self._simulate(self.A, [dict(T=self.T, n_dust=n, dust_mode=1, dust_cap=self.cap)] * P.K, iteration=it)
        s = soc.update_temperature(self.ctx, self.grid, self.table, self.A, self.T_new, self.T, stats=True,
                                   ali_self=self.S_ali, ali_emitted=self.E_ali)
        self.T.copy_(self.T_new)
        s["packages"] = n
        return s

    def n_packages(self, it: int) -> int:
        return int(self.packages(it)) if self.packages is not None else int(self.P.n_dust)

    def run(self, max_iter: int = 30, tol: float = 0.01, T0=None, log=None, on_iter=None, until_stop: bool = True):
        """Constant pass, optional start temperatures, dust iterations until
        the stopping rule (or, with until_stop False, all max_iter of them).
        T0 is a field, or a callable that maps the constant-source
        temperatures to the start field; the constant-source temperatures
        are kept in self.T1.  on_iter(iteration, T) is called after every
        iteration (outside the timing it reports).  Returns (history,
        converged_at) where history holds (iteration, wall seconds since
        the start, statistics) and converged_at is the first iteration that
        met the stopping rule."""
        torch.cuda.synchronize()
        t0 = time.time()
        s = self.constant_pass()
        self.T1 = self.T.clone()
        hist = [(1, time.time() - t0, s)]
        if T0 is not None:
            s = self.set_temperature(T0(self.T1) if callable(T0) else T0)
            hist[-1] = (1, time.time() - t0, s)
        if log:
            log(f"iteration 1: <T> {s['mean_T']:.3f} K hot5 {s['hot5_mean_T']:.3f} K")
        paused = 0.0
        if on_iter:
            tp = time.time()
            on_iter(1, self.T)
            paused += time.time() - tp
        at = None
        for it in range(2, max_iter + 1):
            s = self.dust_iteration(it)
            hist.append((it, time.time() - t0 - paused, s))
            if log:
                log(f"iteration {it}: <T> {s['mean_T']:.3f} K hot5 {s['hot5_mean_T']:.3f} K")
            if on_iter:
                tp = time.time()
                on_iter(it, self.T)
                paused += time.time() - tp
            if at is None and converged(hist[-2][2], s, tol):
                at = it
                if until_stop:
                    break
        return hist, at


def geometric_schedule(n_final: int, factor: float, iterations: int):
    """Packages per frequency for dust iterations 2..iterations, growing so
    that log n is linear in the iteration number, from n_final / factor at
    iteration 2 to n_final at the last (Sect. 3.6)."""
    if iterations < 2 or factor < 1.0 or n_final < 1:
        raise ValueError("need iterations >= 2, factor >= 1, n_final >= 1")

    def n(it: int) -> int:
        if iterations == 2:
            return n_final
        t = min(max((it - 2) / (iterations - 2), 0.0), 1.0)
        return max(1, int(round(n_final * factor ** (t - 1.0))))

    return n


class ReferenceFieldSolver(PlainSolver):
    """Reference-field iteration (Sect. 2.1.2).  Dust iteration i uses
    n_i packages per frequency and the weight beta_i = n_i / (n_2 + ... +
    n_i); after the constant pass the reference absorption A_ref is the
    constant sources'.

    mode "correction": device state adds the reference emission per
    frequency and cell (FP64, K x ncells, zero at the start).  The
    packages carry L(T_{i-1}) - L_ref (the library blends L_ref by beta_i
    in the same call), T_i is solved from A_i = A_ref + their absorption,
    then A_ref is blended towards A_i by beta_i.

    mode "average": the packages carry the whole emission L(T_{i-1}) as in
    the plain method, A_i = A_const + their absorption, A_ref is blended
    towards A_i by beta_i and T_i is solved from A_ref."""

    def __init__(self, ctx: soc.Context, P, seed: int = 1, nT: int = 4096, packages=None, cap: float = 0.0,
                 mode: str = "correction", multi: bool = True):
        super().__init__(ctx, P, seed, nT, packages, cap, ali=False, multi=multi)
        if mode not in ("correction", "average"):
            raise ValueError("mode must be 'correction' or 'average'")
        self.mode = mode
        nc = P.grid.ncells
        self.L_ref = (torch.zeros((P.K, nc), dtype=torch.float64, device="cuda") if mode == "correction"
                      else None)
        self.A_ref = torch.zeros(nc, dtype=torch.float64, device="cuda")
        self.n_sum = 0

    def constant_pass(self) -> dict:
        s = super().constant_pass()
        self.A_ref.copy_(self.A_const)
        if self.L_ref is not None:
            self.L_ref.zero_()
        self.n_sum = 0
        return s

    def seed_prediction(self, T0: torch.Tensor, A0: torch.Tensor, weight: int) -> dict:
        """After the constant pass, start from a predicted solution: the
        temperatures T0 and, as the reference absorption, A0, counted as if
        `weight` packages per frequency had estimated it (mode "average"
        only: later estimates are averaged in and the seed's share falls as
        weight / (weight + packages so far))."""
        if self.mode != "average":
            raise ValueError("a predicted reference absorption seeds the 'average' reading")
        self.A_ref.copy_(A0.reshape(-1))
        self.n_sum = int(weight)
        return self.set_temperature(T0)

    def dust_iteration(self, it: int) -> dict:
        P = self.P
        n = self.n_packages(it)
        self.n_sum += n
        beta = n / self.n_sum
        if self.mode == "correction":
            self.A.copy_(self.A_ref)
            self._simulate(self.A, [dict(T=self.T, n_dust=n, dust_mode=2, L_ref=self.L_ref[k], ref_beta=beta,
                                         dust_cap=self.cap) for k in range(P.K)], iteration=it)
            s = soc.update_temperature(self.ctx, self.grid, self.table, self.A, self.T_new, self.T, stats=True)
            soc.reference_blend(self.ctx, self.A, self.A_ref, beta)
        else:
            self.A.copy_(self.A_const)
            self._simulate(self.A, [dict(T=self.T, n_dust=n, dust_mode=1, dust_cap=self.cap)] * P.K, iteration=it)
            soc.reference_blend(self.ctx, self.A, self.A_ref, beta)
            s = soc.update_temperature(self.ctx, self.grid, self.table, self.A_ref, self.T_new, self.T,
                                       stats=True)
        self.T.copy_(self.T_new)
        s["packages"] = n
        return s


def absorbed_spectra(ctx: soc.Context, grid: soc.Grid, P, T=None, n_dust: int = 0, seed: int = 1,
                     iteration: int = 1, out=None) -> torch.Tensor:
    """Absorbed energy of every cell in each frequency band of problem P,
    float64 [K][ncells] (erg/s): one Monte Carlo pass per frequency into its
    own row, of the constant sources and, given temperatures T, of n_dust
    luminosity-weighted dust-emission packages.  Stochastically heated grains
    need the absorptions per frequency rather than integrated (Sect. 2.1.1);
    the paper keeps them in memory-mapped files on the host, here they stay
    in device memory.  The cross sections are P's (for grains: the model's
    total per H)."""
    K, nc = P.K, P.grid.ncells
    A = out if out is not None else torch.empty((K, nc), dtype=torch.float64, device="cuda")
    have_ps = len(P.ps_pos) > 0
    for k in range(K):
        A[k].zero_()
        f = (float(P.nu[k]), float(P.w[k]), float(P.sigma_abs[k]), float(P.sigma_sca[k]), float(P.g[k]))
        soc.simulate_frequency(ctx, grid, f, A[k], I_bg=float(P.I_bg[k]), ps_pos=P.ps_pos if have_ps else None,
                               ps_Lnu=P.ps_Lnu[:, k] if have_ps else None, n_bg=P.n_bg,
                               n_ps_pk=P.n_ps_pk if have_ps else 0, T=T, n_dust=n_dust if T is not None else 0,
                               dust_mode=1, seed=seed, iteration=iteration, freq_index=k)
    return A
