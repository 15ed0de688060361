"""FP64 oracle of the stochastically heated grain solver.

TEST INFRASTRUCTURE ONLY: imported by tests and the CPU-baseline leg of the
benchmark; never by the GPU library or its binding.  It shares no code with
the HIP path.

What it computes follows Juvela, "SOC program for dust continuum
radiative transfer" (A&A 2019, arXiv:1812.06632), Sect. 2.1.1 and
Appendix A: the temperature distribution of each grain size in each cell
from the absorbed photons, in the "thermal continuous" cooling
approximation, where a grain cools only into the next lower enthalpy bin.

  * Upward rates R[j, i] (bin i -> bin j > i): the photons of frequency
    band k absorbed per second by one grain, r_k, each raising the enthalpy
    from U_i by h nu_k; the target U_i + h nu_k is split between the two
    bins around it in proportion to the distance (so the expected enthalpy
    gain is exactly h nu_k), and a target above the top bin goes to the top
    bin.
  * Cooling R[i-1, i] = L(T_i) / (U_i - U_{i-1}), L(T) = 4 pi sum_k sigma_k
    B_nu_k(T) w_k the power a grain at T emits.
  * Diagonal: minus the sum of the other elements of the column.
  * The stationary distribution R P = 0, sum P = 1, by forward
    substitution: no transition crosses the cut between bins j-1 and j
    downwards except j -> j-1, so P_j R[j-1, j] = sum_{i<j} P_i sum_{m>=j}
    R[m, i].
  * Emission of a cell: sum over sizes of the grain count times
    4 pi sigma_k sum_i P_i B_nu_k(T_i), erg s^-1 Hz^-1.

Absorbed energies come per cell and frequency band (erg/s, the Monte Carlo
tallies of one frequency each); the share of size s in band k is its
fraction abundance_s sigma_sk / sum_s abundance_s sigma_sk of the
absorption, divided among abundance_s n_H V grains.
"""
from __future__ import annotations

import math

import numpy as np

H = 6.62607015e-27
K_B = 1.380649e-16
C_LIGHT = 2.99792458e10


def planck(nu, T):
    """B_nu(T) (erg s-1 cm-2 Hz-1 sr-1), outer product T x nu."""
    nu = np.asarray(nu, dtype=np.float64)
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    x = H * nu[None, :] / (K_B * T[:, None])
    return 2.0 * H * nu[None, :] ** 3 / C_LIGHT ** 2 / np.expm1(np.minimum(x, 700.0))


def grain_power(G, s, T):
    """Power emitted by one grain of size s at temperatures T (erg/s)."""
    return 4.0 * math.pi * planck(G.nu, T) @ (G.sigma[s] * G.w)


def rate_matrix(G, s, r):
    """R[j, i] for size s and photon rates r[k] (per grain, per second)."""
    U = G.U[s]
    N = U.size
    R = np.zeros((N, N))
    E = H * G.nu
    for i in range(N):
        for k in range(len(r)):
            if r[k] == 0.0:
                continue
            t = U[i] + E[k]
            if t >= U[-1]:
                R[N - 1, i] += r[k]
                continue
            m = int(np.searchsorted(U, t, side="right")) - 1     # U[m] <= t < U[m+1]
            f = (t - U[m]) / (U[m + 1] - U[m])
            R[m + 1, i] += r[k] * f
            if m != i:
                R[m, i] += r[k] * (1.0 - f)
    L = grain_power(G, s, G.T[s])
    for i in range(1, N):
        R[i - 1, i] += L[i] / (U[i] - U[i - 1])
    R[np.diag_indices(N)] = 0.0
    R[np.diag_indices(N)] = -R.sum(axis=0)
    return R


def solve_forward(R):
    """Stationary distribution of a thermal-continuous rate matrix."""
    N = R.shape[0]
    up = np.cumsum(R[::-1, :], axis=0)[::-1, :]   # up[j, i] = sum_{m>=j} R[m, i]
    P = np.zeros(N)
    P[0] = 1.0
    for j in range(1, N):
        P[j] = np.dot(P[:j], up[j, :j]) / R[j - 1, j]
        if P[j] > 1e200:
            P[: j + 1] *= 1e-200
    return P / P.sum()


def photon_rates(G, A_k, n_grains, s):
    """Photons per second absorbed by one grain of size s in each band, from
    the cell's absorbed energies A_k (erg/s per band)."""
    tot = (G.abundance[:, None] * G.sigma).sum(axis=0)
    share = np.where(tot > 0, G.abundance[s] * G.sigma[s] / np.where(tot > 0, tot, 1.0), 0.0)
    if n_grains <= 0:
        return np.zeros_like(A_k)
    return A_k * share / (n_grains * H * G.nu)


def solve_cell(G, A_k, n_H_V):
    """Emission (erg s-1 Hz-1, per cell, [K]) and the distributions
    ([S, nE]) of one cell with n_H V hydrogen atoms."""
    S = len(G.a_cm)
    P_all = np.zeros((S, G.U.shape[1]))
    em = np.zeros(len(G.nu))
    for s in range(S):
        Ns = G.abundance[s] * n_H_V
        r = photon_rates(G, np.asarray(A_k, dtype=np.float64), Ns, s)
        P = solve_forward(rate_matrix(G, s, r))
        P_all[s] = P
        em += Ns * 4.0 * math.pi * G.sigma[s] * (P @ planck(G.nu, G.T[s]))
    return em, P_all


def shg_solve(G, density, volume, A):
    """Emission [K, ncells] of every cell (0 where density is 0) and the
    distributions [ncells, S, nE], from absorbed energies A [K, ncells]."""
    A = np.asarray(A, dtype=np.float64)
    K, nc = A.shape
    E = np.zeros((K, nc))
    P = np.zeros((nc, len(G.a_cm), G.U.shape[1]))
    for c in range(nc):
        if density[c] > 0:
            E[:, c], P[c] = solve_cell(G, A[:, c], float(density[c]) * float(volume[c]))
    return E, P


def heating_power(G, s, r, P):
    """Mean enthalpy gain per second of grains of size s distributed as P
    (photons above the top bin gain only up to it)."""
    U = G.U[s]
    E = H * G.nu
    gain = np.minimum(U[:, None] + E[None, :], U[-1]) - U[:, None]   # [nE, K]
    return float(P @ (gain @ r))
