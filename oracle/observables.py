"""Observables of the Coulomb-glass dynamics, written out from their definitions.

TEST INFRASTRUCTURE ONLY (part of the oracle): imported by the test suite, never by the
product library, and sharing no code with it.

* Density of states (section "Results"): the normalized histogram
  g(eps, T) = sum_k delta_{d eps}(eps - eps_k) of the local energies of Eq. 2, counted here
  per bin of width d eps = (e_hi - e_lo) / nbins; bin of eps: floor((eps - e_lo) * scale)
  with scale = nbins / (e_hi - e_lo) in FP64.
* Conductivity (Eq. 3 and section "Results"): sigma(t) = P / (N E t) with P the dipole
  moment change, and the stationary sigma_0 = lim (dP/dt) / (N E), estimated from the slope
  of P against t over the late part of a run.
* Efros-Shklovskii law (section "Results"): sigma_0 = b T^-lambda exp(-(T_0 / T)^(1/2)),
  fitted for a fixed lambda: ln sigma_0 + lambda ln T = ln b - T_0^(1/2) T^(-1/2) is a
  straight line in T^(-1/2).
* Scaling (Eq. 4): sigma(t, T) = sigma_0(T) f(t sigma_0(T) T^2).
"""
from __future__ import annotations

import math

import numpy as np


def dos_counts(eps, occ, e_lo: float, e_hi: float, nbins: int):
    """Counts of occupied and empty sites per bin, and of sites below / at or above the range.
    A plain loop over the sites (the definition, site by site)."""
    scale = nbins / (e_hi - e_lo)
    occupied = [0] * nbins
    empty = [0] * nbins
    below = above = 0
    for e, n in zip(np.asarray(eps, dtype=np.float64).tolist(), np.asarray(occ).tolist()):
        x = math.floor((e - e_lo) * scale)
        if x < 0:
            below += 1
        elif x >= nbins:
            above += 1
        elif n:
            occupied[x] += 1
        else:
            empty[x] += 1
    return np.array(occupied, np.uint64), np.array(empty, np.uint64), below, above


def dos_normalized(counts, n_sites: int, e_lo: float, e_hi: float) -> np.ndarray:
    """g per unit energy: counts / (number of sites x bin width)."""
    width = (e_hi - e_lo) / len(counts)
    return np.asarray(counts, dtype=np.float64) / (n_sites * width)


def sigma_of_t(P, N: int, E: float, t):
    """sigma(t) = P(t) / (N E t)."""
    P = np.asarray(P, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return P / (N * E * t)


def sigma0_from_slope(t, P, N: int, E: float) -> float:
    """Least-squares slope of P against t, divided by N E: the normal equations written out."""
    t = np.asarray(t, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    n = len(t)
    st, sp = sum(t.tolist()), sum(P.tolist())
    stt = sum((t * t).tolist())
    stp = sum((t * P).tolist())
    slope = (n * stp - st * sp) / (n * stt - st * st)
    return slope / (N * E)


def es_fit(T, sigma0, lam: float):
    """(b, T_0) of the Efros-Shklovskii law for a fixed lambda, by least squares on
    y = ln sigma_0 + lambda ln T against x = T^(-1/2): y = ln b - T_0^(1/2) x."""
    x = [1.0 / math.sqrt(v) for v in T]
    y = [math.log(s) + lam * math.log(v) for s, v in zip(sigma0, T)]
    n = len(x)
    sx, sy = sum(x), sum(y)
    sxx = sum(a * a for a in x)
    sxy = sum(a * c for a, c in zip(x, y))
    slope = (n * sxy - sx * sy) / (n * sxx - sx * sx)
    icpt = (sy - slope * sx) / n
    return math.exp(icpt), slope * slope


def es_law(T, b: float, T0: float, lam: float):
    T = np.asarray(T, dtype=np.float64)
    return b * T ** (-lam) * np.exp(-np.sqrt(T0 / T))


def collapse(t, P, N: int, E: float, T: float, sigma0: float):
    """Eq. 4's variables: (t sigma_0 T^2, sigma(t) / sigma_0)."""
    t = np.asarray(t, dtype=np.float64)
    return t * sigma0 * T * T, sigma_of_t(P, N, E, t) / sigma0
