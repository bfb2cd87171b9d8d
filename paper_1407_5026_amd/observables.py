"""Physics observables on top of the hop path: density of states, P(t), sigma_0(T), the
Efros-Shklovskii fit and the scaling collapse of Eq. 4 (section "Results").

The density of states is counted on the GPU (`cg_dos`); P(t) comes from the library's clock
and dipole after `cg_run_time`; the fits are host arithmetic on those series.

    python -m paper_1407_5026_amd.observables [--L 64] [--samples 256] [--temps ...]

runs the temperature sweep (E = T / 10, as in the paper's runs) and prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def dos(batch, first: int, count: int, e_lo: float, e_hi: float, nbins: int):
    """GPU counts and the normalized g(eps) of samples first .. first + count - 1:
    (bin centres, g_total, g_occupied, g_empty, below, above)."""
    occ, emp, below, above = batch.dos(first, count, e_lo, e_hi, nbins)
    n_sites = sum(batch.N[b] for b in range(first, first + count))
    width = (e_hi - e_lo) / nbins
    centres = e_lo + width * (np.arange(nbins) + 0.5)
    norm = 1.0 / (n_sites * width)
    return centres, (occ + emp) * norm, occ * norm, emp * norm, below, above


def p_of_t(batch, times, progress=None):
    """Runs every sample of the batch to each time in `times` (increasing) and returns the
    arrays t[k, b] and P[k, b] (clock after the stopping hop and dipole change)."""
    n = batch.n
    ts = np.zeros((len(times), n))
    Ps = np.zeros((len(times), n))
    for k, t_end in enumerate(times):
        batch.run_time(t_end)
        for b in range(n):
            t, P, _ = batch.current(b)
            ts[k, b], Ps[k, b] = t, P
        if progress:
            progress(k, t_end)
    return ts, Ps


def sigma0(t, P, N: int, E: float) -> float:
    """Stationary conductivity: slope of P(t) (least squares over the given points) / (N E)."""
    slope = np.polyfit(np.asarray(t, float), np.asarray(P, float), 1)[0]
    return float(slope / (N * E))


def es_fit(T, s0, lam: float):
    """(b, T_0) of sigma_0 = b T^-lambda exp(-(T_0/T)^(1/2)) for a fixed lambda."""
    T = np.asarray(T, float)
    y = np.log(np.asarray(s0, float)) + lam * np.log(T)
    slope, icpt = np.polyfit(T ** -0.5, y, 1)
    return float(np.exp(icpt)), float(slope * slope)


def collapse_vars(t, P, N: int, E: float, T: float, s0: float):
    """Eq. 4: (t sigma_0 T^2, sigma(t) / sigma_0) with sigma(t) = P / (N E t)."""
    t = np.asarray(t, float)
    return t * s0 * T * T, np.asarray(P, float) / (N * E * t) / s0


def gap_slope(centres, g, T: float, e_max: float = 0.3):
    """c of g(eps) ~ c |eps| in the Coulomb-gap region 3 T < |eps| < e_max (least squares
    through the origin)."""
    m = (np.abs(centres) > 3 * T) & (np.abs(centres) < e_max)
    x = np.abs(centres[m])
    return float(np.dot(x, g[m]) / np.dot(x, x)) if m.any() else float("nan")


def sweep(cg, L: int, temps, n_samples: int, seed: int, t_factor: float, n_points: int,
          precision: int) -> dict:
    """For each T: n_samples samples (nu = 1/2, W = 1, xi = 1, rc = 10, E = T / 10) from the
    random start, P(t) on a log grid up to t_factor x the transient time expected from the
    paper's lambda = 1 fit, sigma_0 from the last half of the grid, the DOS at the end."""
    from workloads import Sample

    out = {"L": L, "samples_per_T": n_samples, "seed": seed, "temps": []}
    s0s = []
    for T in temps:
        E = T / 10.0
        samples = [Sample(L, L * L // 2, 1.0, 1.0, 10.0, T, E, seed, b) for b in range(n_samples)]
        b = cg.Batch(samples, cg.make_opts(precision=precision))
        tau = 1.0 / (T * T * 2.7 / T * math.exp(-math.sqrt(6.2 / T)))
        times = np.geomspace(tau / 100.0, t_factor * tau, n_points)
        t0 = time.perf_counter()
        ts, Ps = p_of_t(b, times, lambda k, te: print(f"[observables] T={T} point {k + 1}/{n_points} t={te:.4g}",
                                                       file=sys.stderr, flush=True))
        wall = time.perf_counter() - t0
        hops = sum(b.stats(k)["hops"] for k in range(n_samples))
        N = L * L
        tm, Pm = ts.mean(axis=1), Ps.mean(axis=1)
        half = n_points // 2
        s0 = sigma0(tm[half:], Pm[half:], N, E)
        s0s.append(s0)
        centres, g, g_occ, g_emp, below, above = dos(b, 0, n_samples, -2.0, 2.0, 80)
        x, y = collapse_vars(tm, Pm, N, E, T, s0)
        out["temps"].append({"T": T, "E": E, "t": tm.tolist(), "P_mean": Pm.tolist(), "sigma0": s0,
                             "collapse_x": x.tolist(), "collapse_y": y.tolist(),
                             "dos_centres": centres.tolist(), "dos_g": g.tolist(), "dos_outside": [below, above],
                             "gap_slope_c": gap_slope(centres, g, T), "hops": hops, "wall_s": wall})
        b.close()
        print(f"[observables] T={T}: sigma0={s0:.4g} hops={hops} wall={wall:.1f}s", file=sys.stderr, flush=True)
    if len(temps) >= 2 and all(s > 0 for s in s0s):
        out["es_fit"] = {f"lambda{lam}": dict(zip(("b", "T0"), es_fit(temps, s0s, lam))) for lam in (1, 2)}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description="observables of the Coulomb-glass dynamics")
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--samples", type=int, default=256)
    ap.add_argument("--temps", type=float, nargs="+", default=[0.07, 0.1, 0.14, 0.2])
    ap.add_argument("--seed", type=int, default=8)
    ap.add_argument("--t-factor", type=float, default=3.0)
    ap.add_argument("--points", type=int, default=16)
    ap.add_argument("--fp64", action="store_true")
    args = ap.parse_args()
    import torch  # noqa: F401  (device memory and streams)

    import paper_1407_5026_amd as cg

    cg.load()
    res = sweep(cg, args.L, args.temps, args.samples, args.seed, args.t_factor, args.points,
                cg.CG_FP64 if args.fp64 else cg.CG_FP32_REFRESH)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
