"""Checks that pin the oracle to facts fixed outside it.

Each function returns ``(ok, detail)`` so that the same check can be asserted by a
test and, with a planted mistake in the oracle, be shown to fail.  None of them
re-types the oracle's formulas: they use closed forms, brute force on tiny
lattices, identities between different definitions (Eq. 1 energy vs the hop
energy change), invariants of the dynamics, a library Philox, and the stationary
law that detailed balance implies.
"""
from __future__ import annotations

import math

import numpy as np

import oracle


# ---------------------------------------------------------------- geometry
def disk_vectors(rc: float):
    """All integer d != 0 with |d|^2 <= rc^2, by enumeration over a square."""
    k = int(math.floor(rc)) + 1
    out = set()
    for dx in range(-k, k + 1):
        for dy in range(-k, k + 1):
            if (dx, dy) != (0, 0) and dx * dx + dy * dy <= rc * rc:
                out.add((dx, dy))
    return out


def min_image_r(L: int, dx, dy):
    a = np.mod(dx, L)
    b = np.mod(dy, L)
    a = np.minimum(a, L - a)
    b = np.minimum(b, L - b)
    return np.sqrt(a * a + b * b)


def check_displacement_set(o: oracle.Oracle, rc: float):
    t = o.tower()
    got = set(zip(t["dx"].tolist(), t["dy"].tolist()))
    want = disk_vectors(rc)
    ok = got == want and len(t["dx"]) == len(want)
    return ok, f"{len(got)} vectors vs {len(want)} lattice points in the disk"


def check_proposal_symmetry(o: oracle.Oracle):
    t = o.tower()
    q = {(int(dx), int(dy)): o.vec_prob(v) for v, (dx, dy) in enumerate(zip(t["dx"], t["dy"]))}
    bad = 0
    for (dx, dy), p in q.items():
        for img in ((-dx, -dy), (dy, dx), (-dx, dy), (dx, -dy)):
            if q.get(img) != p:
                bad += 1
    thr = t["thr"].astype(np.float64)
    mono = bool(np.all(np.diff(thr) >= 0)) and int(t["thr"][-1]) == 2**32
    tot = sum(q.values())
    return bad == 0 and mono and abs(tot - 1.0) < 1e-15, f"asym={bad} monotone={mono} sum={tot!r}"


def check_gamma_pairs(o: oracle.Oracle, L: int, xi: float, rc: float):
    """Gamma = sum_i sum_{j != i} exp(-2 r_ij / xi) over pairs within the cutoff (brute force)."""
    N = L * L
    x = np.arange(N) % L
    y = np.arange(N) // L
    total = 0.0
    for i in range(N):
        a = np.mod(x - x[i], L)
        b = np.mod(y - y[i], L)
        a = np.minimum(a, L - a)
        b = np.minimum(b, L - b)
        r2 = a * a + b * b
        # a pair is a hop candidate when some displacement |d| <= rc maps i to j
        m = (r2 > 0) & (r2 <= rc * rc)
        total += float(np.exp(-2.0 * np.sqrt(r2[m].astype(float)) / xi).sum())
    G = o.tower()["Gamma"]
    return abs(G - total) <= 1e-12 * total, f"Gamma={G!r} brute force={total!r}"


def check_displacement_draws(o: oracle.Oracle, xi: float, n: int = 200_000, s0: int = 1):
    """Draw frequencies of each displacement vs exp(-2|d|/xi) / sum (chi-square)."""
    t = o.tower()
    dx, dy = t["dx"], t["dy"]
    w = np.exp(-2.0 * np.sqrt(dx.astype(float) ** 2 + dy.astype(float) ** 2) / xi)
    p = w / w.sum()
    counts = np.zeros(len(dx))
    for s in range(s0, s0 + n):
        _, v, _ = o.draw(s)
        counts[v] += 1
    # pool the far tail into one bin so every expected count is >= 20
    order = np.argsort(-p)
    e = n * p[order]
    c = counts[order]
    keep = e >= 20
    ee = np.append(e[keep], e[~keep].sum())
    cc = np.append(c[keep], c[~keep].sum())
    if ee[-1] == 0:
        ee, cc = ee[:-1], cc[:-1]
    chi2 = float(((cc - ee) ** 2 / ee).sum())
    dof = len(ee) - 1
    z = (chi2 - dof) / math.sqrt(2 * dof)
    return z < 5.0, f"chi2={chi2:.1f} dof={dof} z={z:.2f}"


def check_site_and_u(o: oracle.Oracle, n: int = 100_000):
    N = o.N
    counts = np.zeros(N)
    us = np.zeros(n)
    for k, s in enumerate(range(1, n + 1)):
        i, _, u = o.draw(s)
        counts[i] += 1
        us[k] = u
    e = n / N
    chi2 = float(((counts - e) ** 2 / e).sum())
    z = (chi2 - (N - 1)) / math.sqrt(2 * (N - 1))
    ok = z < 5 and us.min() > 0 and us.max() < 1 and abs(us.mean() - 0.5) < 5 / math.sqrt(12 * n)
    return ok, f"site z={z:.2f} u in ({us.min():.3g},{us.max():.3g}) mean={us.mean():.5f}"


# ---------------------------------------------------------------- energies
def eq1_energy(L: int, n, phi, E: float = 0.0, xpos=None):
    """Eq. 1 on the torus (minimum image), with the field term over the given x positions."""
    N = L * L
    nu = float(np.sum(n)) / N
    x = np.arange(N) % L
    y = np.arange(N) // L
    r = min_image_r(L, x[:, None] - x[None, :], y[:, None] - y[None, :])
    V = np.zeros_like(r)
    V[r > 0] = 1.0 / r[r > 0]
    q = n.astype(float) - nu
    H = float(phi @ n) + 0.5 * float(q @ V @ q)
    if xpos is not None:
        H -= E * float(np.sum(n * xpos))
    return H


def check_eps_closed_form_3x3():
    """3x3 torus: every other site is a nearest (r=1, 4 of them) or diagonal (r=sqrt 2, 4)
    neighbour, so with one electron at i0: eps_l = phi_l + [l != i0] v(l - i0) - nu (4 + 2 sqrt 2),
    and with one hole at h0: eps_l = phi_l - [l != h0] v(l - h0) + (1 - nu)(4 + 2 sqrt 2)."""
    worst = 0.0
    S = 4.0 + 4.0 / math.sqrt(2.0)
    for n_e, filled in ((1, False), (8, True)):
        o = oracle.Oracle(L=3, n_e=n_e, W=1.0, rc=math.sqrt(2.0), T=1.0, E=0.0, seed=11)
        phi = o.phi()
        nu = n_e / 9.0
        for k in range(9):
            n = np.zeros(9, np.uint8) if not filled else np.ones(9, np.uint8)
            n[k] = 0 if filled else 1
            o.set_occ(n)
            eps = o.eps()
            for l in range(9):
                ddx = abs((l % 3) - (k % 3))
                ddy = abs((l // 3) - (k // 3))
                v = 0.0 if l == k else (1.0 if ddx == 0 or ddy == 0 else 1.0 / math.sqrt(2.0))
                want = phi[l] + v - nu * S if not filled else phi[l] - v + (1.0 - nu) * S
                worst = max(worst, abs(eps[l] - want))
    return worst < 1e-14, f"max |eps - closed form| = {worst:.3g}"


def _partner(L, i, dx, dy):
    return ((i // L + dy) % L) * L + (i % L + dx) % L


def check_dh_identity(o: oracle.Oracle, n_moves: int = 200, seed: int = 0):
    """dH of a hop equals H(after) - H(before) from Eq. 1, field term -E dx included."""
    L, N, E = o.L, o.N, o.params["E"]
    t = o.tower()
    phi = o.phi()
    rng = np.random.default_rng(seed)
    worst = 0.0
    n0 = o.occ()
    H0 = eq1_energy(L, n0, phi)
    occ_sites = np.flatnonzero(n0 == 1)
    tried = 0
    while tried < n_moves:
        i = int(rng.choice(occ_sites))
        v = int(rng.integers(len(t["dx"])))
        j = _partner(L, i, int(t["dx"][v]), int(t["dy"][v]))
        if n0[j] == 1:
            continue
        _, dH = o.move(i, v)
        n1 = n0.copy()
        n1[i], n1[j] = 0, 1
        want = (eq1_energy(L, n1, phi) - H0) - E * float(t["dx"][v])
        worst = max(worst, abs(dH - want))
        tried += 1
    return worst < 1e-11, f"max |dH - (H(b)-H(a))| = {worst:.3g} over {tried} hops"


def check_incremental_eps(o: oracle.Oracle, hops: int):
    o.run(hops, max_labels=20_000_000)
    d = float(np.abs(o.eps() - o.recompute_eps()).max())
    return d < 1e-12, f"max |eps_incremental - eps_recomputed| = {d:.3g} after {hops} hops"


def check_invariants(o: oracle.Oracle, hops: int):
    """Charge conservation, dipole P = sum of hop dx (mod L against sum n x), clock t*Gamma = s_last."""
    L = o.L
    n0 = o.occ()
    x = np.arange(o.N) % L
    sc0 = o.scalars()
    lab, li, lj = o.run(hops, max_labels=20_000_000)
    sc = o.scalars()
    n1 = o.occ()
    charge = int(n1.sum()) == int(n0.sum()) == o.params["n_e"]
    dP = sc["P"] - sc0["P"]
    dip = (int((n1 * x).sum() - (n0 * x).sum()) - dP) % L == 0
    # replay the logged hops on the initial occupation
    n = n0.copy()
    replay = True
    sum_dx = 0
    for a, b in zip(li.tolist(), lj.tolist()):
        replay &= n[a] == 1 and n[b] == 0
        n[a], n[b] = 0, 1
        d = (b % L - a % L) % L  # hop length along x, unique because |dx| <= rc < L/2
        sum_dx += d - L if d > L // 2 else d
    replay &= bool(np.array_equal(n, n1))
    dip = dip and sum_dx == dP
    clock = True
    if o.params["clock_mode"] == 0:
        clock = sc["t"] == sc["s_last"] / sc["Gamma"]
    ok = charge and dip and replay and clock and len(lab) == hops
    return ok, f"charge={charge} dipole={dip} replay={replay} clock={clock}"


# ---------------------------------------------------------------- stationary law
def _states_3x3(k=4):
    from itertools import combinations

    return [tuple(c) for c in combinations(range(9), k)]


def check_boltzmann_exact_3x3(T: float = 0.5, seed: int = 5):
    """Per-proposal transition matrix of the chain on a 3x3 torus with 4 electrons at E=0:
    pi(a) ~ exp(-H(a)/T) from Eq. 1 must satisfy pi P = pi (detailed balance of Eq. 2)."""
    o = oracle.Oracle(L=3, n_e=4, W=1.0, rc=math.sqrt(2.0), T=T, E=0.0, seed=seed)
    phi = o.phi()
    t = o.tower()
    states = _states_3x3()
    index = {s: k for k, s in enumerate(states)}
    S = len(states)
    P = np.zeros((S, S))
    H = np.zeros(S)
    qv = np.array([o.vec_prob(v) for v in range(len(t["dx"]))])
    for a, s in enumerate(states):
        n = np.zeros(9, np.uint8)
        n[list(s)] = 1
        o.set_occ(n)
        H[a] = eq1_energy(3, n, phi)
        for i in range(9):
            for v in range(len(qv)):
                p, _ = o.move(i, v)
                if p == 0.0:
                    continue
                j = _partner(3, i, int(t["dx"][v]), int(t["dy"][v]))
                m = n.copy()
                m[i], m[j] = 0, 1
                b = index[tuple(np.flatnonzero(m).tolist())]
                P[a, b] += (1.0 / 9.0) * qv[v] * p
        P[a, a] = 1.0 - (P[a].sum() - P[a, a])
    pi = np.exp(-(H - H.min()) / T)
    pi /= pi.sum()
    res = float(np.abs(pi @ P - pi).max())
    return res < 1e-13, f"max |pi P - pi| = {res:.3g}"


def check_boltzmann_sampled_3x3(T: float = 0.5, hops: int = 100_000, seed: int = 6):
    """Fraction of serial proposals spent in each of the 126 states of a long oracle run
    vs exp(-H/T)/Z (total variation distance)."""
    o = oracle.Oracle(L=3, n_e=4, W=1.0, rc=math.sqrt(2.0), T=T, E=0.0, seed=seed)
    phi = o.phi()
    states = _states_3x3()
    index = {s: k for k, s in enumerate(states)}
    H = np.array([eq1_energy(3, np.isin(np.arange(9), s).astype(np.uint8), phi) for s in states])
    pi = np.exp(-(H - H.min()) / T)
    pi /= pi.sum()
    n = o.occ()
    lab, li, lj = o.run(hops)
    w = np.zeros(len(states))
    code = 0
    for k in range(9):
        code |= int(n[k]) << k
    codes = {sum(1 << k for k in s): idx for s, idx in index.items()}
    prev = 0
    cur = codes[code]
    for s, a, b in zip(lab.tolist(), li.tolist(), lj.tolist()):
        w[cur] += s - prev  # proposals spent in the current state, the executed one included
        prev = s
        code = (code & ~(1 << a)) | (1 << b)
        cur = codes[code]
    w /= w.sum()
    tv = 0.5 * float(np.abs(w - pi).sum())
    return tv < 0.02, f"total variation distance = {tv:.4f} over {hops} hops"


# ---------------------------------------------------------------- parallel-rejection closed form
def check_geometric_m(L=16, T=0.1, E=0.01, M=64, relax=1000, hops=1500, seed=7):
    """Given the configuration, the number m of serial proposals to the next hop is geometric
    with the exact acceptance A, so E[m] = 1/A and, for M threads, E[p] = 1/[1-(1-A)^M]
    with p = ceil(m/M) (section "Parallel rejection algorithm").  Standardised sums ~ N(0,1)."""
    o = oracle.Oracle(L=L, n_e=L * L // 2, W=1.0, rc=6.0, T=T, E=E, seed=seed)
    o.run(relax)
    zm = 0.0
    zp = 0.0
    for _ in range(hops):
        A = o.acceptance()
        s0 = o.scalars()["s_last"]
        lab, _, _ = o.run(1)
        m = int(lab[0] - s0)
        zm += (m - 1.0 / A) / math.sqrt((1.0 - A) / (A * A))
        p = -(-m // M)
        g = (1.0 - A) ** M
        zp += (p - 1.0 / (1.0 - g)) / math.sqrt(g / (1.0 - g) ** 2)
    zm /= math.sqrt(hops)
    zp /= math.sqrt(hops)
    return abs(zm) < 4.0 and abs(zp) < 4.0, f"z(m)={zm:.2f} z(p)={zp:.2f}"


# ---------------------------------------------------------------- pair hops
def _pair_sites(L, t, i, v1, ve, v2):
    j = _partner(L, i, int(t["dx"][v1]), int(t["dy"][v1]))
    k = _partner(L, i, int(t["dx"][ve]), int(t["dy"][ve]))
    l = _partner(L, k, int(t["dx"][v2]), int(t["dy"][v2]))
    return j, k, l


def check_pair_dh_identity(o: oracle.Oracle, n_moves: int = 150, seed: int = 0):
    """dH of a pair hop i -> j, k -> l equals H(after) - H(before) from Eq. 1, the field term
    -E (dx1 + dx2) included, for random valid pair moves (brute-force Eq. 1, no use of the
    oracle's energies)."""
    L, E = o.L, o.params["E"]
    t = o.tower()
    phi = o.phi()
    rng = np.random.default_rng(seed)
    n0 = o.occ()
    H0 = eq1_energy(L, n0, phi)
    nv = len(t["dx"])
    worst, tried, attempts = 0.0, 0, 0
    while tried < n_moves and attempts < 200 * n_moves:
        attempts += 1
        i = int(rng.choice(np.flatnonzero(n0 == 1)))
        v1, ve, v2 = (int(x) for x in rng.integers(nv, size=3))
        j, k, l = _pair_sites(L, t, i, v1, ve, v2)
        p, dH = o.move_pair(i, v1, ve, v2)
        valid = n0[k] == 1 and n0[j] == 0 and n0[l] == 0 and j != l
        if not valid:
            if p != 0.0:
                return False, f"invalid pair move (i={i}, j={j}, k={k}, l={l}) has acceptance {p}"
            continue
        if not math.isfinite(dH):  # final sites beyond the cutoff
            continue
        n1 = n0.copy()
        n1[i], n1[j], n1[k], n1[l] = 0, 1, 0, 1
        want = (eq1_energy(L, n1, phi) - H0) - E * float(t["dx"][v1] + t["dx"][v2])
        worst = max(worst, abs(dH - want))
        tried += 1
    return tried == n_moves and worst < 1e-11, f"max |dH - (H(b)-H(a))| = {worst:.3g} over {tried} pair moves"


def check_pair_boltzmann_exact(L: int = 3, n_e: int = 4, rc: float = math.sqrt(2.0), T: float = 0.5,
                               pair: float = 0.4, seed: int = 5):
    """Per-proposal transition matrix on a tiny torus at E = 0 when a label is a pair proposal
    with probability `pair` (site 1/N; partner offset uniform over the hop vectors; hop vectors
    from the tunnelling tower): pi ~ exp(-H/T) from Eq. 1 must satisfy pi P = pi, which holds
    only if pair moves are proposed as often as their reverse and accepted by their true
    energy change.  On the 3x3 torus every two sites are within sqrt 2 of each other; the 4x4
    torus with rc = 1 also exercises the final-separation filter."""
    from itertools import combinations

    N = L * L
    o = oracle.Oracle(L=L, n_e=n_e, W=1.0, rc=rc, T=T, E=0.0, seed=seed, pair=pair)
    phi = o.phi()
    t = o.tower()
    nv = len(t["dx"])
    states = [tuple(c) for c in combinations(range(N), n_e)]
    index = {s: k for k, s in enumerate(states)}
    S = len(states)
    P = np.zeros((S, S))
    H = np.zeros(S)
    qv = np.array([o.vec_prob(v) for v in range(nv)])
    for a, s in enumerate(states):
        n = np.zeros(N, np.uint8)
        n[list(s)] = 1
        o.set_occ(n)
        H[a] = eq1_energy(L, n, phi)
        for i in range(N):
            for v in range(nv):
                p, _ = o.move(i, v)
                if p > 0.0:
                    j = _partner(L, i, int(t["dx"][v]), int(t["dy"][v]))
                    m = n.copy()
                    m[i], m[j] = 0, 1
                    P[a, index[tuple(np.flatnonzero(m).tolist())]] += (1.0 - pair) / N * qv[v] * p
            if n[i] == 0:
                continue
            for v1 in range(nv):
                for ve in range(nv):
                    for v2 in range(nv):
                        p, _ = o.move_pair(i, v1, ve, v2)
                        if p == 0.0:
                            continue
                        j, k, l = _pair_sites(L, t, i, v1, ve, v2)
                        m = n.copy()
                        m[i], m[j], m[k], m[l] = 0, 1, 0, 1
                        b = index[tuple(np.flatnonzero(m).tolist())]
                        P[a, b] += pair / N / nv * qv[v1] * qv[v2] * p
        P[a, a] = 1.0 - (P[a].sum() - P[a, a])
    pi = np.exp(-(H - H.min()) / T)
    pi /= pi.sum()
    res = float(np.abs(pi @ P - pi).max())
    moves = int((P > 0).sum())
    return res < 1e-13, f"max |pi P - pi| = {res:.3g} ({moves} nonzero entries)"


def check_pair_invariants(o: oracle.Oracle, hops: int):
    """With pair hops: charge conservation, the log replays (each entry moves an electron to an
    empty site; a pair hop's two entries share a label), the dipole is the sum of the logged
    dx, the clock is s_last / Gamma_lab with Gamma_lab = Gamma / (1 - pair), the incremental
    energies equal the O(N^2) recompute, and pair hops occur."""
    L = o.L
    n0 = o.occ()
    sc0 = o.scalars()
    lab, li, lj = o.run(hops, max_labels=50_000_000)
    sc = o.scalars()
    n = n0.copy()
    replay, sum_dx = True, 0
    for a, b in zip(li.tolist(), lj.tolist()):
        replay &= n[a] == 1 and n[b] == 0
        n[a], n[b] = 0, 1
        d = (b % L - a % L) % L
        sum_dx += d - L if d > L // 2 else d
    replay &= bool(np.array_equal(n, o.occ()))
    pairs = int(np.sum(np.diff(lab.astype(np.int64)) == 0))
    hops_ok = len(lab) - pairs == hops == o.last_run_hops
    gl = sc["Gamma"] / (1.0 - o.params["pair"])
    clock = abs(sc["t"] - sc["s_last"] / gl) <= 1e-15 * sc["t"] and sc["Gamma_lab"] == gl
    dip = sum_dx == sc["P"] - sc0["P"]
    charge = int(o.occ().sum()) == o.params["n_e"]
    d = float(np.abs(o.eps() - o.recompute_eps()).max())
    ok = replay and hops_ok and clock and dip and charge and d < 1e-12 and pairs > 0
    return ok, (f"replay={replay} hops={hops_ok} clock={clock} dipole={dip} charge={charge} "
                f"eps drift={d:.3g} pair hops={pairs}")


def check_pair_draws(o: oracle.Oracle, xi: float, n: int = 60_000):
    """Pair labels: their fraction is `pair` (binomial z), the partner offset is uniform over
    the hop vectors and the second hop vector follows exp(-2|d|/xi) (chi-square each)."""
    t = o.tower()
    nv = len(t["dx"])
    w = np.exp(-2.0 * np.sqrt(t["dx"].astype(float) ** 2 + t["dy"].astype(float) ** 2) / xi)
    q = w / w.sum()
    ce = np.zeros(nv)
    c2 = np.zeros(nv)
    npair = 0
    for s in range(1, n + 1):
        ip, _, _, ve, v2, _ = o.draw_label(s)
        if ip:
            npair += 1
            ce[ve] += 1
            c2[v2] += 1
    p = o.params["pair"]
    zf = (npair - n * p) / math.sqrt(n * p * (1 - p))

    def chi2_z(c, prob):
        e = npair * prob
        keep = e >= 20
        ee = np.append(e[keep], e[~keep].sum())
        cc = np.append(c[keep], c[~keep].sum())
        if ee[-1] == 0:
            ee, cc = ee[:-1], cc[:-1]
        x2 = float(((cc - ee) ** 2 / ee).sum())
        dof = len(ee) - 1
        return (x2 - dof) / math.sqrt(2 * dof)

    ze = chi2_z(ce, np.full(nv, 1.0 / nv))
    z2 = chi2_z(c2, q)
    return abs(zf) < 5 and ze < 5 and z2 < 5, f"fraction z={zf:.2f} offset z={ze:.2f} hop z={z2:.2f}"
