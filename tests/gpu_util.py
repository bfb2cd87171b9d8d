"""Helpers for the GPU tests: GPU guard, oracle construction, hop-log comparison."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import oracle


def say(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def require_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test needs an MI355X (torch.cuda.is_available() is False)")
    import paper_1407_5026_amd as cg

    cg.load()
    return cg


def oracle_of(s, clock_mode=0):
    d = s if isinstance(s, dict) else s.as_dict()
    if d.get("dim", 2) == 3:
        return oracle.Oracle3D(L=d["L"], n_e=d["n_e"], W=d["W"], xi=d["xi"], rc=d["rc"], T=d["T"], E=d["E"],
                               seed=d["seed"], sample_id=d["sample_id"])
    return oracle.Oracle(L=d["L"], n_e=d["n_e"], W=d["W"], xi=d["xi"], rc=d["rc"], T=d["T"], E=d["E"],
                         seed=d["seed"], sample_id=d["sample_id"], clock_mode=clock_mode,
                         pair=d.get("pair", 0.0))


def lazy_oracle_of(s):
    """Oracle with occupation, disorder and proposal law only (no O(N^2) energies)."""
    d = s if isinstance(s, dict) else s.as_dict()
    return oracle.Oracle(L=d["L"], n_e=d["n_e"], W=d["W"], xi=d["xi"], rc=d["rc"], T=d["T"], E=d["E"],
                         seed=d["seed"], sample_id=d["sample_id"], lazy=True)


def compare_logs(sample, gpu_log, or_log, tol=1e-12):
    """Hop-for-hop equality of (label, from, to).  The only allowed divergence is a flip at the
    first differing label s where the oracle's |u - P_acc| < tol; returns the number of hops that
    agree (all of them when there is no flip)."""
    gl, gi, gj = gpu_log
    ol, oi, oj = or_log
    n = min(len(gl), len(ol))
    same = (gl[:n] == ol[:n]) & (gi[:n] == oi[:n]) & (gj[:n] == oj[:n])
    if same.all():
        assert len(gl) == len(ol), (len(gl), len(ol))
        return n
    k = int(np.argmin(same))
    o = oracle_of(sample)
    if k:
        o.run(k)
    s = int(min(gl[k], ol[k]))
    i, v, u = o.draw(s)
    p, dH = o.move(i, v)
    margin = abs(u - p)
    # the first differing label must be a near-tie of the FP64 decision, or a label the
    # oracle never reached in its log (both sides stop at the requested hop count)
    assert margin < tol, (f"hop {k}: gpu (label {gl[k]}, {gi[k]}->{gj[k]}) vs oracle (label {ol[k]}, "
                          f"{oi[k]}->{oj[k]}); at label {s} u={u!r} P_acc={p!r} dH={dH!r}")
    say(f"allowed flip at hop {k}: label {s} |u - P_acc| = {margin:.3g}")
    return k


def _ulp32(x: float) -> float:
    x = abs(x)
    return 2.0 ** (math.floor(math.log2(x)) - 23) if x > 0 else 2.0 ** -149


def fp32_decision_bound(T: float, u: float, drift: float, eps_max: float) -> float:
    """How far (in energy) the FP64 energy change dH of a label may lie from the acceptance
    boundary -T ln u (accept iff dH < -T ln u, Eq. 2's Metropolis factor) and still be decided
    the other way by the FP32 form: both energies off by the drift since the last refresh plus
    one FP32 ulp of the largest energy each (the value words), the threshold terms' FP32
    rounding, the FP32 acceptance uniform (2k + 1) 2^-24 against the FP64 one (T 2^-23 / u in
    dH), and the FP32 exponential's rounding (a few ulp, T 2^-20 in dH)."""
    return 2.0 * drift + 4.0 * _ulp32(eps_max) + 4.0 * _ulp32(2.0) + T * 2.0 ** -22 / u + T * 2.0 ** -20


def compare_logs_fp32(sample, gpu_log, or_log, drift: float, eps_max: float):
    """FP32 form against the FP64 oracle: (label, from, to) equal up to the first difference,
    which must sit at a label whose FP64 decision the FP32 rounding can flip
    (|dH + T ln u| <= fp32_decision_bound).  Returns the number of identical hops."""
    gl, gi, gj = gpu_log
    ol, oi, oj = or_log
    n = min(len(gl), len(ol))
    same = (gl[:n] == ol[:n]) & (gi[:n] == oi[:n]) & (gj[:n] == oj[:n])
    if same.all():
        assert len(gl) == len(ol), (len(gl), len(ol))
        return n
    k = int(np.argmin(same))
    d = sample if isinstance(sample, dict) else sample.as_dict()
    o = oracle_of(sample)
    if k:
        o.run(k)
    s = int(min(gl[k], ol[k]))
    i, v, u = o.draw(s)
    p, dH = o.move(i, v)
    bound = fp32_decision_bound(d["T"], u, drift, eps_max)
    margin = abs(dH + d["T"] * math.log(u))
    assert p > 0.0 and margin <= bound, (
        f"hop {k}: gpu (label {gl[k]}, {gi[k]}->{gj[k]}) vs oracle (label {ol[k]}, {oi[k]}->{oj[k]}); "
        f"at label {s} u={u!r} P_acc={p!r} dH={dH!r}: |dH + T ln u| = {margin:.3g} > bound {bound:.3g}")
    say(f"first FP32/FP64 difference at hop {k}: label {s}, |dH + T ln u| = {margin:.3g} <= {bound:.3g}")
    return k
