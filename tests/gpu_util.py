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
                         seed=d["seed"], sample_id=d["sample_id"], clock_mode=clock_mode)


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
